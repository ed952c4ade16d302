// placeholder, replaced by the traversal implementation
#include "dfgt_internal.h"
namespace dfgt {
dfgt_status run_gauss_sum(dfgt_tree_s *, dfgt_tree_s *, const double *, int, double, int, int, double *,
                          dfgt_stats *, hipStream_t) {
    set_error("dfgt_gauss_sum: not implemented yet");
    return DFGT_EINVAL;
}
}  // namespace dfgt
