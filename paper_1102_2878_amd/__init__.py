"""MI355X-native Dual-Tree Fast Gauss Transform.

The compute path is the HIP library ``libdfgt.so`` behind the C-ABI declared in
``include/dfgt.h``; :mod:`paper_1102_2878_amd.dfgt` is its thin Python binding.
Importing this package loads nothing: the binding is loaded on first use.
"""
