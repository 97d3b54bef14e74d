"""MI355X-native lattice-Boltzmann + DEM step for sheared dense suspensions.

The compute path lives in the HIP library ``libsusp.so`` (C ABI declared in
``include/susp.h``); ``paper_1904_02929_amd.susp`` is its thin Python binding.  Importing
the package does not load the library.
"""
