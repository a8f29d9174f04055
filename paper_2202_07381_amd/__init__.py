"""MI355X-native stage-coupled Vanka multigrid for IRK discretisations of
incompressible flow (Abu-Labdeh, MacLachlan, Farrell, arXiv 2202.07381).

The solver lives in the HIP/C++ library ``libirkmg.so`` behind the C ABI declared in
``include/irk_mg.h``; :mod:`paper_2202_07381_amd.irkmg` is its thin ctypes binding.
:mod:`paper_2202_07381_amd.workloads` holds the seeded synthetic inputs.
"""
