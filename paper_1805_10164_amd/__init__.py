"""MI355X-native Monte Carlo NEGF with elastic Buttiker dephasing (HIP library + binding).

Submodules: mcnegf (ctypes binding of include/mcnegf.h), build (hipcc build step),
inputs (seeded synthetic workloads).
"""
