"""MI355X-native Monte Carlo NEGF with elastic Buttiker dephasing (HIP library + binding).

Submodules: mcnegf (ctypes binding of include/mcnegf.h), autograd (torch.autograd entry to
the DIRECT current and its adjoint), build (hipcc build step), inputs (seeded synthetic
workloads), profiling (rocprofv3 summaries).
"""
