"""Thin Python binding of the C ABI in include/mcnegf.h (argument marshalling only).

Every step of the method runs in the HIP library libmcnegf.so; this module only passes
device pointers of torch tensors and torch's current HIP stream.  Importing it does not
need a GPU; calling anything that launches work does.  If the library has not been built,
`lib()` raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcnegf.so")

# status codes (include/mcnegf.h)
OK, WTRUNC, WNUMERIC = 0, 1, 2
EINVAL, EWS, EHIP, ENUMERIC, ENOTIMPL = -1, -2, -3, -4, -5
FLAG_NONFINITE, FLAG_SINGULAR, FLAG_ROWSUM, FLAG_NOABSORB, FLAG_TRUNC, FLAG_NOTSPD = (
    0x01, 0x02, 0x04, 0x08, 0x10, 0x20)
FLAG_RANGE = 0x40
LEAD_NTERMS = 8
LEAD_TLL, LEAD_TRL, LEAD_TLR, LEAD_TRR, LEAD_CL, LEAD_CR, LEAD_TRGLA, LEAD_TRGRA = range(8)
TALLY_N = 5
TALLY_EXIT_L, TALLY_EXIT_R, TALLY_TRUNC, TALLY_STEPS, TALLY_STEPS2 = range(5)
EXPORTED = ("mc_negf_workspace_bytes", "mc_negf_build_kernel", "mc_negf_walk",
            "mc_negf_current", "mc_negf_grad_workspace_bytes",
            "mc_negf_grad_workspace_bytes_chunk", "mc_negf_grad",
            "mc_negf_current_async", "mc_negf_walk_sampled_bytes", "mc_negf_walk_sampled",
            "mc_negf_walk_sampled_noalloc", "mc_negf_interp_distances", "mc_negf_interp_plan",
            "mc_negf_walk_interp", "mc_negf_current_interp",
            "mc_negf_walk_counts_bytes", "mc_negf_walk_counts", "mc_negf_grad_mc",
            "mc_negf_weighted_tables_bytes", "mc_negf_weighted_tables",
            "mc_negf_walk_weighted_bytes", "mc_negf_walk_weighted", "mc_negf_current_weighted",
            "mc_negf_energy_table_bytes", "mc_negf_energy_table", "mc_negf_walk_inelastic",
            "mc_negf_spectrum",
            "mc_negf_batch_bytes", "mc_negf_batch_prepare",
            "mc_negf_walk_batch", "mc_negf_walk_batch_autotune", "mc_negf_plan_waves",
            "mc_negf_graph_begin", "mc_negf_graph_end", "mc_negf_graph_launch",
            "mc_negf_graph_destroy", "mc_negf_profile_begin", "mc_negf_profile_end",
            "mc_negf_status", "mc_negf_last_hip_error", "mc_negf_version")
PROFILE_MAX = 512


class McnegfError(RuntimeError):
    def __init__(self, call: str, code: int, hip_error: int = 0):
        super().__init__(f"{call} returned {code}" + (f" (hipError {hip_error})" if hip_error else ""))
        self.code = code


class System(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("L", ctypes.c_int32), ("t", ctypes.c_double),
                ("lead_model", ctypes.c_int32), ("gamma_l", ctypes.c_double),
                ("delta_lead", ctypes.c_double), ("flags", ctypes.c_uint32)]


class WalkConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("wg_size", ctypes.c_int32), ("groups", ctypes.c_int32),
                ("walks_per_slot", ctypes.c_int32), ("chunk", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Batch(ctypes.Structure):
    _fields_ = [("d_units", ctypes.c_void_p), ("d_scratch_tallies", ctypes.c_void_p),
                ("n_units", ctypes.c_uint32), ("n_kernels", ctypes.c_uint32)]


class KernelStruct(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("L", ctypes.c_int32), ("N", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("nE", ctypes.c_int32),
                ("lead_model", ctypes.c_int32), ("t", ctypes.c_double),
                ("delta_lead", ctypes.c_double), ("alias_pitch", ctypes.c_int64), ("p_pitch", ctypes.c_int64),
                ("energies", ctypes.c_void_p), ("gamma", ctypes.c_void_p),
                ("alias", ctypes.c_void_p), ("alias_lo", ctypes.c_void_p), ("P", ctypes.c_void_p), ("wL", ctypes.c_void_p),
                ("wR", ctypes.c_void_p), ("Adiag", ctypes.c_void_p), ("lead", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p), ("gam_lead", ctypes.c_void_p),
                ("gL", ctypes.c_void_p), ("gR", ctypes.c_void_p), ("Gd", ctypes.c_void_p),
                ("corner", ctypes.c_void_p), ("direct", ctypes.c_void_p),
                ("direct_vec", ctypes.c_void_p), ("reduce", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("counters", ctypes.c_void_p),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_uint64)]


class Profile(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dropped", ctypes.c_int32),
                ("name", ctypes.c_char_p * PROFILE_MAX), ("start", ctypes.c_void_p * PROFILE_MAX),
                ("stop", ctypes.c_void_p * PROFILE_MAX)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmcnegf.so (built by paper_1805_10164_amd.build); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1805_10164_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, u64, dp = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.POINTER(ctypes.c_double))
    L.mc_negf_workspace_bytes.argtypes = [ctypes.POINTER(System), i32, ctypes.POINTER(u64)]
    L.mc_negf_build_kernel.argtypes = [ctypes.POINTER(System), vp, vp, vp, i32, vp, u64,
                                       ctypes.POINTER(KernelStruct), vp]
    L.mc_negf_walk.argtypes = [ctypes.POINTER(KernelStruct), u64, u32, u32, u64, u64, u32, vp, vp]
    L.mc_negf_current.argtypes = [ctypes.POINTER(KernelStruct), i32, u32, vp, vp, vp, vp, dp, vp]
    L.mc_negf_grad_workspace_bytes.argtypes = [ctypes.POINTER(KernelStruct), ctypes.POINTER(u64)]
    L.mc_negf_grad_workspace_bytes_chunk.argtypes = [ctypes.POINTER(KernelStruct), i32,
                                                     ctypes.POINTER(u64)]
    L.mc_negf_grad.argtypes = [ctypes.POINTER(KernelStruct), u32, vp, vp, u64, vp, vp, dp, vp]
    L.mc_negf_status.argtypes = [ctypes.POINTER(KernelStruct), ctypes.POINTER(u32), vp]
    L.mc_negf_current_async.argtypes = [ctypes.POINTER(KernelStruct), i32, u32, vp, vp, vp, vp,
                                        vp, vp]
    L.mc_negf_walk_sampled_bytes.argtypes = [ctypes.POINTER(KernelStruct), u64,
                                             ctypes.POINTER(u64)]
    L.mc_negf_walk_sampled.argtypes = [ctypes.POINTER(KernelStruct), u64, u32, u32, u64, u64,
                                       u32, vp, vp, vp, u64, vp]
    L.mc_negf_walk_sampled_noalloc.argtypes = [ctypes.POINTER(KernelStruct), u64, u32, u32,
                                               u64, u64, u32, vp, vp, vp]
    L.mc_negf_interp_distances.argtypes = [ctypes.POINTER(KernelStruct), vp, vp]
    L.mc_negf_interp_plan.argtypes = [dp, i32, dp, dp, i32, ctypes.c_double,
                                      ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mc_negf_walk_interp.argtypes = [ctypes.POINTER(KernelStruct), vp, i32, u64, u32, u32, u64,
                                      u64, u32, vp, vp]
    L.mc_negf_current_interp.argtypes = [ctypes.POINTER(KernelStruct), vp, i32, u32, vp, vp, vp,
                                         vp, dp, vp]
    L.mc_negf_walk_counts_bytes.argtypes = [ctypes.POINTER(KernelStruct), ctypes.POINTER(u64)]
    L.mc_negf_walk_counts.argtypes = [ctypes.POINTER(KernelStruct), u64, u32, u32, u64, u64,
                                      u32, vp, vp, vp]
    L.mc_negf_grad_mc.argtypes = [ctypes.POINTER(KernelStruct), u32, vp, vp, vp, vp, u64, vp,
                                  vp, vp]
    L.mc_negf_weighted_tables_bytes.argtypes = [ctypes.POINTER(KernelStruct),
                                                ctypes.POINTER(u64)]
    L.mc_negf_weighted_tables.argtypes = [ctypes.POINTER(KernelStruct), vp, vp, u64, vp]
    L.mc_negf_walk_weighted_bytes.argtypes = [ctypes.POINTER(KernelStruct), u64,
                                              ctypes.POINTER(u64)]
    L.mc_negf_walk_weighted.argtypes = [ctypes.POINTER(KernelStruct), vp, u64, vp, u64, u32, u32,
                                        u64, u64, u32, vp, vp, vp, u64, vp]
    L.mc_negf_current_weighted.argtypes = [ctypes.POINTER(KernelStruct), u32, vp, vp, vp, vp, vp,
                                           dp, vp]
    L.mc_negf_energy_table_bytes.argtypes = [ctypes.POINTER(KernelStruct), i32,
                                             ctypes.POINTER(u64)]
    L.mc_negf_energy_table.argtypes = [ctypes.POINTER(KernelStruct), i32, vp, vp, vp, u64, vp]
    L.mc_negf_walk_inelastic.argtypes = [ctypes.POINTER(KernelStruct), i32, vp, vp, u64, u64, u32,
                                         u32, u64, u64, u32, vp, vp, vp]
    L.mc_negf_spectrum.argtypes = [ctypes.POINTER(KernelStruct), u32, vp, vp, vp, vp, vp]
    L.mc_negf_batch_bytes.argtypes = [ctypes.POINTER(KernelStruct), i32, ctypes.POINTER(u64)]
    L.mc_negf_batch_prepare.argtypes = [ctypes.POINTER(KernelStruct), i32,
                                        ctypes.POINTER(u32), u32, ctypes.POINTER(vp), vp, u64,
                                        ctypes.POINTER(Batch), vp]
    L.mc_negf_walk_batch.argtypes = [ctypes.POINTER(Batch), u64, u64, u64, u32,
                                     ctypes.POINTER(WalkConfig), vp]
    L.mc_negf_walk_batch_autotune.argtypes = [ctypes.POINTER(Batch), u64, u64, u32,
                                              ctypes.POINTER(WalkConfig),
                                              ctypes.POINTER(ctypes.c_float), vp]
    L.mc_negf_plan_waves.argtypes = [ctypes.POINTER(System), i32, i32, u64,
                                     ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.mc_negf_graph_begin.argtypes = [vp]
    L.mc_negf_graph_end.argtypes = [vp, ctypes.POINTER(vp)]
    L.mc_negf_graph_launch.argtypes = [vp, vp]
    L.mc_negf_graph_destroy.argtypes = [vp]
    L.mc_negf_profile_begin.argtypes = [ctypes.POINTER(Profile)]
    L.mc_negf_profile_end.argtypes = [ctypes.POINTER(Profile), ctypes.POINTER(ctypes.c_float)]
    L.mc_negf_last_hip_error.argtypes = []
    L.mc_negf_version.argtypes = []
    for name in EXPORTED:
        getattr(L, name).restype = i32
    _lib = L
    return L


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check(call: str, code: int, allow=(OK,)):
    if code not in allow:
        raise McnegfError(call, code, lib().mc_negf_last_hip_error())
    return code


def _ptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    return ctypes.c_void_p(t.data_ptr())


BUILD_NO_ALIAS = 0x1
BUILD_NO_DIRECT = 0x2
BUILD_FP32_PRODUCTS = 0x4
BUILD_FP32_REFINE = 0x8
BUILD_FP32_SWEEPS = 0x10


def make_system(W: int, L: int, t: float = 1.0, lead_model: int = 0, gamma_l: float = 0.0,
                delta_lead: float = 1e-10, flags: int = 0) -> System:
    """flags: BUILD_NO_ALIAS builds no alias tables (DIRECT current and gradient only),
    BUILD_NO_DIRECT reserves nothing for the DIRECT solve (Monte Carlo only),
    BUILD_FP32_PRODUCTS runs the full inverse's block products in FP32 (W = 16, 32), with
    BUILD_FP32_REFINE one FP64 refinement step on G and with BUILD_FP32_SWEEPS the RGF sweeps
    in FP32 too."""
    return System(W, L, t, lead_model, gamma_l, delta_lead, flags)


class Kernel:
    """A built kernel handle plus the torch tensors it borrows (workspace, gamma, energies)."""

    def __init__(self, struct: KernelStruct, ws, gamma, energies):
        self.struct = struct
        self.ws = ws
        self.gamma = gamma
        self.energies = energies

    def __getattr__(self, name):
        return getattr(self.__dict__["struct"], name)

    def view(self, field: str, dtype, shape):
        """torch view of a workspace region named by a pointer field of the handle."""
        import torch
        ptr = getattr(self.struct, field)
        if not ptr:
            raise ValueError(f"this kernel has no {field} (built with BUILD_NO_ALIAS?)")
        off = ptr - self.ws.data_ptr()
        nbytes = int(np.prod(shape)) * torch.empty((), dtype=dtype).element_size()
        return self.ws[off:off + nbytes].view(dtype).view(*shape)

    # named views
    def P(self):
        import torch
        return self.view("P", torch.float64, (self.nE, self.N, self.p_pitch))[:, :, :self.N]

    def wL(self):
        import torch
        return self.view("wL", torch.float64, (self.nE, self.N))

    def wR(self):
        import torch
        return self.view("wR", torch.float64, (self.nE, self.N))

    def Adiag(self):
        import torch
        return self.view("Adiag", torch.float64, (self.nE, self.N))

    def lead(self):
        import torch
        return self.view("lead", torch.float64, (self.nE, LEAD_NTERMS))

    def sigma(self):
        import torch
        return self.view("sigma", torch.float64, (self.nE, self.W, self.W, 2))

    def Gd(self):
        import torch
        return self.view("Gd", torch.float64, (self.nE, self.L, self.W, self.W, 2))

    def alias_packed(self):
        """[nE][n_out][alias_pitch] packed entries (thr >> 16) << 16 | alias, int32 storage."""
        import torch
        return self.view("alias", torch.int32, (self.nE, self.n_out, self.alias_pitch))

    def alias_low(self):
        """[nE][n_out][alias_pitch] low 16 bits of the thresholds, int16 storage."""
        import torch
        return self.view("alias_lo", torch.int16, (self.nE, self.n_out, self.alias_pitch))

    def alias_tables(self):
        """(thr uint32, alias int32) numpy arrays [nE][n_out][alias_pitch] read back from the
        device format (format conversion only)."""
        packed = self.alias_packed().cpu().numpy().view(np.uint32)
        low = self.alias_low().cpu().numpy().view(np.uint16).astype(np.uint32)
        return (packed & np.uint32(0xFFFF0000)) | low, (packed & np.uint32(0xFFFF)).astype(np.int32)

    def alias_rows(self, e, rows):
        """(thr uint32, alias int32) [len(rows)][n_out] of energy e's alias rows `rows`, read
        back from the device format (format conversion only; copies only those rows)."""
        import torch
        idx = torch.as_tensor(list(rows), dtype=torch.int64, device=self.ws.device)
        n = self.n_out
        packed = self.alias_packed()[e].index_select(0, idx)[:, :n].cpu().numpy().view(np.uint32)
        low = (self.alias_low()[e].index_select(0, idx)[:, :n].cpu().numpy().view(np.uint16)
               .astype(np.uint32))
        return (packed & np.uint32(0xFFFF0000)) | low, (packed & np.uint32(0xFFFF)).astype(np.int32)

    def set_alias_tables(self, thr, alias):
        """Store uint32 thresholds and alias indices [nE][n_out][alias_pitch] in the device
        format (format conversion only)."""
        import torch
        thr = np.asarray(thr, dtype=np.uint32)
        alias = np.asarray(alias, dtype=np.uint32)
        packed = (thr & np.uint32(0xFFFF0000)) | (alias & np.uint32(0xFFFF))
        low = (thr & np.uint32(0xFFFF)).astype(np.uint16)
        dev = self.ws.device
        self.alias_packed().copy_(torch.from_numpy(packed.view(np.int32)).to(dev))
        self.alias_low().copy_(torch.from_numpy(low.view(np.int16)).to(dev))


def mc_negf_workspace_bytes(system: System, nE: int) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_workspace_bytes",
           lib().mc_negf_workspace_bytes(ctypes.byref(system), int(nE), ctypes.byref(out)))
    return int(out.value)


def mc_negf_build_kernel(system: System, onsite, gamma, energies, ws, stream=None) -> Kernel:
    """Build G, kernel rows and alias tables for every energy (asynchronous on the stream)."""
    for name, t in (("onsite", onsite), ("gamma", gamma), ("energies", energies)):
        if not (t.is_cuda and t.dtype.is_floating_point and t.element_size() == 8 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    ks = KernelStruct()
    code = lib().mc_negf_build_kernel(ctypes.byref(system), _ptr(onsite), _ptr(gamma),
                                      _ptr(energies), int(energies.numel()), _ptr(ws),
                                      ws.numel() * ws.element_size(), ctypes.byref(ks),
                                      _stream(stream))
    _check("mc_negf_build_kernel", code)
    return Kernel(ks, ws, gamma, energies)


def mc_negf_walk(k: Kernel, seed: int, realization: int, inject_lead: int, walker_begin: int,
                 n_walkers: int, max_steps: int, tallies, stream=None) -> int:
    code = lib().mc_negf_walk(ctypes.byref(k.struct), int(seed), int(realization),
                              int(inject_lead), int(walker_begin), int(n_walkers),
                              int(max_steps), _ptr(tallies), _stream(stream))
    return _check("mc_negf_walk", code)


def mc_negf_current(k: Kernel, mode: int, inject_lead: int, tallies, weights, T, sigmaT,
                    stream=None, allow=(OK, WTRUNC, WNUMERIC)):
    """Returns (status, I, sigma_I); synchronises the stream."""
    out = (ctypes.c_double * 2)()
    code = lib().mc_negf_current(ctypes.byref(k.struct), int(mode), int(inject_lead),
                                 _ptr(tallies), _ptr(weights), _ptr(T), _ptr(sigmaT),
                                 ctypes.cast(out, ctypes.POINTER(ctypes.c_double)),
                                 _stream(stream))
    _check("mc_negf_current", code, allow)
    return code, float(out[0]), float(out[1])


def mc_negf_grad_workspace_bytes(k: Kernel) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_grad_workspace_bytes",
           lib().mc_negf_grad_workspace_bytes(ctypes.byref(k.struct), ctypes.byref(out)))
    return int(out.value)


def mc_negf_grad_workspace_bytes_chunk(k: Kernel, chunk: int) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_grad_workspace_bytes_chunk",
           lib().mc_negf_grad_workspace_bytes_chunk(ctypes.byref(k.struct), int(chunk),
                                                    ctypes.byref(out)))
    return int(out.value)


def mc_negf_grad(k: Kernel, inject_lead, weights, gws, dI_dV, dI_dgamma, stream=None,
                 allow=(OK, WNUMERIC)):
    """dI/dV_i and dI/dgamma_i of the DIRECT current into the [N] device tensors dI_dV and
    dI_dgamma; gws is a device byte tensor of >= mc_negf_grad_workspace_bytes(k).  Returns
    (status, I)."""
    out = ctypes.c_double(0.0)
    code = int(lib().mc_negf_grad(ctypes.byref(k.struct), int(inject_lead), _ptr(weights),
                                  _ptr(gws), int(gws.numel()), _ptr(dI_dV), _ptr(dI_dgamma),
                                  ctypes.byref(out), _stream(stream)))
    _check("mc_negf_grad", code, allow)
    return code, float(out.value)


def mc_negf_status(k: Kernel, stream=None) -> int:
    flags = ctypes.c_uint32(0)
    _check("mc_negf_status", lib().mc_negf_status(ctypes.byref(k.struct), ctypes.byref(flags),
                                                  _stream(stream)))
    return int(flags.value)


class LaunchTimes:
    """Context manager: times every launch of this library from the calling thread with HIP
    events on the launch stream; after exit, `.records` is a list of (kernel name, ms)."""

    def __init__(self):
        self.p = Profile()
        self.records = []

    def __enter__(self):
        _check("mc_negf_profile_begin", lib().mc_negf_profile_begin(ctypes.byref(self.p)))
        return self

    def __exit__(self, *exc):
        ms = (ctypes.c_float * PROFILE_MAX)()
        code = lib().mc_negf_profile_end(ctypes.byref(self.p), ms)
        self.records = [(self.p.name[i].decode(), float(ms[i])) for i in range(self.p.n)]
        self.dropped = int(self.p.dropped)
        if exc[0] is None:
            _check("mc_negf_profile_end", code)
        return False

    def total_ms(self, name):
        return sum(ms for n, ms in self.records if n == name)

    def count(self, name):
        return sum(1 for n, _ in self.records if n == name)


def allocate_workspace(system: System, nE: int, device="cuda"):
    import torch
    nbytes = mc_negf_workspace_bytes(system, nE)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ---- async current, batched walks, wave planning, graphs ------------------------------------

def mc_negf_current_async(k: Kernel, mode: int, inject_lead: int, tallies, weights, T, sigmaT,
                          I_sigma, stream=None) -> int:
    """As mc_negf_current, but writes (I, sigma_I) into the [2] device tensor I_sigma and
    does not synchronise (capturable)."""
    code = lib().mc_negf_current_async(ctypes.byref(k.struct), int(mode), int(inject_lead),
                                       _ptr(tallies), _ptr(weights), _ptr(T), _ptr(sigmaT),
                                       _ptr(I_sigma), _stream(stream))
    return _check("mc_negf_current_async", code)


class WalkBatch:
    """A batched walk over built kernels: the C batch handle plus the buffers it borrows."""

    def __init__(self, struct: Batch, buf, kernels, tallies):
        self.struct = struct
        self.buf = buf
        self.kernels = kernels
        self.tallies = tallies


def _kernel_array(kernels):
    arr = (KernelStruct * len(kernels))()
    for i, k in enumerate(kernels):
        arr[i] = k.struct
    return arr


def mc_negf_batch_prepare(kernels, realizations, inject_lead, tallies, device="cuda",
                          stream=None) -> WalkBatch:
    """Unit table for walking every energy of every kernel in one launch; tallies[i] is
    kernel i's [nE][5] int64 device tensor (accumulated).  Synchronises the stream."""
    import torch
    arr = _kernel_array(kernels)
    nbytes = ctypes.c_uint64(0)
    _check("mc_negf_batch_bytes", lib().mc_negf_batch_bytes(arr, len(kernels), ctypes.byref(nbytes)))
    buf = torch.empty(int(nbytes.value), dtype=torch.uint8, device=device)
    reals = (ctypes.c_uint32 * len(kernels))(*[int(r) for r in realizations])
    tp = (ctypes.c_void_p * len(kernels))(*[t.data_ptr() for t in tallies])
    b = Batch()
    _check("mc_negf_batch_prepare",
           lib().mc_negf_batch_prepare(arr, len(kernels), reals, int(inject_lead), tp, _ptr(buf),
                                       int(nbytes.value), ctypes.byref(b), _stream(stream)))
    return WalkBatch(b, buf, list(kernels), list(tallies))


def walk_config(slots=3, wg_size=256, groups=8, walks_per_slot=8, chunk=0) -> WalkConfig:
    return WalkConfig(slots, wg_size, groups, walks_per_slot, chunk)


def mc_negf_walk_batch(b: WalkBatch, seed: int, walker_begin: int, n_walkers: int,
                       max_steps: int, cfg: WalkConfig = None, stream=None) -> int:
    code = lib().mc_negf_walk_batch(ctypes.byref(b.struct), int(seed), int(walker_begin),
                                    int(n_walkers), int(max_steps),
                                    ctypes.byref(cfg) if cfg is not None else None,
                                    _stream(stream))
    return _check("mc_negf_walk_batch", code)


def mc_negf_walk_batch_autotune(b: WalkBatch, seed: int, n_walkers: int, max_steps: int,
                                stream=None):
    """(fastest WalkConfig, its time in ms) over the library's candidate launch shapes."""
    best = WalkConfig()
    ms = ctypes.c_float(0.0)
    _check("mc_negf_walk_batch_autotune",
           lib().mc_negf_walk_batch_autotune(ctypes.byref(b.struct), int(seed), int(n_walkers),
                                             int(max_steps), ctypes.byref(best),
                                             ctypes.byref(ms), _stream(stream)))
    return best, float(ms.value)


def mc_negf_plan_waves(systems, nE: int, budget_bytes: int):
    """(order, wave_of, n_waves): first-fit-decreasing assignment of systems to waves whose
    build workspaces fit budget_bytes (host only)."""
    n = len(systems)
    arr = (System * n)(*systems)
    order = (ctypes.c_int32 * n)()
    wave_of = (ctypes.c_int32 * n)()
    nw = ctypes.c_int32(0)
    _check("mc_negf_plan_waves", lib().mc_negf_plan_waves(arr, n, int(nE), int(budget_bytes),
                                                          order, wave_of, ctypes.byref(nw)))
    return list(order), list(wave_of), int(nw.value)


class Graph:
    """A captured and instantiated HIP graph of library calls (and other stream work)."""

    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream=None):
        _check("mc_negf_graph_launch", lib().mc_negf_graph_launch(self.handle, _stream(stream)))

    def destroy(self):
        if self.handle:
            _check("mc_negf_graph_destroy", lib().mc_negf_graph_destroy(self.handle))
            self.handle = None


def mc_negf_graph_begin(stream=None):
    _check("mc_negf_graph_begin", lib().mc_negf_graph_begin(_stream(stream)))


def mc_negf_graph_end(stream=None) -> Graph:
    h = ctypes.c_void_p(0)
    _check("mc_negf_graph_end", lib().mc_negf_graph_end(_stream(stream), ctypes.byref(h)))
    return Graph(h)


def mc_negf_walk_sampled_bytes(k: Kernel, n_walkers: int) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_walk_sampled_bytes",
           lib().mc_negf_walk_sampled_bytes(ctypes.byref(k.struct), int(n_walkers),
                                            ctypes.byref(out)))
    return int(out.value)


def mc_negf_walk_sampled(k: Kernel, seed: int, realization: int, inject_lead: int,
                         walker_begin: int, n_walkers: int, max_steps: int, weights, tallies,
                         scratch, stream=None) -> int:
    """Walkers draw their energies with probability weights[k] / sum (device draws and
    sort), then walk; counts go to tallies[k].  Estimate with mc_negf_current mode 2."""
    code = lib().mc_negf_walk_sampled(ctypes.byref(k.struct), int(seed), int(realization),
                                      int(inject_lead), int(walker_begin), int(n_walkers),
                                      int(max_steps), _ptr(weights), _ptr(tallies), _ptr(scratch),
                                      int(scratch.numel()), _stream(stream))
    return _check("mc_negf_walk_sampled", code)


STATIC_SCRATCH_BYTES = 64 << 20


def mc_negf_walk_sampled_noalloc(k: Kernel, seed: int, realization: int, inject_lead: int,
                                 walker_begin: int, n_walkers: int, max_steps: int, weights,
                                 tallies, stream=None) -> int:
    """As mc_negf_walk_sampled, with the library's fixed per-device scratch instead of a
    caller buffer (no device allocation)."""
    code = lib().mc_negf_walk_sampled_noalloc(ctypes.byref(k.struct), int(seed),
                                              int(realization), int(inject_lead),
                                              int(walker_begin), int(n_walkers),
                                              int(max_steps), _ptr(weights), _ptr(tallies),
                                              _stream(stream))
    return _check("mc_negf_walk_sampled_noalloc", code)


# ---- score-function gradient of the Monte Carlo current ----------------------------------------

def mc_negf_walk_counts_bytes(k: Kernel) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_walk_counts_bytes",
           lib().mc_negf_walk_counts_bytes(ctypes.byref(k.struct), ctypes.byref(out)))
    return int(out.value)


def mc_negf_walk_counts(k: Kernel, seed: int, realization: int, inject_lead: int,
                        walker_begin: int, n_walkers: int, max_steps: int, counts, tallies,
                        stream=None) -> int:
    """Walks as mc_negf_walk; the steps of the walks that exit at q are added to counts
    [nE][n_out][n_out] (int32 storage of uint32 counts, outcome-major)."""
    return _check("mc_negf_walk_counts",
                  lib().mc_negf_walk_counts(ctypes.byref(k.struct), int(seed), int(realization),
                                            int(inject_lead), int(walker_begin), int(n_walkers),
                                            int(max_steps), _ptr(counts), _ptr(tallies),
                                            _stream(stream)))


def mc_negf_grad_mc(k: Kernel, inject_lead: int, counts, tallies, weights, gws, dI_dV,
                    dI_dgamma, stream=None) -> int:
    """Score-function estimate of dI/dV_i and dI/dgamma_i from transition counts (workspace of
    mc_negf_grad)."""
    return _check("mc_negf_grad_mc",
                  lib().mc_negf_grad_mc(ctypes.byref(k.struct), int(inject_lead), _ptr(counts),
                                        _ptr(tallies), _ptr(weights), _ptr(gws),
                                        int(gws.numel()), _ptr(dI_dV), _ptr(dI_dgamma),
                                        _stream(stream)))


# ---- inelastic walks (step 7') -----------------------------------------------------------------

def _lines(offsets, lambdas=None):
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    lam = None if lambdas is None else np.ascontiguousarray(lambdas, dtype=np.float64)
    if lam is not None and lam.shape != off.shape:
        raise ValueError("offsets and lambdas must have the same length")
    return off, lam


def mc_negf_energy_table_bytes(k: Kernel, n_lines: int) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_energy_table_bytes",
           lib().mc_negf_energy_table_bytes(ctypes.byref(k.struct), int(n_lines),
                                            ctypes.byref(out)))
    return int(out.value)


def mc_negf_energy_table(k: Kernel, offsets, lambdas, table, stream=None) -> int:
    """Step-7' thresholds [nE][N][n_lines] (int64 storage of uint64) from the handle's A_jj for
    energy lines at `offsets` grid steps with weights `lambdas` (host sequences)."""
    off, lam = _lines(offsets, lambdas)
    return _check("mc_negf_energy_table",
                  lib().mc_negf_energy_table(ctypes.byref(k.struct), int(off.size),
                                             off.ctypes.data_as(ctypes.c_void_p),
                                             lam.ctypes.data_as(ctypes.c_void_p), _ptr(table),
                                             int(table.numel() * table.element_size()),
                                             _stream(stream)))


def mc_negf_walk_inelastic(k: Kernel, offsets, table, seed: int, realization: int,
                           inject_lead: int, walker_begin: int, n_walkers: int, max_steps: int,
                           tallies, hist, stream=None) -> int:
    """Inelastic walks on the handle's alias tables with step 7' drawn from `table`; adds to
    tallies [nE][TALLY_N] and hist [2][nE][nE] (int64)."""
    off, _ = _lines(offsets)
    return _check("mc_negf_walk_inelastic",
                  lib().mc_negf_walk_inelastic(ctypes.byref(k.struct), int(off.size),
                                               off.ctypes.data_as(ctypes.c_void_p), _ptr(table),
                                               int(table.numel() * table.element_size()),
                                               int(seed), int(realization), int(inject_lead),
                                               int(walker_begin), int(n_walkers), int(max_steps),
                                               _ptr(tallies), _ptr(hist), _stream(stream)))


def mc_negf_spectrum(k: Kernel, inject_lead: int, tallies, hist, weights, spectrum,
                     stream=None) -> int:
    """Energy-resolved current [2][nE] of inelastic walks."""
    return _check("mc_negf_spectrum",
                  lib().mc_negf_spectrum(ctypes.byref(k.struct), int(inject_lead), _ptr(tallies),
                                         _ptr(hist), _ptr(weights), _ptr(spectrum),
                                         _stream(stream)))


# ---- importance-sampled walks ---------------------------------------------------------------

def mc_negf_weighted_tables_bytes(k: Kernel) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_weighted_tables_bytes",
           lib().mc_negf_weighted_tables_bytes(ctypes.byref(k.struct), ctypes.byref(out)))
    return int(out.value)


def mc_negf_weighted_tables(k: Kernel, bias, tables, stream=None) -> int:
    """Alias tables of the modified rows K_ij b_j (bias [nE][n_out] device) and rho into the
    byte tensor `tables` (mc_negf_weighted_tables_bytes long)."""
    return _check("mc_negf_weighted_tables",
                  lib().mc_negf_weighted_tables(ctypes.byref(k.struct), _ptr(bias), _ptr(tables),
                                                int(tables.numel()), _stream(stream)))


def weighted_tables_views(k: Kernel, tables):
    """(packed [nE][n_out][pitch] int32, low bits uint16, rho [nE][n_out] float64) views of
    a modified-tables buffer, in the layout the library writes."""
    import torch
    ent = k.nE * k.n_out * k.alias_pitch
    a256 = lambda x: (x + 255) & ~255
    off_lo = a256(ent * 4)
    off_rho = off_lo + a256(ent * 2)
    shape = (k.nE, k.n_out, k.alias_pitch)
    packed = tables[:ent * 4].view(torch.int32).view(shape)
    low = tables[off_lo:off_lo + ent * 2].view(torch.int16).view(shape)
    rho = tables[off_rho:off_rho + k.nE * k.n_out * 8].view(torch.float64).view(k.nE, k.n_out)
    return packed, low, rho


def mc_negf_walk_weighted_bytes(k: Kernel, n_walkers: int) -> int:
    out = ctypes.c_uint64(0)
    _check("mc_negf_walk_weighted_bytes",
           lib().mc_negf_walk_weighted_bytes(ctypes.byref(k.struct), int(n_walkers),
                                             ctypes.byref(out)))
    return int(out.value)


def mc_negf_walk_weighted(k: Kernel, tables, bias, seed: int, realization: int,
                          inject_lead: int, walker_begin: int, n_walkers: int, max_steps: int,
                          tallies, wsum, scratch, stream=None) -> int:
    """Importance-sampled walks on the modified tables; counts to tallies, score sums to
    wsum [nE][2]."""
    code = lib().mc_negf_walk_weighted(ctypes.byref(k.struct), _ptr(tables),
                                       int(tables.numel()), _ptr(bias), int(seed),
                                       int(realization), int(inject_lead), int(walker_begin),
                                       int(n_walkers), int(max_steps), _ptr(tallies), _ptr(wsum),
                                       _ptr(scratch), int(scratch.numel()), _stream(stream))
    return _check("mc_negf_walk_weighted", code)


def mc_negf_current_weighted(k: Kernel, inject_lead: int, tallies, wsum, weights, T, sigmaT,
                             stream=None, allow=(OK, WTRUNC, WNUMERIC)):
    """(status, I, sigma_I) of importance-sampled walks; synchronises the stream."""
    out = (ctypes.c_double * 2)()
    code = lib().mc_negf_current_weighted(ctypes.byref(k.struct), int(inject_lead),
                                          _ptr(tallies), _ptr(wsum), _ptr(weights), _ptr(T),
                                          _ptr(sigmaT),
                                          ctypes.cast(out, ctypes.POINTER(ctypes.c_double)),
                                          _stream(stream))
    _check("mc_negf_current_weighted", code, allow)
    return code, float(out[0]), float(out[1])


# ---- interpolated step-6' probabilities -------------------------------------------------------

def mc_negf_interp_distances(k: Kernel, dist, stream=None) -> int:
    """dist [nE - 1] device: largest row L1 distance between neighbouring built energies."""
    return _check("mc_negf_interp_distances",
                  lib().mc_negf_interp_distances(ctypes.byref(k.struct), _ptr(dist),
                                                 _stream(stream)))


def mc_negf_interp_plan(nodes, dist, fine, tol):
    """Indices of the fine energies that must be built exactly (host only)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    dist = np.ascontiguousarray(dist, dtype=np.float64)
    fine = np.ascontiguousarray(fine, dtype=np.float64)
    out = np.zeros(len(fine), dtype=np.int32)
    m = ctypes.c_int32(0)
    dp = ctypes.POINTER(ctypes.c_double)
    _check("mc_negf_interp_plan",
           lib().mc_negf_interp_plan(nodes.ctypes.data_as(dp), len(nodes),
                                     dist.ctypes.data_as(dp), fine.ctypes.data_as(dp),
                                     len(fine), float(tol),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                     ctypes.byref(m)))
    return [int(x) for x in out[:m.value]]


def mc_negf_walk_interp(k: Kernel, fine, seed: int, realization: int, inject_lead: int,
                        walker_begin: int, n_walkers: int, max_steps: int, tallies,
                        stream=None) -> int:
    code = lib().mc_negf_walk_interp(ctypes.byref(k.struct), _ptr(fine), int(fine.numel()),
                                     int(seed), int(realization), int(inject_lead),
                                     int(walker_begin), int(n_walkers), int(max_steps),
                                     _ptr(tallies), _stream(stream))
    return _check("mc_negf_walk_interp", code)


def mc_negf_current_interp(k: Kernel, fine, inject_lead: int, tallies, weights, T, sigmaT,
                           stream=None, allow=(OK, WTRUNC, WNUMERIC)):
    """(status, I, sigma_I) of interpolated walks; synchronises the stream."""
    out = (ctypes.c_double * 2)()
    code = lib().mc_negf_current_interp(ctypes.byref(k.struct), _ptr(fine), int(fine.numel()),
                                        int(inject_lead), _ptr(tallies), _ptr(weights), _ptr(T),
                                        _ptr(sigmaT),
                                        ctypes.cast(out, ctypes.POINTER(ctypes.c_double)),
                                        _stream(stream))
    _check("mc_negf_current_interp", code, allow)
    return code, float(out[0]), float(out[1])
