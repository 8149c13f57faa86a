"""Python binding of libc3pt: spin-open three-point contractions on MI355X.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libc3pt.so``.  PyTorch supplies device memory and the current
stream.  If the library is missing the import fails: there is no fallback.

Entry points (same names as the C ABI in include/c3pt.h, without the prefix
they are also exported as ``spectator_meson`` etc.):

* ``c3pt_spectator_meson(G_tf, eta, k, geom)``      Eq. (9) spectator part
* ``c3pt_spectator_baryon(G1_tf, G2_tf, eta, k, geom)``  epsilon-tensor spectator
* ``c3pt_insertion(G_t, s_t, taus, k, geom, U_t=None, n_ops=1)``  Eq. (10);
  n_ops 5: + D_nu, 9: + symmetrized <->D_nu, 21: + D_nu D_rho
* ``c3pt_combine(spec, ins, ...)``                 noise-weighted product
* ``c3pt_two_sink_meson(...)``                     forward + backward diagrams, time-partitioned noise
* ``c3pt_gamma_meson(C, ...)`` / ``c3pt_gamma_nucleon(C, channel, ...)``  Gamma channels
* ``smear_propagator(G, U, geom, kappa, n)`` / ``smear_vectors(v, ...)``  (c3pt_smear) quark smearing
* ``Batch`` and ``Server``: many sources in one recorded graph; continuous batching
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libc3pt.so")

C3PT_OK = 0
C3PT_EINVAL = -1
C3PT_ENOMEM = -2
C3PT_EDEVICE = -3
C3PT_EUNSUPPORTED = -4
C3PT_C64 = 0
C3PT_C128 = 1
PROJ_NATIVE = 0
PROJ_SPLIT_F16 = 1
PROJ_SPLIT_BF16 = 2
PROJ_FACTORED = 3
PROJ_FACTORED_F16 = 4
PROJ_FACTORED_BF16 = 5
PROTON_D = 0   # current on the d quark; nucleon data of spectators (u, u)
PROTON_U = 1   # current on a u quark; nucleon data of spectators (u, d)

EXPORTED = ("c3pt_spectator_meson", "c3pt_spectator_baryon", "c3pt_insertion", "c3pt_combine",
            "c3pt_two_sink_meson", "c3pt_gamma_meson", "c3pt_gamma_nucleon", "c3pt_smear", "c3pt_strerror", "c3pt_last_error", "c3pt_version", "c3pt_scratch_bytes",
            "c3pt_release_scratch", "c3pt_profile_enable", "c3pt_profile_read", "c3pt_variant_count",
            "c3pt_set_variant", "c3pt_get_variant", "c3pt_batch_create", "c3pt_batch_run", "c3pt_batch_info",
            "c3pt_batch_destroy", "c3pt_server_create", "c3pt_server_submit", "c3pt_server_step",
            "c3pt_server_poll", "c3pt_server_result", "c3pt_server_release", "c3pt_server_info",
            "c3pt_server_destroy", "c3pt_insertion_noalloc", "c3pt_noalloc_scratch_bytes",
            "c3pt_debug_scale_allocations", "c3pt_server_set_step_work")

KIND = {"spectator_meson": 0, "spectator_baryon": 1, "insertion": 2}
MODE = {"f64": 0, "f32": 1, "bf16x2": 2, "f16x2": 3, "fac": 4, "fs16": 5, "fsbf16": 5, "batchfac": 6}
# "fac", "fs16" / "fsbf16", "batchfac": variant slots of the factored projection, the
# split-precision fused projection and the factored kernels of batches and serving


class C3ptError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"c3pt status {status}: {msg}")
        self.status = status


class _KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("count", ctypes.c_longlong), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class _Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 3), ("T", ctypes.c_int), ("r", ctypes.c_int * 3),
                ("dtype", ctypes.c_int), ("proj", ctypes.c_int), ("stream", ctypes.c_void_p)]


class _Job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("L", ctypes.c_int * 3), ("T", ctypes.c_int), ("r", ctypes.c_int * 3),
                ("n_noise", ctypes.c_int), ("G", ctypes.c_void_p), ("G2", ctypes.c_void_p),
                ("eta", ctypes.c_void_p), ("G_t", ctypes.POINTER(ctypes.c_void_p)),
                ("s_t", ctypes.POINTER(ctypes.c_void_p)), ("U_t", ctypes.POINTER(ctypes.c_void_p)),
                ("taus", ctypes.POINTER(ctypes.c_int)), ("n_tau", ctypes.c_int), ("n_ops", ctypes.c_int),
                ("out", ctypes.c_void_p)]


class _CombineJob(ctypes.Structure):
    _fields_ = [("spec_job", ctypes.c_int), ("ins_job", ctypes.c_int), ("op_begin", ctypes.c_int),
                ("op_end", ctypes.c_int), ("w", ctypes.POINTER(ctypes.c_double)),
                ("pairs", ctypes.POINTER(ctypes.c_int)), ("n_pairs", ctypes.c_int), ("out", ctypes.c_void_p)]


class _Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("L", ctypes.c_int * 3), ("T", ctypes.c_int), ("r", ctypes.c_int * 3),
                ("t_src", ctypes.c_int), ("t_f", ctypes.c_int), ("n_noise", ctypes.c_int), ("n_ops", ctypes.c_int),
                ("G_t", ctypes.POINTER(ctypes.c_void_p)), ("G2_t", ctypes.POINTER(ctypes.c_void_p)),
                ("s_t", ctypes.POINTER(ctypes.c_void_p)), ("U_t", ctypes.POINTER(ctypes.c_void_p)),
                ("eta", ctypes.c_void_p), ("k", ctypes.POINTER(ctypes.c_int)), ("n_mom", ctypes.c_int),
                ("pairs", ctypes.POINTER(ctypes.c_int)), ("n_pairs", ctypes.c_int)]


class _Result(ctypes.Structure):
    _fields_ = [("spec", ctypes.c_void_p * 2), ("ins", ctypes.c_void_p * 2), ("comb", ctypes.c_void_p * 2),
                ("n_parts", ctypes.c_int), ("n_tau", ctypes.c_int), ("n_pairs", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1711_02384_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, i = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.c_int
    gp = ctypes.POINTER(_Geom)
    lib.c3pt_spectator_meson.argtypes = [gp, vp, vp, i, ip, i, vp]
    lib.c3pt_spectator_baryon.argtypes = [gp, vp, vp, vp, i, ip, i, vp]
    lib.c3pt_insertion.argtypes = [gp, ctypes.POINTER(vp), ctypes.POINTER(vp), i, ip, i,
                                   ctypes.POINTER(vp), i, ip, i, vp]
    lib.c3pt_insertion_noalloc.argtypes = lib.c3pt_insertion.argtypes
    lib.c3pt_insertion_noalloc.restype = ctypes.c_int
    lib.c3pt_noalloc_scratch_bytes.argtypes = []
    lib.c3pt_noalloc_scratch_bytes.restype = ctypes.c_ulonglong
    lib.c3pt_debug_scale_allocations.argtypes = [ctypes.c_double]
    lib.c3pt_debug_scale_allocations.restype = None
    lib.c3pt_combine.argtypes = [vp, i, vp, i, i, i, i, i, i, i, ctypes.POINTER(ctypes.c_double), ip, i,
                                 vp, vp]
    lib.c3pt_two_sink_meson.argtypes = [gp, vp, vp, i, vp, vp, i, i, i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                        ctypes.POINTER(vp), i, ip, i, ctypes.POINTER(ctypes.c_double), ip, i,
                                        vp, vp, vp, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.c3pt_gamma_meson.argtypes = [vp, i, dp, i, dp, i, dp, i, vp, vp]
    lib.c3pt_gamma_nucleon.argtypes = [vp, i, i, dp, dp, dp, i, dp, i, vp, vp]
    lib.c3pt_smear.argtypes = [gp, vp, vp, i, i, vp, ctypes.c_double, i]
    for name in ("c3pt_spectator_meson", "c3pt_spectator_baryon", "c3pt_insertion", "c3pt_combine",
                 "c3pt_two_sink_meson", "c3pt_gamma_meson", "c3pt_gamma_nucleon", "c3pt_smear"):
        getattr(lib, name).restype = ctypes.c_int
    lib.c3pt_strerror.argtypes = [i]
    lib.c3pt_strerror.restype = ctypes.c_char_p
    lib.c3pt_last_error.argtypes = []
    lib.c3pt_last_error.restype = ctypes.c_char_p
    lib.c3pt_version.restype = ctypes.c_int
    lib.c3pt_scratch_bytes.argtypes = [vp]
    lib.c3pt_scratch_bytes.restype = ctypes.c_ulonglong
    lib.c3pt_release_scratch.restype = ctypes.c_int
    lib.c3pt_profile_enable.argtypes = [i]
    lib.c3pt_profile_enable.restype = ctypes.c_int
    lib.c3pt_profile_read.argtypes = [ctypes.POINTER(_KernelStat), i, i]
    lib.c3pt_profile_read.restype = ctypes.c_int
    for name in ("c3pt_variant_count", "c3pt_set_variant", "c3pt_get_variant"):
        getattr(lib, name).restype = ctypes.c_int
    lib.c3pt_variant_count.argtypes = [i, i, i]
    lib.c3pt_set_variant.argtypes = [i, i, i, i]
    lib.c3pt_get_variant.argtypes = [i, i, i]
    lib.c3pt_batch_create.argtypes = [ctypes.POINTER(_Job), i, ctypes.POINTER(_CombineJob), i, ip, i, i,
                                      ctypes.c_ulonglong, ctypes.POINTER(vp)]
    lib.c3pt_batch_run.argtypes = [vp, vp]
    lib.c3pt_batch_info.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_ulonglong)]
    lib.c3pt_batch_destroy.argtypes = [vp]
    for name in ("c3pt_batch_create", "c3pt_batch_run", "c3pt_batch_info", "c3pt_batch_destroy"):
        getattr(lib, name).restype = ctypes.c_int
    ull = ctypes.c_ulonglong
    lib.c3pt_server_create.argtypes = [i, vp, ull, ull, i, vp, ctypes.POINTER(vp)]
    lib.c3pt_server_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ctypes.c_longlong)]
    lib.c3pt_server_step.argtypes = [vp, ip, ip]
    lib.c3pt_server_poll.argtypes = [vp, ctypes.c_longlong]
    lib.c3pt_server_result.argtypes = [vp, ctypes.c_longlong, ctypes.POINTER(_Result)]
    lib.c3pt_server_release.argtypes = [vp, ctypes.c_longlong]
    lib.c3pt_server_info.argtypes = [vp, ip, ip, ctypes.POINTER(ull)]
    lib.c3pt_server_destroy.argtypes = [vp]
    lib.c3pt_server_set_step_work.argtypes = [vp, ctypes.c_double]
    for name in ("c3pt_server_create", "c3pt_server_submit", "c3pt_server_step", "c3pt_server_poll",
                 "c3pt_server_result", "c3pt_server_release", "c3pt_server_info", "c3pt_server_destroy",
                 "c3pt_server_set_step_work"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


lib = _load()


def _check(rc: int):
    if rc != C3PT_OK:
        raise C3ptError(rc, lib.c3pt_last_error().decode() or lib.c3pt_strerror(rc).decode())


@dataclass
class Geom:
    """Lattice geometry and execution options of one call (c3pt_geom)."""
    L: Sequence[int]
    T: int
    r: Sequence[int] = (0, 0, 0)
    proj: int = PROJ_NATIVE
    stream: Optional[int] = None      # raw hipStream_t; None = torch's current stream

    def c(self, dtype: torch.dtype) -> _Geom:
        g = _Geom()
        for j in range(3):
            g.L[j] = int(self.L[j])
            g.r[j] = int(self.r[j])
        g.T = int(self.T)
        g.dtype = C3PT_C128 if dtype == torch.complex128 else C3PT_C64
        g.proj = int(self.proj)
        st = self.stream if self.stream is not None else torch.cuda.current_stream().cuda_stream
        g.stream = ctypes.c_void_p(st)
        return g

    @property
    def V3(self) -> int:
        return int(self.L[0]) * int(self.L[1]) * int(self.L[2])


def _field(t: torch.Tensor, name: str, shape, dtype) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


def _momenta(k):
    import numpy as np
    ka = np.ascontiguousarray(np.asarray(k, dtype=np.int32).reshape(-1, 3))
    return ka, ka.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ka.shape[0]


def _out(out, shape, like: torch.Tensor):
    if out is None:
        return torch.empty(shape, dtype=torch.complex128, device=like.device)
    _field(out, "out", shape, torch.complex128)
    return out


def c3pt_spectator_meson(G_tf: torch.Tensor, eta: torch.Tensor, k, geom: Geom, out=None) -> torch.Tensor:
    """Meson spectator, Eq. (9).  G_tf [12,12,V3], eta [N,12,V3] -> [N, n_mom, 192] complex128."""
    V3 = geom.V3
    N = eta.shape[0]
    _field(G_tf, "G_tf", (12, 12, V3), G_tf.dtype)
    _field(eta, "eta", (N, 12, V3), G_tf.dtype)
    ka, kp, n_mom = _momenta(k)
    out = _out(out, (N, n_mom, 192), G_tf)
    g = geom.c(G_tf.dtype)
    _check(lib.c3pt_spectator_meson(ctypes.byref(g), G_tf.data_ptr(), eta.data_ptr(), N, kp, n_mom,
                                    out.data_ptr()))
    return out


def c3pt_spectator_baryon(G1_tf: torch.Tensor, G2_tf: torch.Tensor, eta: torch.Tensor, k, geom: Geom,
                          out=None) -> torch.Tensor:
    """Epsilon-tensor (nucleon-type) spectator -> [N, n_mom, 3072] complex128."""
    V3 = geom.V3
    N = eta.shape[0]
    _field(G1_tf, "G1_tf", (12, 12, V3), G1_tf.dtype)
    _field(G2_tf, "G2_tf", (12, 12, V3), G1_tf.dtype)
    _field(eta, "eta", (N, 12, V3), G1_tf.dtype)
    ka, kp, n_mom = _momenta(k)
    out = _out(out, (N, n_mom, 3072), G1_tf)
    g = geom.c(G1_tf.dtype)
    _check(lib.c3pt_spectator_baryon(ctypes.byref(g), G1_tf.data_ptr(), G2_tf.data_ptr(), eta.data_ptr(),
                                     N, kp, n_mom, out.data_ptr()))
    return out


def _slice_table(slices, T: int, name: str, shape, dtype):
    arr = (ctypes.c_void_p * T)()
    if slices is None:
        return arr
    items = slices.items() if isinstance(slices, dict) else enumerate(slices)
    for t, x in items:
        if x is None:
            continue
        if not 0 <= int(t) < T:
            raise ValueError(f"{name}: timeslice {t} outside [0, {T})")
        arr[int(t)] = _field(x, f"{name}[{t}]", shape, dtype)
    return arr


def c3pt_insertion(G_t, s_t, taus, k, geom: Geom, U_t=None, n_ops: int = 1, out=None) -> torch.Tensor:
    """Insertion, Eq. (10), for every tau in taus.

    G_t, s_t, U_t: dict or list indexed by timeslice t (missing / None allowed
    where not needed); G_t[t] [12,12,V3], s_t[t] [N,12,V3], U_t[t] [4,3,3,V3].
    Returns [N, n_tau, n_ops, n_mom, 192] complex128."""
    return _insertion_call(lib.c3pt_insertion, G_t, s_t, taus, k, geom, U_t, n_ops, out)


def c3pt_insertion_noalloc(G_t, s_t, taus, k, geom: Geom, U_t=None, n_ops: int = 1, out=None) -> torch.Tensor:
    """c3pt_insertion through the entry point that allocates no device memory
    in the library (fixed scratch array; n_ops 1 or 5, factored projection).
    With out given, the call itself allocates nothing anywhere."""
    return _insertion_call(lib.c3pt_insertion_noalloc, G_t, s_t, taus, k, geom, U_t, n_ops, out)


def noalloc_scratch_bytes() -> int:
    return int(lib.c3pt_noalloc_scratch_bytes())


def _insertion_call(fn, G_t, s_t, taus, k, geom: Geom, U_t, n_ops: int, out):
    V3, T = geom.V3, int(geom.T)
    taus = [int(t) for t in taus]
    first = (s_t[taus[0]])
    N = first.shape[0]
    dtype = first.dtype
    Gtab = _slice_table(G_t, T, "G_t", (12, 12, V3), dtype)
    stab = _slice_table(s_t, T, "s_t", (N, 12, V3), dtype)
    Utab = _slice_table(U_t, T, "U_t", (4, 3, 3, V3), dtype) if U_t is not None else None
    ka, kp, n_mom = _momenta(k)
    out = _out(out, (N, len(taus), n_ops, n_mom, 192), first)
    tau_arr = (ctypes.c_int * len(taus))(*taus)
    g = geom.c(dtype)
    _check(fn(ctypes.byref(g), Gtab, stab, N, tau_arr, len(taus), Utab if Utab is not None else None, n_ops, kp,
              n_mom, out.data_ptr()))
    return out


def c3pt_combine(spec: torch.Tensor, ins: torch.Tensor, w=None, pairs=None, op_begin: int = 0,
                 op_end: Optional[int] = None, out=None, stream: Optional[int] = None) -> torch.Tensor:
    """Noise-weighted product of spectator [N, n_p, spin*3] and insertion
    [N, n_tau, n_ops, n_q, 192] -> [n_pairs, n_tau, n_sel, spin, 64] complex128."""
    import numpy as np
    N, n_p, sc = spec.shape
    spin = sc // 3
    _, n_tau, n_ops, n_q, _ = ins.shape
    _field(spec, "spec", (N, n_p, sc), torch.complex128)
    _field(ins, "ins", (N, n_tau, n_ops, n_q, 192), torch.complex128)
    op_end = n_ops if op_end is None else int(op_end)
    wp = None
    if w is not None:
        wa = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(N))
        wp = wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if pairs is None:
        n_pairs, pp = n_p * n_q, None
    else:
        pa = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        n_pairs, pp = pa.shape[0], pa.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    out = _out(out, (n_pairs, n_tau, op_end - op_begin, spin, 64), spec)
    st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
    _check(lib.c3pt_combine(spec.data_ptr(), spin, ins.data_ptr(), N, n_p, n_q, n_tau, n_ops, op_begin,
                            op_end, wp, pp, n_pairs, out.data_ptr(), ctypes.c_void_p(st)))
    return out


def c3pt_two_sink_meson(G_fwd: torch.Tensor, eta_fwd: torch.Tensor, t_fwd: int, G_bwd: torch.Tensor,
                        eta_bwd: torch.Tensor, t_bwd: int, t_src: int, G_t, s_t, k, geom: Geom, U_t=None,
                        n_ops: int = 1, w=None, pairs=None) -> dict:
    """Forward and backward meson diagrams with time-partitioned noise (one
    call of c3pt_two_sink_meson).  Returns {"spec": [2, N, n_mom, 192],
    "ins": [N, n_span, n_ops, n_mom, 192], "fwd": [n_pairs, n_fwd, n_ops, 64, 64],
    "bwd": [n_pairs, n_bwd, n_ops, 64, 64], "taus": span timeslices}, complex128."""
    import numpy as np
    V3, T = geom.V3, int(geom.T)
    N = eta_fwd.shape[0]
    dtype = eta_fwd.dtype
    _field(G_fwd, "G_fwd", (12, 12, V3), dtype)
    _field(G_bwd, "G_bwd", (12, 12, V3), dtype)
    _field(eta_fwd, "eta_fwd", (N, 12, V3), dtype)
    _field(eta_bwd, "eta_bwd", (N, 12, V3), dtype)
    t_fwd, t_src, t_bwd = int(t_fwd), int(t_src), int(t_bwd)
    n_fwd = (t_src - t_fwd) % T + 1
    n_bwd = (t_bwd - t_src) % T + 1
    n_span = n_fwd + n_bwd - 1
    Gtab = _slice_table(G_t, T, "G_t", (12, 12, V3), dtype)
    stab = _slice_table(s_t, T, "s_t", (N, 12, V3), dtype)
    Utab = _slice_table(U_t, T, "U_t", (4, 3, 3, V3), dtype) if U_t is not None else None
    ka, kp, n_mom = _momenta(k)
    wp = None
    if w is not None:
        wa = np.ascontiguousarray(np.asarray(w, dtype=np.float64).reshape(N))
        wp = wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if pairs is None:
        n_pairs, pp = n_mom * n_mom, None
    else:
        pa = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
        n_pairs, pp = pa.shape[0], pa.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    spec = _out(None, (2, N, n_mom, 192), eta_fwd)
    ins = _out(None, (N, n_span, n_ops, n_mom, 192), eta_fwd)
    fwd = _out(None, (n_pairs, n_fwd, n_ops, 64, 64), eta_fwd)
    bwd = _out(None, (n_pairs, n_bwd, n_ops, 64, 64), eta_fwd)
    g = geom.c(dtype)
    _check(lib.c3pt_two_sink_meson(ctypes.byref(g), G_fwd.data_ptr(), eta_fwd.data_ptr(), t_fwd, G_bwd.data_ptr(),
                                   eta_bwd.data_ptr(), t_bwd, t_src, N, Gtab, stab,
                                   Utab if Utab is not None else None, n_ops, kp, n_mom, wp, pp, n_pairs,
                                   spec.data_ptr(), ins.data_ptr(), fwd.data_ptr(), bwd.data_ptr()))
    taus = [(t_fwd + j) % T for j in range(n_span)]
    return {"spec": spec, "ins": ins, "fwd": fwd, "bwd": bwd, "taus": taus}


def _mats(m, name):
    """Host complex matrices [n][4][4] as (pointer, count, keep-alive array), or NULL."""
    import numpy as np
    if m is None:
        return None, 0, None
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(-1, 4, 4))
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.shape[0], a


def _stream(stream):
    return ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream().cuda_stream)


def c3pt_gamma_meson(C: torch.Tensor, g_snk=None, g_ins=None, g_src=None, out=None, stream=None) -> torch.Tensor:
    """Gamma channels of meson combine output C [..., 64, 64] (c3pt_gamma_meson).
    Returns [..., n_snk, n_ins, n_src]; None selects the 16 Gamma_n (sink and
    insertion) and gamma4 Gamma_n^dag gamma4 (source)."""
    if C.shape[-2:] != (64, 64):
        raise ValueError(f"C: shape {tuple(C.shape)}, expected [..., 64, 64]")
    _field(C, "C", tuple(C.shape), torch.complex128)
    n_blk = C.numel() // 4096
    ps, ns, ks = _mats(g_snk, "g_snk")
    pi, ni, ki = _mats(g_ins, "g_ins")
    pc, nc, kc = _mats(g_src, "g_src")
    ns, ni, nc = ns or 16, ni or 16, nc or 16
    shape = tuple(C.shape[:-2]) + (ns, ni, nc)
    out = _out(out, shape, C)
    _check(lib.c3pt_gamma_meson(C.data_ptr(), n_blk, ps, ns, pi, ni, pc, nc, out.data_ptr(), _stream(stream)))
    return out


def c3pt_gamma_nucleon(C: torch.Tensor, channel: int, A=None, Abar=None, P=None, g_ins=None, out=None,
                       stream=None) -> torch.Tensor:
    """Proton channels of nucleon combine output C [..., 1024, 64] (c3pt_gamma_nucleon).
    Returns [..., n_proj, n_ins]."""
    if C.shape[-2:] != (1024, 64):
        raise ValueError(f"C: shape {tuple(C.shape)}, expected [..., 1024, 64]")
    _field(C, "C", tuple(C.shape), torch.complex128)
    n_blk = C.numel() // 65536
    pa, na, ka = _mats(A, "A")
    pb, nb, kb = _mats(Abar, "Abar")
    if na not in (0, 1) or nb not in (0, 1):
        raise ValueError("A and Abar are single 4x4 matrices")
    pp, npj, kp = _mats(P, "P")
    pi, ni, ki = _mats(g_ins, "g_ins")
    npj, ni = npj or 2, ni or 16
    shape = tuple(C.shape[:-2]) + (npj, ni)
    out = _out(out, shape, C)
    _check(lib.c3pt_gamma_nucleon(C.data_ptr(), n_blk, int(channel), pa, pb, pp, npj, pi, ni, out.data_ptr(),
                                  _stream(stream)))
    return out


def _smear(field, U, geom: Geom, kappa: float, n_iter: int, n_outer: int, n_inner: int, out=None):
    V3 = geom.V3
    dtype = field.dtype
    _field(field, "field", tuple(field.shape), dtype)
    _field(U, "U", (4, 3, 3, V3), dtype)
    if out is None:
        out = torch.empty_like(field)
    else:
        _field(out, "out", tuple(field.shape), dtype)
    g = geom.c(dtype)
    _check(lib.c3pt_smear(ctypes.byref(g), field.data_ptr(), out.data_ptr(), n_outer, n_inner, U.data_ptr(),
                          float(kappa), int(n_iter)))
    return out


def smear_propagator(G: torch.Tensor, U: torch.Tensor, geom: Geom, kappa: float, n_iter: int, out=None):
    """Smear a propagator slice [12, 12, V3] on its row (field point) index (c3pt_smear)."""
    if tuple(G.shape) != (12, 12, geom.V3):
        raise ValueError(f"G: shape {tuple(G.shape)}, expected (12, 12, {geom.V3})")
    return _smear(G, U, geom, kappa, n_iter, 4, 12, out)


def smear_vectors(v: torch.Tensor, U: torch.Tensor, geom: Geom, kappa: float, n_iter: int, out=None):
    """Smear noise or solution vectors [N, 12, V3] (c3pt_smear)."""
    if v.dim() != 3 or tuple(v.shape[1:]) != (12, geom.V3):
        raise ValueError(f"v: shape {tuple(v.shape)}, expected (N, 12, {geom.V3})")
    return _smear(v, U, geom, kappa, n_iter, 4 * v.shape[0], 1, out)


spectator_meson = c3pt_spectator_meson
spectator_baryon = c3pt_spectator_baryon
insertion = c3pt_insertion
insertion_noalloc = c3pt_insertion_noalloc
combine = c3pt_combine
two_sink_meson = c3pt_two_sink_meson
gamma_meson = c3pt_gamma_meson
gamma_nucleon = c3pt_gamma_nucleon


def momentum_list(n2max: int):
    """Integer momenta k with |k|^2 <= n2max as an int32 array [n][3], ordered by
    |k|^2, then k1, k2, k3 (p = 2 pi k / L)."""
    import numpy as np
    kmax = 0
    while (kmax + 1) * (kmax + 1) <= n2max:
        kmax += 1
    rng = np.arange(-kmax, kmax + 1)
    k1, k2, k3 = np.meshgrid(rng, rng, rng, indexing="ij")
    ks = np.stack([k1.ravel(), k2.ravel(), k3.ravel()], axis=1)
    n2 = (ks * ks).sum(axis=1)
    ks, n2 = ks[n2 <= n2max], n2[n2 <= n2max]
    order = np.lexsort((ks[:, 2], ks[:, 1], ks[:, 0], n2))
    return np.ascontiguousarray(ks[order].astype(np.int32))


def version() -> int:
    return int(lib.c3pt_version())


def mt_class(n_mom: int, f64: bool = False) -> int:
    """Momentum-tile class of a call with n_mom momenta (FP64 groups of 32 use class 0)."""
    if f64:
        return 0
    mt = (min(n_mom, 128) + 7) // 8
    return 0 if mt <= 4 else 1 if mt <= 8 else 2 if mt <= 12 else 3


def variant_count(kind: int, mode: int, cls: int) -> int:
    return int(lib.c3pt_variant_count(kind, mode, cls))


def set_variant(kind: int, mode: int, cls: int, variant: int) -> None:
    _check(lib.c3pt_set_variant(kind, mode, cls, variant))


def get_variant(kind: int, mode: int, cls: int) -> int:
    v = int(lib.c3pt_get_variant(kind, mode, cls))
    if v < 0:
        _check(v)
    return v


def apply_tuning(table) -> int:
    """Select kernel variants from a tuning table (dict or JSON path); returns entries applied."""
    import json
    if isinstance(table, str):
        if not os.path.exists(table):
            return 0
        with open(table) as f:
            table = json.load(f)
    n = 0
    for e in table.get("entries", []):
        if variant_count(e["kind"], e["mode"], e["mt_class"]) > e["variant"]:
            set_variant(e["kind"], e["mode"], e["mt_class"], e["variant"])
            n += 1
    return n


DEFAULT_TUNING = os.path.join(_HERE, "tuning_mi355x.json")
apply_tuning(os.environ.get("C3PT_TUNING", DEFAULT_TUNING))


def profile_enable(on: bool = True) -> None:
    """Bracket every library kernel with HIP events on its stream (c3pt_profile_enable)."""
    _check(lib.c3pt_profile_enable(1 if on else 0))


def profile_read(reset: bool = False) -> dict:
    """Per-kernel {name: {count, total_ms, min_ms, max_ms, avg_ms}} (c3pt_profile_read)."""
    arr = (_KernelStat * 64)()
    n = lib.c3pt_profile_read(arr, 64, 1 if reset else 0)
    if n < 0:
        _check(n)
    out = {}
    for j in range(min(n, 64)):
        s = arr[j]
        out[s.name.decode()] = {"count": int(s.count), "total_ms": s.total_ms, "min_ms": s.min_ms,
                                "max_ms": s.max_ms, "avg_ms": s.total_ms / max(1, s.count)}
    return out


# ---------------------------------------------------------------------------
# Batches (c3pt_batch_*): many spectator / insertion calls and their combines,
# recorded once into a HIP graph and replayed.
# ---------------------------------------------------------------------------
JOB_KIND = {"spectator_meson": 0, "spectator_baryon": 1, "insertion": 2}


class Batch:
    """A recorded batch of jobs (c3pt_batch_create) replayed by ``run()``.

    ``jobs``: list of dicts with ``kind`` ("spectator_meson", "spectator_baryon",
    "insertion"), ``L``, ``T``, optional ``r``, and the inputs of the matching
    single call: ``G``, ``eta`` (meson); ``G1``, ``G2``, ``eta`` (baryon);
    ``G_t``, ``s_t``, ``taus``, optional ``U_t`` and ``n_ops`` (insertion).
    ``combines``: list of dicts with ``spec``, ``ins`` (job indices) and the
    optional ``w``, ``pairs``, ``op_begin``, ``op_end`` of c3pt_combine.
    All inputs are complex64 device tensors; they are held by the batch and
    may be refilled in place between runs.  Outputs (complex128, single-call
    layout) are ``outputs[i]`` and ``combine_outputs[j]``."""

    def __init__(self, jobs, k, proj: int = PROJ_NATIVE, combines=(), partial_budget: int = 0):
        import numpy as np
        self._keep = []
        self._handle = ctypes.c_void_p()
        ka, kp, n_mom = _momenta(k)
        self.n_mom = n_mom
        cjobs = (_Job * len(jobs))()
        self.outputs = []
        dt = torch.complex64
        for i, j in enumerate(jobs):
            kind = JOB_KIND[j["kind"]]
            L = [int(x) for x in j["L"]]
            T = int(j["T"])
            V3 = L[0] * L[1] * L[2]
            c = cjobs[i]
            c.kind = kind
            for d in range(3):
                c.L[d] = L[d]
                c.r[d] = int(j.get("r", (0, 0, 0))[d])
            c.T = T
            if kind in (0, 1):
                eta = j["eta"]
                N = eta.shape[0]
                c.eta = _field(eta, "eta", (N, 12, V3), dt)
                if kind == 0:
                    c.G = _field(j["G"], "G", (12, 12, V3), dt)
                    self._keep += [j["G"], eta]
                    shape = (N, n_mom, 192)
                else:
                    c.G = _field(j["G1"], "G1", (12, 12, V3), dt)
                    c.G2 = _field(j["G2"], "G2", (12, 12, V3), dt)
                    self._keep += [j["G1"], j["G2"], eta]
                    shape = (N, n_mom, 3072)
            else:
                taus = [int(t) for t in j["taus"]]
                N = j["s_t"][taus[0]].shape[0]
                n_ops = int(j.get("n_ops", 1))
                Gtab = _slice_table(j["G_t"], T, "G_t", (12, 12, V3), dt)
                stab = _slice_table(j["s_t"], T, "s_t", (N, 12, V3), dt)
                Utab = _slice_table(j.get("U_t"), T, "U_t", (4, 3, 3, V3), dt)
                tau_arr = (ctypes.c_int * len(taus))(*taus)
                self._keep += [Gtab, stab, Utab, tau_arr, j["G_t"], j["s_t"], j.get("U_t")]
                c.G_t = ctypes.cast(Gtab, ctypes.POINTER(ctypes.c_void_p))
                c.s_t = ctypes.cast(stab, ctypes.POINTER(ctypes.c_void_p))
                c.U_t = ctypes.cast(Utab, ctypes.POINTER(ctypes.c_void_p)) if j.get("U_t") is not None else None
                c.taus = ctypes.cast(tau_arr, ctypes.POINTER(ctypes.c_int))
                c.n_tau = len(taus)
                c.n_ops = n_ops
                shape = (N, len(taus), n_ops, n_mom, 192)
            c.n_noise = N
            out = j.get("out")
            out = torch.empty(shape, dtype=torch.complex128, device="cuda") if out is None else out
            _field(out, "out", shape, torch.complex128)
            c.out = out.data_ptr()
            self.outputs.append(out)
        ccomb = (_CombineJob * max(1, len(combines)))()
        self.combine_outputs = []
        for i, cm in enumerate(combines):
            s_i, q_i = int(cm["spec"]), int(cm["ins"])
            spec_out, ins_out = self.outputs[s_i], self.outputs[q_i]
            N, _, sc = spec_out.shape
            n_tau, n_ops = ins_out.shape[1], ins_out.shape[2]
            op_begin = int(cm.get("op_begin", 0))
            op_end = int(cm.get("op_end", n_ops))
            c = ccomb[i]
            c.spec_job, c.ins_job, c.op_begin, c.op_end = s_i, q_i, op_begin, op_end
            if cm.get("w") is not None:
                wa = np.ascontiguousarray(np.asarray(cm["w"], dtype=np.float64).reshape(N))
                self._keep.append(wa)
                c.w = wa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            if cm.get("pairs") is not None:
                pa = np.ascontiguousarray(np.asarray(cm["pairs"], dtype=np.int32).reshape(-1, 2))
                self._keep.append(pa)
                c.pairs = pa.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
                n_pairs = pa.shape[0]
            else:
                n_pairs = n_mom * n_mom
            c.n_pairs = n_pairs
            out = torch.empty((n_pairs, n_tau, op_end - op_begin, sc // 3, 64), dtype=torch.complex128,
                              device="cuda")
            c.out = out.data_ptr()
            self.combine_outputs.append(out)
        # inputs written by torch on its current stream must be complete before
        # creation builds tables and records the graph on a stream of its own
        torch.cuda.current_stream().synchronize()
        _check(lib.c3pt_batch_create(cjobs, len(jobs), ccomb if combines else None, len(combines), kp, n_mom,
                                     int(proj), int(partial_budget), ctypes.byref(self._handle)))

    def run(self, stream: Optional[int] = None) -> None:
        st = stream if stream is not None else torch.cuda.current_stream().cuda_stream
        _check(lib.c3pt_batch_run(self._handle, ctypes.c_void_p(st)))

    def info(self) -> dict:
        n_items, n_groups, pb = ctypes.c_int(), ctypes.c_int(), ctypes.c_ulonglong()
        _check(lib.c3pt_batch_info(self._handle, ctypes.byref(n_items), ctypes.byref(n_groups), ctypes.byref(pb)))
        return {"items": n_items.value, "groups": n_groups.value, "partial_bytes": pb.value}

    def close(self) -> None:
        if self._handle:
            _check(lib.c3pt_batch_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Serving (c3pt_server_*): continuous batching of contraction requests.
# ---------------------------------------------------------------------------
REQ_KIND = {"meson": 0, "nucleon": 1}


class Server:
    """Continuous-batching engine (c3pt_server_*).

    The arena (outputs of admitted requests) is a torch uint8 tensor owned by
    this object; results are returned as complex128 views into it, valid until
    ``release(id)``.  Requests name device tensors that must stay allocated
    until the request is released; the object keeps references to them."""

    def __init__(self, proj: int = PROJ_NATIVE, arena_bytes: int = 1 << 30, step_bytes: int = 256 << 20,
                 max_active: int = 8, stream=None, step_work: float = 0.0):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self._handle = ctypes.c_void_p()
        self._keep = {}
        self._shapes = {}
        torch.cuda.current_stream().synchronize()
        _check(lib.c3pt_server_create(int(proj), self.arena.data_ptr(), int(arena_bytes), int(step_bytes),
                                      int(max_active), ctypes.c_void_p(self.stream.cuda_stream),
                                      ctypes.byref(self._handle)))
        if step_work:
            _check(lib.c3pt_server_set_step_work(self._handle, float(step_work)))

    def submit(self, req: dict) -> int:
        """req: kind ("meson" | "nucleon"), L, T, r, t_src, t_f, eta [N,12,V3], G_t (dict/list of
        [12,12,V3] slices), G2_t (nucleon), s_t ([N,12,V3] slices), optional U_t and n_ops (1 or 5),
        k (momenta [n][3]), optional pairs [n_pairs][2].  All tensors complex64 on the GPU."""
        import numpy as np
        dt = torch.complex64
        L = [int(x) for x in req["L"]]
        T = int(req["T"])
        V3 = L[0] * L[1] * L[2]
        eta = req["eta"]
        N = eta.shape[0]
        n_ops = int(req.get("n_ops", 1))
        c = _Request()
        c.kind = REQ_KIND[req["kind"]]
        for d in range(3):
            c.L[d] = L[d]
            c.r[d] = int(req.get("r", (0, 0, 0))[d])
        c.T, c.t_src, c.t_f, c.n_noise, c.n_ops = T, int(req["t_src"]), int(req["t_f"]), N, n_ops
        c.eta = _field(eta, "eta", (N, 12, V3), dt)
        Gt = _slice_table(req["G_t"], T, "G_t", (12, 12, V3), dt)
        G2t = _slice_table(req.get("G2_t"), T, "G2_t", (12, 12, V3), dt)
        st = _slice_table(req["s_t"], T, "s_t", (N, 12, V3), dt)
        Ut = _slice_table(req.get("U_t"), T, "U_t", (4, 3, 3, V3), dt)
        c.G_t = ctypes.cast(Gt, ctypes.POINTER(ctypes.c_void_p))
        c.G2_t = ctypes.cast(G2t, ctypes.POINTER(ctypes.c_void_p)) if req.get("G2_t") is not None else None
        c.s_t = ctypes.cast(st, ctypes.POINTER(ctypes.c_void_p))
        c.U_t = ctypes.cast(Ut, ctypes.POINTER(ctypes.c_void_p)) if req.get("U_t") is not None else None
        ka, kp, n_mom = _momenta(req["k"])
        c.k, c.n_mom = kp, n_mom
        if req.get("pairs") is not None:
            pa = np.ascontiguousarray(np.asarray(req["pairs"], dtype=np.int32).reshape(-1, 2))
            c.pairs, c.n_pairs = pa.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), pa.shape[0]
            n_pairs = pa.shape[0]
        else:
            n_pairs = n_mom * n_mom
        rid = ctypes.c_longlong()
        _check(lib.c3pt_server_submit(self._handle, ctypes.byref(c), ctypes.byref(rid)))
        self._keep[rid.value] = (req, Gt, G2t, st, Ut)
        t0, tf = int(req["t_src"]), int(req["t_f"])
        n_tau = (tf - t0) % T + 1
        spin = 64 if c.kind == 0 else 1024
        self._shapes[rid.value] = {"spec": (N, n_mom, spin * 3), "ins": (N, n_tau, n_ops, n_mom, 192),
                                   "comb": (n_pairs, n_tau, n_ops, spin, 64), "parts": 1 if c.kind == 0 else 2}
        return rid.value

    def step(self):
        na, nq = ctypes.c_int(), ctypes.c_int()
        _check(lib.c3pt_server_step(self._handle, ctypes.byref(na), ctypes.byref(nq)))
        return na.value, nq.value

    def poll(self, rid: int) -> bool:
        rc = int(lib.c3pt_server_poll(self._handle, int(rid)))
        if rc < 0:
            _check(rc)
        return rc == 1

    def result(self, rid: int) -> dict:
        """Views of the request's outputs: spec, ins, comb (lists over parts)."""
        r = _Result()
        _check(lib.c3pt_server_result(self._handle, int(rid), ctypes.byref(r)))
        sh = self._shapes[int(rid)]
        base = self.arena.data_ptr()
        out = {}
        for name in ("spec", "ins", "comb"):
            views = []
            for p in range(sh["parts"]):
                n = 1
                for x in sh[name]:
                    n *= x
                off = getattr(r, name)[p] - base
                views.append(self.arena[off: off + 16 * n].view(torch.complex128).view(sh[name]))
            out[name] = views
        return out

    def release(self, rid: int) -> None:
        _check(lib.c3pt_server_release(self._handle, int(rid)))
        self._keep.pop(int(rid), None)
        self._shapes.pop(int(rid), None)

    def info(self) -> dict:
        na, nq, lf = ctypes.c_int(), ctypes.c_int(), ctypes.c_ulonglong()
        _check(lib.c3pt_server_info(self._handle, ctypes.byref(na), ctypes.byref(nq), ctypes.byref(lf)))
        return {"active": na.value, "queued": nq.value, "largest_free": lf.value}

    def run_until_done(self, ids) -> None:
        """Step until every request in ids has completed."""
        pending = set(int(i) for i in ids)
        while pending:
            na, nq = self.step()
            pending = {i for i in pending if not self.poll(i)}
            if pending and na == 0:
                if nq == 0:                 # everything left is enqueued: wait for it
                    self.stream.synchronize()
                    pending = {i for i in pending if not self.poll(i)}
                else:                       # nothing running: the next step must admit
                    na2, nq2 = self.step()
                    if na2 == 0 and nq2 == nq:
                        raise C3ptError(C3PT_ENOMEM, "queued requests cannot be admitted: the arena is held "
                                                     "by results that were not released")
                    pending = {i for i in pending if not self.poll(i)}

    def close(self) -> None:
        if self._handle:
            _check(lib.c3pt_server_destroy(self._handle))
            self._handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
