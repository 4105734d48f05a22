"""ctypes binding of ``libvqmc.so``: argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; torch supplies device
memory and the current HIP stream.  If the library has not been built, importing this
module raises (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvqmc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2106_13308_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

PAD = 64
F64, F32, BF16 = 0, 1, 2
OK, EINVAL, EDTYPE, EWORKSPACE, EHIP, ENONFINITE = 0, -1, -2, -3, -4, -5
H_CSR_INT, H_CSR_F32, H_DENSE_F32 = 0, 1, 2
WS_LOGPROB, WS_BACKWARD, WS_SAMPLE_PLAIN, WS_STEP, WS_BACKWARD_SAMPLED, WS_SR_GRAM, WS_SR_JVP = 0, 1, 2, 3, 4, 5, 6
WS_SR_DIRECTION = 7
WS_TIM_ENERGY, WS_TIM_STEP = 8, 9
NOALLOC_SCRATCH_BYTES = 64 << 20   # VQMC_NOALLOC_SCRATCH_BYTES
BAND_REC = 260
TAG_TRAIN, TAG_EVAL = 0, 1

_vp = ctypes.c_void_p
_i32, _i64, _u32, _u64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_size_t


class MadeC(ctypes.Structure):
    _fields_ = [("n", _i32), ("h", _i32), ("wdtype", _i32), ("P", _vp), ("Pt", _vp),
                ("b1", _vp), ("b2", _vp), ("c", _vp), ("band", _vp)]


class HamC(ctypes.Structure):
    _fields_ = [("n", _i32), ("kind", _i32), ("nnz", _i64), ("rowptr", _vp), ("col", _vp),
                ("w", _vp), ("J", _vp)]


class StatsC(ctypes.Structure):
    _fields_ = [("mean_E", ctypes.c_double), ("var_E", ctypes.c_double), ("min_E", ctypes.c_double),
                ("argmin", _i64), ("sum_E", ctypes.c_double)]


class TimC(ctypes.Structure):
    _fields_ = [("n", _i32), ("alpha", _vp), ("beta", _vp), ("J", _vp)]


STATS_BYTES = ctypes.sizeof(StatsC)

_SIGS = {
    "vqmc_ld": (_i64, [_i64]),
    "vqmc_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "vqmc_last_error": (ctypes.c_char_p, []),
    "vqmc_workspace_bytes": (_sz, [ctypes.c_int, _i32, _i32, _i64, _i32]),
    "vqmc_pack": (ctypes.c_int, [_i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vqmc_unpack": (ctypes.c_int, [_i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "vqmc_cast": (ctypes.c_int, [_i32, _i32, _vp, _i32, _vp, _vp, _vp]),
    "vqmc_band": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _vp]),
    "vqmc_band_bytes": (ctypes.c_size_t, [_i32, _i32, _i32]),
    "vqmc_refresh": (ctypes.c_int, [_i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "vqmc_check_nonfinite": (ctypes.c_int, [_i32]),
    "vqmc_sample": (ctypes.c_int, [ctypes.POINTER(MadeC), _i64, _u64, _u64, _i64, _u32, _vp, _vp, _vp]),
    "vqmc_sample_cycles": (ctypes.c_int, [ctypes.POINTER(MadeC), _i64, _u64, _u64, _vp, _vp, _vp,
                                          ctypes.POINTER(ctypes.c_int32), _vp]),
    "vqmc_sample_fwd": (ctypes.c_int, [ctypes.POINTER(MadeC), _i64, _u64, _u64, _i64, _u32, _vp, _vp, _vp, _vp,
                                       _vp]),
    "vqmc_backward_sampled": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _sz, _vp]),
    "vqmc_sample_plain": (ctypes.c_int, [ctypes.POINTER(MadeC), _i64, _u64, _u64, _i64, _u32, _vp, _vp,
                                         _vp, _sz, _vp]),
    "vqmc_energy": (ctypes.c_int, [ctypes.POINTER(HamC), _vp, _i64, _vp, _vp, _sz, _vp]),
    "vqmc_energy_workspace_bytes": (_sz, [ctypes.POINTER(HamC), _i64]),
    "vqmc_batch_stats": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _vp]),
    "vqmc_logprob": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "vqmc_logprob_noalloc": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp]),
    "vqmc_tim_energy": (ctypes.c_int, [ctypes.POINTER(MadeC), ctypes.POINTER(TimC), _vp, _i64, _vp, _vp, _vp, _sz,
                                       _vp]),
    "vqmc_tim_step": (ctypes.c_int, [ctypes.POINTER(MadeC), ctypes.POINTER(TimC), _i64, _u64, _u64, _i64, _vp, _vp,
                                     _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vqmc_logprob_backward": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, _vp, _vp,
                                             _sz, _vp]),
    "vqmc_sr_gram": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _sz, _vp]),
    "vqmc_sr_jvp": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vqmc_sr_gram_sampled": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vqmc_sr_solve": (ctypes.c_int, [_i64, _vp, ctypes.c_double, _vp, ctypes.c_double, _vp, _vp, _sz, _vp]),
    "vqmc_sr_solve_workspace_bytes": (_sz, [_i64]),
    "vqmc_sr_direction": (ctypes.c_int, [ctypes.POINTER(MadeC), _vp, _i64, _vp, _vp, _vp, ctypes.c_double, _vp, _vp,
                                         _vp, _vp, _vp, _sz, _vp]),
    "vqmc_step": (ctypes.c_int, [ctypes.POINTER(MadeC), ctypes.POINTER(HamC), _i64, _u64, _u64, _i64, _i32,
                                 _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "vqmc_csr_from_edges": (ctypes.c_int, [_i32, _i64, _vp, _vp, _i32, _vp, _vp, _vp]),
    "vqmc_uniforms": (ctypes.c_int, [_i32, _i64, _u64, _u64, _i64, _u32, _vp, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

lib = _lib


class VqmcError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = _lib.vqmc_last_error().decode(errors="replace")
        super().__init__(f"{fn} failed: {_lib.vqmc_error_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(fn: str, status: int):
    if status != OK:
        raise VqmcError(fn, status)


def ld(x: int) -> int:
    return int(_lib.vqmc_ld(x))


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t


def _need(t: torch.Tensor, name: str, dtype, shape) -> torch.Tensor:
    """A contiguous device tensor of the given dtype with at least the given leading extents."""
    _dev(t)
    if t.dtype != dtype:
        raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
    if t.dim() != len(shape) or any(a < b for a, b in zip(t.shape, shape)):
        raise ValueError(f"{name}: expected shape at least {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _need_spins(made, S: torch.Tensor, B: int) -> torch.Tensor:
    _need(S, "S", torch.int8, (B, ld(made.n)))
    if S.shape[1] != ld(made.n):
        raise ValueError(f"S: rows must be ld(n) = {ld(made.n)} long, got {S.shape[1]}")
    return S


def _need_fwd(made, Zs: torch.Tensor, Rt: torch.Tensor, B: int):
    """vqmc_sample_fwd's byproducts for B samples: Zs B x ld(n) float32, Rt h x ld(B) in the weight dtype."""
    _need(Zs, "Zs", torch.float32, (B, ld(made.n)))
    if Zs.shape[1] != ld(made.n):
        raise ValueError(f"Zs: rows must be ld(n) = {ld(made.n)} long")
    rdt = torch.bfloat16 if made.wdtype == BF16 else torch.float32
    _need(Rt, "Rt", rdt, (made.h, ld(B)))
    if Rt.shape[1] != ld(B):
        raise ValueError(f"Rt: rows must be ld(B) = {ld(B)} long, got {Rt.shape[1]}")


# ---------------------------------------------------------------- parameters
class Made:
    """MADE parameters: the FP32 master packed matrix P32 (n x h), biases, the
    staircase index c, and the kernels' working copies (P, Pt, and the sampler's band
    unless ``band=False``) in ``wdtype``."""

    def __init__(self, n: int, h: int, P32: torch.Tensor, b1: torch.Tensor, b2: torch.Tensor,
                 c: torch.Tensor, wdtype: int = F32, band: bool = True):
        self.n, self.h = int(n), int(h)
        self.P32, self.b1, self.b2, self.c = P32, b1, b2, c
        self.wdtype = wdtype
        dev = P32.device
        tdt = torch.bfloat16 if wdtype == BF16 else torch.float32
        self.P = torch.zeros((self.n, ld(self.h)), dtype=tdt, device=dev)
        self.Pt = torch.zeros((self.h, ld(self.n)), dtype=tdt, device=dev)
        nbytes = int(_lib.vqmc_band_bytes(self.n, self.h, self.wdtype)) if band else 0
        self.band = torch.zeros(nbytes // 4, dtype=torch.float32, device=dev) if band else None
        # set by every refresh when a parameter is NaN or infinite (sticky until cleared)
        self.nonfinite = torch.zeros(1, dtype=torch.int32, device=dev)
        self.refresh()

    @classmethod
    def from_dense(cls, W1, b1, W2, b2, degrees, wdtype: int = F32, device="cuda", band: bool = True):
        """Pack dense float32 weights (numpy or torch) on the device."""
        W1 = torch.as_tensor(np.asarray(W1, np.float32), device=device).contiguous()
        W2 = torch.as_tensor(np.asarray(W2, np.float32), device=device).contiguous()
        h, n = W1.shape
        deg = np.ascontiguousarray(np.asarray(degrees, np.int32))
        P32 = torch.empty((n, h), dtype=torch.float32, device=device)
        c = torch.empty(n, dtype=torch.int32, device=device)
        _check("vqmc_pack", _lib.vqmc_pack(n, h, W1.data_ptr(), W2.data_ptr(),
                                           deg.ctypes.data_as(_vp), P32.data_ptr(), c.data_ptr(), _stream()))
        b1t = torch.as_tensor(np.asarray(b1, np.float32), device=device).contiguous()
        b2t = torch.as_tensor(np.asarray(b2, np.float32), device=device).contiguous()
        return cls(n, h, P32, b1t, b2t, c, wdtype, band)

    def refresh(self):
        """Re-derive the working copies (and the sampler tables) after P32 changed (e.g. after an
        optimiser step): one vqmc_refresh call."""
        _check("vqmc_refresh", _lib.vqmc_refresh(self.n, self.h, self.P32.data_ptr(), self.wdtype,
                                                 self.P.data_ptr(), self.Pt.data_ptr(), self.b1.data_ptr(),
                                                 self.b2.data_ptr(), self.c.data_ptr(), _ptr(self.band),
                                                 self.nonfinite.data_ptr(), _stream()))

    def check_finite(self):
        """Raise VqmcError (VQMC_ENONFINITE) if a refresh has seen a NaN or infinite parameter
        (reads the device flag back: synchronises the stream)."""
        _check("vqmc_check_nonfinite", _lib.vqmc_check_nonfinite(int(self.nonfinite.item())))

    def cstruct(self) -> MadeC:
        return MadeC(self.n, self.h, self.wdtype, self.P.data_ptr(), self.Pt.data_ptr(),
                     self.b1.data_ptr(), self.b2.data_ptr(), self.c.data_ptr(), _ptr(self.band))

    def unpack(self, P32: torch.Tensor | None = None):
        """Dense (W1, W2) from a packed matrix (default: the master weights)."""
        P32 = self.P32 if P32 is None else P32
        W1 = torch.empty((self.h, self.n), dtype=torch.float32, device=P32.device)
        W2 = torch.empty((self.n, self.h), dtype=torch.float32, device=P32.device)
        _check("vqmc_unpack", _lib.vqmc_unpack(self.n, self.h, _dev(P32).data_ptr(), self.c.data_ptr(),
                                               W1.data_ptr(), W2.data_ptr(), _stream()))
        return W1, W2


class Hamiltonian:
    """Diagonal Hamiltonian sum_{i<j} J_ij s_i s_j on the device."""

    def __init__(self, n: int, kind: int, rowptr=None, col=None, w=None, J=None, W_tot=None):
        self.n, self.kind = int(n), kind
        self.rowptr, self.col, self.w, self.J = rowptr, col, w, J
        self.nnz = 0 if col is None else int(col.numel())
        self.W_tot = W_tot

    @classmethod
    def from_edges(cls, n: int, edges, weights, device="cuda"):
        edges = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
        weights = np.asarray(weights)
        integer = np.issubdtype(weights.dtype, np.integer)
        kind = H_CSR_INT if integer else H_CSR_F32
        w = np.ascontiguousarray(weights.astype(np.int32 if integer else np.float32))
        m = edges.shape[0]
        rowptr = np.zeros(n + 1, np.int64)
        col = np.zeros(max(m, 1), np.int32)
        wout = np.zeros(max(m, 1), w.dtype)
        _check("vqmc_csr_from_edges", _lib.vqmc_csr_from_edges(
            n, m, edges.ctypes.data_as(_vp), w.ctypes.data_as(_vp), kind, rowptr.ctypes.data_as(_vp),
            col.ctypes.data_as(_vp), wout.ctypes.data_as(_vp)))
        W_tot = int(w.astype(np.int64).sum()) if integer else float(w.astype(np.float64).sum())
        return cls(n, kind, torch.from_numpy(rowptr).to(device), torch.from_numpy(col[:m].copy()).to(device),
                   torch.from_numpy(wout[:m].copy()).to(device), None, W_tot)

    @classmethod
    def dense(cls, J, device="cuda"):
        J = torch.as_tensor(np.asarray(J, np.float32), device=device).contiguous()
        return cls(J.shape[0], H_DENSE_F32, J=J)

    def cstruct(self) -> HamC:
        return HamC(self.n, self.kind, self.nnz, _ptr(self.rowptr), _ptr(self.col), _ptr(self.w), _ptr(self.J))

    @property
    def e_is_int(self) -> bool:
        return self.kind == H_CSR_INT

    def energy_dtype(self):
        return torch.int64 if self.e_is_int else torch.float64


class Tim:
    """Transverse-field Ising couplings on the device: alpha (n), beta (n), beta_ij (n x n dense,
    symmetric, zero diagonal)."""

    def __init__(self, alpha, beta, J, device="cuda"):
        self.alpha = torch.as_tensor(np.asarray(alpha, np.float32), device=device).contiguous()
        self.beta = torch.as_tensor(np.asarray(beta, np.float32), device=device).contiguous()
        self.J = torch.as_tensor(np.asarray(J, np.float32), device=device).contiguous()
        self.n = int(self.alpha.numel())
        if self.beta.numel() != self.n or tuple(self.J.shape) != (self.n, self.n):
            raise ValueError("alpha, beta must have n entries and J must be n x n")
        self.W_tot = None

    def cstruct(self) -> TimC:
        return TimC(self.n, self.alpha.data_ptr(), self.beta.data_ptr(), self.J.data_ptr())

    @property
    def e_is_int(self) -> bool:
        return False

    def energy_dtype(self):
        return torch.float64


# ---------------------------------------------------------------- calls
def workspace(which: int, made: Made, B: int) -> torch.Tensor:
    nb = int(_lib.vqmc_workspace_bytes(which, made.n, made.h, B, made.wdtype))
    return torch.empty(max(nb, 256), dtype=torch.uint8, device=made.P.device)


def empty_spins(B: int, n: int, device="cuda") -> torch.Tensor:
    return torch.empty((B, ld(n)), dtype=torch.int8, device=device)


def sample(made: Made, B: int, seed: int, step: int = 0, offset: int = 0, tag: int = TAG_TRAIN,
           S: torch.Tensor | None = None, logp: torch.Tensor | None = None, want_logp: bool = True):
    """Incremental sampler.  Returns (S [B x ld(n) int8], logp [B] or None)."""
    dev = made.P.device
    S = empty_spins(B, made.n, dev) if S is None else _dev(S)
    if want_logp and logp is None:
        logp = torch.empty(B, dtype=torch.float32, device=dev)
    m = made.cstruct()
    _check("vqmc_sample", _lib.vqmc_sample(ctypes.byref(m), B, seed, step, offset, tag, S.data_ptr(),
                                           _ptr(logp), _stream()))
    return S, logp


def uniforms(n: int, B: int, seed: int, step: int = 0, offset: int = 0, tag: int = TAG_TRAIN,
             device="cuda") -> torch.Tensor:
    """The device Philox uniforms u[b][d] (B x n float32)."""
    u = torch.empty((B, n), dtype=torch.float32, device=device)
    _check("vqmc_uniforms", _lib.vqmc_uniforms(n, B, seed, step, offset, tag, u.data_ptr(), _stream()))
    return u


def sample_plain(made: Made, B: int, seed: int, step: int = 0, offset: int = 0, tag: int = TAG_TRAIN,
                 ws: torch.Tensor | None = None):
    dev = made.P.device
    S = empty_spins(B, made.n, dev)
    logp = torch.empty(B, dtype=torch.float32, device=dev)
    ws = workspace(WS_SAMPLE_PLAIN, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_sample_plain", _lib.vqmc_sample_plain(ctypes.byref(m), B, seed, step, offset, tag,
                                                       S.data_ptr(), logp.data_ptr(), ws.data_ptr(),
                                                       ws.numel(), _stream()))
    return S, logp


def energy(H: Hamiltonian, S: torch.Tensor, B: int | None = None) -> torch.Tensor:
    B = S.shape[0] if B is None else B
    E = torch.empty(B, dtype=H.energy_dtype(), device=S.device)
    hc = H.cstruct()
    nb = int(_lib.vqmc_energy_workspace_bytes(ctypes.byref(hc), B))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=S.device)
    _check("vqmc_energy", _lib.vqmc_energy(ctypes.byref(hc), _dev(S).data_ptr(), B, E.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _stream()))
    return E


def batch_stats(E: torch.Tensor, want_coef: bool = True):
    """Returns (stats dict tensor-backed, coef [B] float32)."""
    B = E.shape[0]
    st = torch.zeros(STATS_BYTES, dtype=torch.uint8, device=E.device)
    coef = torch.empty(B, dtype=torch.float32, device=E.device) if want_coef else None
    _check("vqmc_batch_stats", _lib.vqmc_batch_stats(_dev(E).data_ptr(), int(E.dtype == torch.int64), B,
                                                     st.data_ptr(), _ptr(coef), _stream()))
    return st, coef


def stats_to_dict(st: torch.Tensor) -> dict:
    raw = st.cpu().numpy().tobytes()
    s = StatsC.from_buffer_copy(raw)
    return {"mean": s.mean_E, "var": s.var_E, "min": s.min_E, "argmin": int(s.argmin), "sum": s.sum_E}


def sample_fwd(made: Made, B: int, seed: int, step: int, offset: int = 0, tag: int = TAG_TRAIN,
               S: torch.Tensor | None = None, logp: torch.Tensor | None = None, Zs: torch.Tensor | None = None,
               Rt: torch.Tensor | None = None):
    """Pipelined sampling that also returns Zs (s_d z_d, B x ld(n)) and Rt (relu(A), h x ld(B))."""
    dev = made.P.device
    S = empty_spins(B, made.n, dev) if S is None else S
    logp = torch.empty(B, dtype=torch.float32, device=dev) if logp is None else logp
    Zs = torch.empty((B, ld(made.n)), dtype=torch.float32, device=dev) if Zs is None else Zs
    if Rt is None:
        Rt = torch.empty((made.h, ld(B)), dtype=torch.bfloat16 if made.wdtype == BF16 else torch.float32, device=dev)
    m = made.cstruct()
    _check("vqmc_sample_fwd", _lib.vqmc_sample_fwd(ctypes.byref(m), B, seed, step, offset, tag, _dev(S).data_ptr(),
                                                   _dev(logp).data_ptr(), _dev(Zs).data_ptr(), _dev(Rt).data_ptr(),
                                                   _stream()))
    return S, logp, Zs, Rt


def sample_cycles(made: Made, B: int, seed: int, step: int):
    """vqmc_sample_cycles: the pipelined draw with per-wave cycle counts.  Returns (S, logp,
    cycles) with cycles a host int64 array [ceil(B / 8), waves, 3]: shader-clock cycles spent
    working between the per-block barriers, cycles from the first departure to the last, and
    that span in 100 MHz ticks (waves 0-1: the sweep)."""
    dev = made.P.device
    S = empty_spins(B, made.n, dev)
    logp = torch.empty(B, dtype=torch.float32, device=dev)
    groups = (B + 7) // 8
    cyc = torch.zeros(groups * 64 * 3, dtype=torch.int64, device=dev)  # room for up to 64 waves
    waves = ctypes.c_int32(0)
    m = made.cstruct()
    _check("vqmc_sample_cycles", _lib.vqmc_sample_cycles(ctypes.byref(m), B, seed, step, _dev(S).data_ptr(),
                                                         logp.data_ptr(), cyc.data_ptr(), ctypes.byref(waves),
                                                         _stream()))
    W = waves.value
    return S, logp, cyc[: groups * W * 3].view(groups, W, 3).cpu().numpy()


def backward_sampled(made: Made, S: torch.Tensor, coef: torch.Tensor, Zs: torch.Tensor, Rt: torch.Tensor,
                     B: int | None = None, ws: torch.Tensor | None = None):
    """Gradient of sum_b coef_b log pi(s_b) from sample_fwd's Zs and Rt (no forward recompute)."""
    B = S.shape[0] if B is None else B
    dev = S.device
    dP = torch.empty((made.n, made.h), dtype=torch.float32, device=dev)
    db1 = torch.empty(made.h, dtype=torch.float32, device=dev)
    db2 = torch.empty(made.n, dtype=torch.float32, device=dev)
    ws = workspace(WS_BACKWARD_SAMPLED, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_backward_sampled", _lib.vqmc_backward_sampled(
        ctypes.byref(m), _dev(S).data_ptr(), B, _dev(coef).data_ptr(), _dev(Zs).data_ptr(), _dev(Rt).data_ptr(),
        dP.data_ptr(), db1.data_ptr(), db2.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return dP, db1, db2


def logprob(made: Made, S: torch.Tensor, B: int | None = None, want_z: bool = False,
            ws: torch.Tensor | None = None):
    B = S.shape[0] if B is None else B
    dev = S.device
    logp = torch.empty(B, dtype=torch.float32, device=dev)
    Z = torch.empty((B, ld(made.n)), dtype=torch.float32, device=dev) if want_z else None
    ws = workspace(WS_LOGPROB, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_logprob", _lib.vqmc_logprob(ctypes.byref(m), _dev(S).data_ptr(), B, logp.data_ptr(),
                                             _ptr(Z), ws.data_ptr(), ws.numel(), _stream()))
    return (logp, Z) if want_z else logp


def logprob_noalloc(made: Made, S: torch.Tensor, B: int | None = None, want_z: bool = False,
                    logp: torch.Tensor | None = None, Z: torch.Tensor | None = None):
    """vqmc_logprob_noalloc: log pi(S) with the library's fixed scratch instead of a workspace.
    logp (B floats) and Z (B x ld(n) floats) may be passed in, so that the call allocates
    nothing at all."""
    B = S.shape[0] if B is None else B
    dev = S.device
    if logp is None:
        logp = torch.empty(B, dtype=torch.float32, device=dev)
    else:
        logp = _need(logp, "logp", torch.float32, (B,))
    if want_z and Z is None:
        Z = torch.empty((B, ld(made.n)), dtype=torch.float32, device=dev)
    elif Z is not None:
        Z = _need(Z, "Z", torch.float32, (B, ld(made.n)))
    _need_spins(made, S, B)
    m = made.cstruct()
    _check("vqmc_logprob_noalloc", _lib.vqmc_logprob_noalloc(ctypes.byref(m), _dev(S).data_ptr(), B,
                                                             logp.data_ptr(), _ptr(Z), _stream()))
    return (logp, Z) if Z is not None else logp


def logprob_backward(made: Made, S: torch.Tensor, coef: torch.Tensor, B: int | None = None,
                     ws: torch.Tensor | None = None):
    B = S.shape[0] if B is None else B
    dev = S.device
    dP = torch.empty((made.n, made.h), dtype=torch.float32, device=dev)
    db1 = torch.empty(made.h, dtype=torch.float32, device=dev)
    db2 = torch.empty(made.n, dtype=torch.float32, device=dev)
    ws = workspace(WS_BACKWARD, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_logprob_backward", _lib.vqmc_logprob_backward(
        ctypes.byref(m), _dev(S).data_ptr(), B, _dev(coef).data_ptr(), dP.data_ptr(), db1.data_ptr(),
        db2.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return dP, db1, db2


def sr_gram(made: Made, S: torch.Tensor, B: int | None = None, ws: torch.Tensor | None = None,
            K: torch.Tensor | None = None) -> torch.Tensor:
    """K = O O^T (B x B float), the sample-space Gram of the per-sample scores."""
    B = S.shape[0] if B is None else B
    _need_spins(made, S, B)
    K = torch.empty((B, B), dtype=torch.float32, device=S.device) if K is None else _need(K, "K", torch.float32, (B, B))
    ws = workspace(WS_SR_GRAM, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_sr_gram", _lib.vqmc_sr_gram(ctypes.byref(m), S.data_ptr(), B, K.data_ptr(), ws.data_ptr(),
                                              ws.numel(), _stream()))
    return K


def sr_gram_sampled(made: Made, S: torch.Tensor, Zs: torch.Tensor, Rt: torch.Tensor, B: int | None = None,
                    ws: torch.Tensor | None = None, K: torch.Tensor | None = None) -> torch.Tensor:
    """sr_gram for spins drawn by sample_fwd, from its Zs and Rt (no forward recompute)."""
    B = S.shape[0] if B is None else B
    _need_spins(made, S, B)
    _need_fwd(made, Zs, Rt, B)
    K = torch.empty((B, B), dtype=torch.float32, device=S.device) if K is None else _need(K, "K", torch.float32, (B, B))
    ws = workspace(WS_SR_GRAM, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_sr_gram_sampled", _lib.vqmc_sr_gram_sampled(
        ctypes.byref(m), S.data_ptr(), B, Zs.data_ptr(), Rt.data_ptr(), K.data_ptr(),
        ws.data_ptr(), ws.numel(), _stream()))
    return K


def sr_jvp(made: Made, S: torch.Tensor, gP: torch.Tensor, gb1: torch.Tensor, gb2: torch.Tensor,
           B: int | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """v = O g (B floats): the score of every sample contracted with the direction (gP, gb1, gb2)."""
    B = S.shape[0] if B is None else B
    _need_spins(made, S, B)
    _need(gP, "gP", torch.float32, (made.n, made.h))
    if tuple(gP.shape) != (made.n, made.h):
        raise ValueError("gP must be n x h (packed like P32)")
    _need(gb1, "gb1", torch.float32, (made.h,))
    _need(gb2, "gb2", torch.float32, (made.n,))
    v = torch.empty(B, dtype=torch.float32, device=S.device)
    ws = workspace(WS_SR_JVP, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_sr_jvp", _lib.vqmc_sr_jvp(ctypes.byref(m), S.data_ptr(), B, gP.data_ptr(), gb1.data_ptr(),
                                            gb2.data_ptr(), v.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return v


def sr_solve(K: torch.Tensor, shift: float, rhs: torch.Tensor, scale: float = 1.0,
             ws: torch.Tensor | None = None) -> torch.Tensor:
    """y = (K + shift I)^{-1} (scale rhs) by the library's FP64 Cholesky (K: B x B float32, symmetric PSD)."""
    B = rhs.shape[0]
    _need(K, "K", torch.float32, (B, B))
    if tuple(K.shape) != (B, B):
        raise ValueError("K must be B x B")
    _need(rhs, "rhs", torch.float32, (B,))
    y = torch.empty(B, dtype=torch.float32, device=K.device)
    nb = int(_lib.vqmc_sr_solve_workspace_bytes(B))
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=K.device) if ws is None else ws
    _check("vqmc_sr_solve", _lib.vqmc_sr_solve(B, K.data_ptr(), float(shift), rhs.data_ptr(), float(scale),
                                                y.data_ptr(), ws.data_ptr(), ws.numel(), _stream()))
    return y


def sr_direction(made: Made, S: torch.Tensor, coef: torch.Tensor, lam: float, B: int | None = None,
                 Zs: torch.Tensor | None = None, Rt: torch.Tensor | None = None, ws: torch.Tensor | None = None,
                 want_K: bool = False):
    """SR direction of the batch gradient sum_b coef_b grad log pi(s_b): x = O^T y with
    (K + lam B I) y = B coef.  Returns (xP n x h, xb1, xb2) and, with want_K, K."""
    B = S.shape[0] if B is None else B
    _need_spins(made, S, B)
    _need(coef, "coef", torch.float32, (B,))
    if (Zs is None) != (Rt is None):
        raise ValueError("give both Zs and Rt, or neither")
    if Zs is not None:
        _need_fwd(made, Zs, Rt, B)
    dev = S.device
    xP = torch.empty((made.n, made.h), dtype=torch.float32, device=dev)
    xb1 = torch.empty(made.h, dtype=torch.float32, device=dev)
    xb2 = torch.empty(made.n, dtype=torch.float32, device=dev)
    K = torch.empty((B, B), dtype=torch.float32, device=dev) if want_K else None
    ws = workspace(WS_SR_DIRECTION, made, B) if ws is None else ws
    m = made.cstruct()
    _check("vqmc_sr_direction", _lib.vqmc_sr_direction(
        ctypes.byref(m), S.data_ptr(), B, coef.data_ptr(), _ptr(Zs), _ptr(Rt), float(lam), xP.data_ptr(),
        xb1.data_ptr(), xb2.data_ptr(), _ptr(K), ws.data_ptr(), ws.numel(), _stream()))
    return (xP, xb1, xb2, K) if want_K else (xP, xb1, xb2)


def tim_energy(made: Made, H: Tim, S: torch.Tensor, B: int | None = None, want_D: bool = False,
               ws: torch.Tensor | None = None, E: torch.Tensor | None = None):
    """TIM local energies l(s_b) (B float64) and, with want_D, D[b][i] = log pi(s_b^(i)) - log pi(s_b)
    (B x ld(n) float32)."""
    B = S.shape[0] if B is None else B
    _need_spins(made, S, B)
    if H.n != made.n:
        raise ValueError("Hamiltonian and model sizes differ")
    dev = S.device
    E = torch.empty(B, dtype=torch.float64, device=dev) if E is None else _need(E, "E", torch.float64, (B,))
    D = torch.zeros((B, ld(made.n)), dtype=torch.float32, device=dev) if want_D else None
    ws = workspace(WS_TIM_ENERGY, made, B) if ws is None else ws
    m = made.cstruct()
    hc = H.cstruct()
    _check("vqmc_tim_energy", _lib.vqmc_tim_energy(ctypes.byref(m), ctypes.byref(hc), S.data_ptr(), B, E.data_ptr(),
                                                   _ptr(D), ws.data_ptr(), ws.numel(), _stream()))
    return (E, D) if want_D else E


@dataclass
class StepBuffers:
    """Caller-owned buffers of one optimisation step (allocated once, reused)."""
    S: torch.Tensor
    logp: torch.Tensor
    E: torch.Tensor
    stats: torch.Tensor
    coef: torch.Tensor
    dP: torch.Tensor
    db1: torch.Tensor
    db2: torch.Tensor
    ws: torch.Tensor

    @classmethod
    def allocate(cls, made: Made, H: Hamiltonian, B: int):
        dev = made.P.device
        return cls(
            S=empty_spins(B, made.n, dev),
            logp=torch.empty(B, dtype=torch.float32, device=dev),
            E=torch.empty(B, dtype=H.energy_dtype(), device=dev),
            stats=torch.zeros(STATS_BYTES, dtype=torch.uint8, device=dev),
            coef=torch.empty(B, dtype=torch.float32, device=dev),
            dP=torch.empty((made.n, made.h), dtype=torch.float32, device=dev),
            db1=torch.empty(made.h, dtype=torch.float32, device=dev),
            db2=torch.empty(made.n, dtype=torch.float32, device=dev),
            ws=workspace(WS_TIM_STEP if isinstance(H, Tim) else WS_STEP, made, B),
        )


def step(made: Made, H, B: int, seed: int, step_idx: int, bufs: StepBuffers,
         algo: int = 0, offset: int = 0):
    """One optimisation step (sample, energy, statistics, gradient) into ``bufs``: vqmc_step for
    a diagonal Hamiltonian, vqmc_tim_step for a Tim (incremental sampler only)."""
    m = made.cstruct()
    hc = H.cstruct()
    if isinstance(H, Tim):
        if algo != 0:
            raise ValueError("the TIM step runs the incremental sampler only")
        _check("vqmc_tim_step", _lib.vqmc_tim_step(
            ctypes.byref(m), ctypes.byref(hc), B, seed, step_idx, offset, bufs.S.data_ptr(), bufs.logp.data_ptr(),
            bufs.E.data_ptr(), bufs.stats.data_ptr(), bufs.coef.data_ptr(), bufs.dP.data_ptr(),
            bufs.db1.data_ptr(), bufs.db2.data_ptr(), bufs.ws.data_ptr(), bufs.ws.numel(), _stream()))
        return bufs
    _check("vqmc_step", _lib.vqmc_step(
        ctypes.byref(m), ctypes.byref(hc), B, seed, step_idx, offset, algo, bufs.S.data_ptr(),
        bufs.logp.data_ptr(), bufs.E.data_ptr(), bufs.stats.data_ptr(), bufs.coef.data_ptr(),
        bufs.dP.data_ptr(), bufs.db1.data_ptr(), bufs.db2.data_ptr(), bufs.ws.data_ptr(),
        bufs.ws.numel(), _stream()))
    return bufs
