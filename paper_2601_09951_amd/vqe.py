"""Python binding of libvqe: handles plus thin calls that marshal torch tensors.

Every computation runs in the HIP library; this module only converts
arguments (device pointers, the current HIP stream, host arrays) and raises
on error codes.  PyTorch provides device memory and streams.

Names follow the problem statement of arXiv 2601.09951: prepare the
reference state, apply the ansatz U(theta), expect <psi|H|psi>, gradient,
optimiser step, and the per-bond-length loop of Algorithm 1.
"""
from __future__ import annotations

import ctypes
from typing import Sequence, Union

import numpy as np
import torch

from . import capi
from .capi import VQEError, check, lib

_P = ctypes.c_void_p


def _stream(device=None):
    return _P(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: torch.Tensor):
    return _P(t.data_ptr())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a: np.ndarray):
    return a.ctypes.data_as(_P)


_DEDICATED = {}  # (device, index) -> torch.cuda.ExternalStream on a hardware queue of its own


class Context:
    """A libvqe context bound to one device (device=-1: host-only planning)."""

    def __init__(self, device: int = 0):
        h = _P()
        rc = lib().vqe_ctx_create(int(device), ctypes.byref(h))
        if rc:
            raise VQEError(rc, f"vqe_ctx_create({device}) failed: {lib().vqe_strerror(rc).decode()}")
        self._h = h
        self.device = device

    @property
    def handle(self):
        return self._h

    def check(self, rc):
        check(rc, self._h)

    def set_tile(self, k_fwd: int = 0, k_rev: int = 0, c_low: int = 0):
        self.check(lib().vqe_ctx_set_tile(self._h, k_fwd, k_rev, c_low))

    def set_mem_budget(self, nbytes: int):
        self.check(lib().vqe_ctx_set_mem_budget(self._h, int(nbytes)))

    def set_loop_mode(self, mode: int):
        """0: persistent single-launch loop when the state fits on chip; 1: per-step launches."""
        self.check(lib().vqe_ctx_set_loop_mode(self._h, int(mode)))

    def set_staged(self, staged):
        """Pass kernels: 2 or True (default): fused stages where a forward pass
        allows them, register stages elsewhere; 1: register stages only;
        0 or False: one LDS round trip per gate."""
        mode = 2 if staged is True else (0 if staged is False else int(staged))
        self.check(lib().vqe_ctx_set_staged(self._h, mode))

    def set_profiling(self, on: bool = True):
        """Time the pass, sweep and loop launches with HIP events on their streams."""
        self.check(lib().vqe_ctx_set_profiling(self._h, 1 if on else 0))

    def profile(self, reset: bool = True) -> dict:
        """Per-kernel totals of the timed launches: {name: {launches, ms, bytes}}
        (waits for the timed launches to finish)."""
        cnt = ctypes.c_int()
        self.check(lib().vqe_ctx_profile(self._h, None, 0, ctypes.byref(cnt), 0))
        buf = (capi.KernelStat * max(1, cnt.value))()
        self.check(lib().vqe_ctx_profile(self._h, buf, cnt.value, ctypes.byref(cnt), 1 if reset else 0))
        return {buf[i].name.decode(): {"launches": int(buf[i].launches), "ms": float(buf[i].total_ms),
                                       "bytes": float(buf[i].bytes)} for i in range(cnt.value)}

    def reserve(self, nbytes: int):
        self.check(lib().vqe_ctx_reserve(self._h, int(nbytes)))

    def set_graphs(self, on: bool = True):
        """Capture repeated launch sequences into hipGraphs and replay them (default on)."""
        self.check(lib().vqe_ctx_set_graphs(self._h, 1 if on else 0))

    def graph_stats(self) -> dict:
        c, l, k = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self.check(lib().vqe_ctx_graph_stats(self._h, ctypes.byref(c), ctypes.byref(l), ctypes.byref(k)))
        return {"captures": c.value, "launches": l.value, "cached": k.value}

    def clear_tuning(self):
        self.check(lib().vqe_ctx_clear_tuning(self._h))

    def dedicated_stream(self, index: int):
        """Stream `index` of this device's dedicated streams: a HIP stream on a
        hardware queue of its own (vqe_stream_create), as a
        torch.cuda.ExternalStream.  Like torch's own stream pool these live
        until the process ends (torch's pinned-memory allocator records
        events on the streams a buffer was copied on when it frees the
        buffer, so a stream must outlive every tensor used on it)."""
        key = (self.device, int(index))
        if key not in _DEDICATED:
            h = _P()
            self.check(lib().vqe_stream_create(self._h, ctypes.byref(h)))
            _DEDICATED[key] = torch.cuda.ExternalStream(h.value, device=torch.device(f"cuda:{self.device}"))
        return _DEDICATED[key]

    def close(self):
        if self._h:
            lib().vqe_ctx_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class Hamiltonian:
    """A Pauli sum resident on the device (vqe_ham_t)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self._h = handle
        n = ctypes.c_int()
        t = ctypes.c_int64()
        g = ctypes.c_int64()
        ctx.check(lib().vqe_ham_info(handle, ctypes.byref(n), ctypes.byref(t), ctypes.byref(g)))
        self.n_qubits, self.n_terms, self.n_groups = n.value, t.value, g.value

    @classmethod
    def from_pauli(cls, ctx: Context, n_qubits: int, xmask, zmask, coeff) -> "Hamiltonian":
        x, z, c = _host(xmask, np.uint64), _host(zmask, np.uint64), _host(coeff, np.float64)
        h = _P()
        ctx.check(lib().vqe_ham_create(ctx.handle, int(n_qubits), int(c.shape[0]), _hp(x), _hp(z), _hp(c),
                                       ctypes.byref(h)))
        return cls(ctx, h)

    @classmethod
    def from_sum(cls, ctx: Context, pauli_sum) -> "Hamiltonian":
        """From any object with n, xmask, zmask, coeff."""
        return cls.from_pauli(ctx, pauli_sum.n, pauli_sum.xmask, pauli_sum.zmask, pauli_sum.coeff)

    @classmethod
    def from_integrals(cls, ctx: Context, h1, h2, e_core: float = 0.0) -> "Hamiltonian":
        h1 = _host(h1, np.float64)
        h2 = _host(h2, np.float64)
        n_orb = h1.shape[0]
        if h1.shape != (n_orb, n_orb) or h2.shape != (n_orb,) * 4:
            raise ValueError("h1 must be [n_orb, n_orb] and h2 [n_orb]^4")
        h = _P()
        ctx.check(lib().vqe_ham_from_integrals(ctx.handle, n_orb, _hp(h1), _hp(h2), float(e_core),
                                               ctypes.byref(h)))
        return cls(ctx, h)

    def terms(self):
        x = np.zeros(self.n_terms, dtype=np.uint64)
        z = np.zeros(self.n_terms, dtype=np.uint64)
        c = np.zeros(self.n_terms, dtype=np.float64)
        self.ctx.check(lib().vqe_ham_terms(self._h, _hp(x), _hp(z), _hp(c)))
        return x, z, c

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().vqe_ham_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class HamFamily:
    """Eq. (3) for many integral sets: the Jordan-Wigner map integrals ->
    coefficients, with member Hamiltonians whose coefficients live on the device."""

    def __init__(self, ctx: Context, n_orb: int, capacity: int):
        h = _P()
        ctx.check(lib().vqe_hfam_create(ctx.handle, int(n_orb), int(capacity), ctypes.byref(h)))
        self.ctx = ctx
        self._h = h
        self.n_orb = int(n_orb)
        self.capacity = int(capacity)
        nq, nt, ni = ctypes.c_int(), ctypes.c_int64(), ctypes.c_int64()
        ctx.check(lib().vqe_hfam_info(h, ctypes.byref(nq), ctypes.byref(nt), ctypes.byref(ni)))
        self.n_qubits, self.n_terms, self.n_inputs = nq.value, nt.value, ni.value
        self._members = []

    def member(self, index: int) -> "Hamiltonian":
        h = _P()
        self.ctx.check(lib().vqe_hfam_member(self._h, int(index), ctypes.byref(h)))
        m = Hamiltonian(self.ctx, h)
        self._members.append(m)
        return m

    def members(self, count: int, first: int = 0):
        return [self.member(first + i) for i in range(count)]

    @staticmethod
    def pack(integrals) -> np.ndarray:
        """[count, 1 + n^2 + n^4] float64 rows {e_core, h1, h2} from objects with h1, h2, e_core."""
        return np.stack([np.concatenate([[float(i.e_core)], np.asarray(i.h1, dtype=np.float64).ravel(),
                                         np.asarray(i.h2, dtype=np.float64).ravel()]) for i in integrals])

    def set_integrals(self, ints: torch.Tensor, first: int = 0):
        """Coefficients of members [first, first + len(ints)) from device integrals."""
        _check_tensor(ints, torch.float64, (ints.shape[0], self.n_inputs), "integrals")
        self.ctx.check(lib().vqe_hfam_set_integrals(self.ctx.handle, self._h, int(first), int(ints.shape[0]),
                                                    _ptr(ints), _stream(ints.device)))

    def close(self):
        for m in self._members:
            m.close()
        self._members = []
        if self._h:
            lib().vqe_hfam_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class Circuit:
    """An ansatz gate list compiled by the library (vqe_circ_t)."""

    def __init__(self, ctx: Context, n_qubits: int, kinds: Sequence[Union[str, int]], wires, param_idx,
                 fixed_angle=None, n_params: int = None, ref_index: int = 0):
        k = _host([capi.GATE_CODES[x] if isinstance(x, str) else int(x) for x in kinds], np.int32)
        w = _host(wires, np.int32).reshape(-1, 4)
        p = _host(param_idx, np.int32)
        f = _host(fixed_angle if fixed_angle is not None else np.zeros(len(k)), np.float64)
        if n_params is None:
            n_params = int(p.max()) + 1 if p.size and p.max() >= 0 else 0
        h = _P()
        ctx.check(lib().vqe_circ_create(ctx.handle, int(n_qubits), int(k.shape[0]), _hp(k), _hp(w), _hp(p),
                                        _hp(f), int(n_params), ctypes.byref(h)))
        self.ctx = ctx
        self._h = h
        self.n_qubits = int(n_qubits)
        self.n_params = int(n_params)
        self.n_gates = int(k.shape[0])
        self.ref_index = int(ref_index)

    @classmethod
    def from_spec(cls, ctx: Context, spec) -> "Circuit":
        """From any object with n, kinds, wires, param_idx, fixed_angle, n_params, ref_index."""
        return cls(ctx, spec.n, spec.kinds, spec.wires, spec.param_idx, spec.fixed_angle, spec.n_params,
                   spec.ref_index)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().vqe_circ_destroy(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


def _hams_array(hams):
    if isinstance(hams, Hamiltonian):
        hams = [hams]
    arr = (_P * len(hams))(*[h.handle for h in hams])
    return arr, len(hams)


def _check_tensor(t: torch.Tensor, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


# ---------------------------------------------------------------------------
# the hot path
# ---------------------------------------------------------------------------
def workspace_bytes(ctx: Context, circ: Circuit, hams, batch: int, want_grad: int) -> int:
    arr, nh = _hams_array(hams)
    out = ctypes.c_size_t()
    ctx.check(lib().vqe_workspace_bytes(ctx.handle, circ.handle, nh, arr, int(batch), int(want_grad),
                                        ctypes.byref(out)))
    return out.value


def workspace(ctx: Context, circ: Circuit, hams, batch: int, want_grad: int, device=None) -> torch.Tensor:
    nbytes = workspace_bytes(ctx, circ, hams, batch, want_grad)
    return torch.empty(nbytes, dtype=torch.uint8, device=device or f"cuda:{ctx.device}")


def prepare_reference(ctx: Context, n_qubits: int, batch: int, ref_index: int, psi: torch.Tensor):
    _check_tensor(psi, torch.complex128, (batch, 1 << n_qubits), "psi")
    ctx.check(lib().vqe_prepare_reference(ctx.handle, n_qubits, batch, ref_index, _ptr(psi), _stream(psi.device)))


def apply_ansatz(ctx: Context, circ: Circuit, theta: torch.Tensor, psi: torch.Tensor):
    B = psi.shape[0]
    _check_tensor(psi, torch.complex128, (B, 1 << circ.n_qubits), "psi")
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    ctx.check(lib().vqe_apply_ansatz(ctx.handle, circ.handle, B, _ptr(theta), _ptr(psi), _stream(psi.device)))


def expect(ctx: Context, hams, psi: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    arr, nh = _hams_array(hams)
    B = psi.shape[0]
    _check_tensor(psi, torch.complex128, None, "psi")
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=psi.device)
    _check_tensor(out, torch.float64, (B,), "energy")
    ctx.check(lib().vqe_expect(ctx.handle, nh, arr, B, _ptr(psi), _ptr(out), _stream(psi.device)))
    return out


def apply_ansatz_noalloc(ctx: Context, circ: Circuit, theta: torch.Tensor, psi: torch.Tensor):
    """vqe_apply_ansatz_noalloc: apply_ansatz with the matrices in the library's
    static per-GPU array (no allocation; overlapping calls on one GPU race)."""
    B = psi.shape[0]
    _check_tensor(psi, torch.complex128, (B, 1 << circ.n_qubits), "psi")
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    ctx.check(lib().vqe_apply_ansatz_noalloc(ctx.handle, circ.handle, B, _ptr(theta), _ptr(psi),
                                             _stream(psi.device)))


def apply_hamiltonian(ctx: Context, hams, psi: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    arr, nh = _hams_array(hams)
    _check_tensor(psi, torch.complex128, None, "psi")
    if out is None:
        out = torch.empty_like(psi)
    _check_tensor(out, torch.complex128, tuple(psi.shape), "out")
    ctx.check(lib().vqe_apply_hamiltonian(ctx.handle, nh, arr, psi.shape[0], _ptr(psi), _ptr(out),
                                          _stream(psi.device)))
    return out


def energy(ctx: Context, circ: Circuit, hams, theta: torch.Tensor, ref_index: int = None,
           ws: torch.Tensor = None, out: torch.Tensor = None) -> torch.Tensor:
    B = theta.shape[0]
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    arr, nh = _hams_array(hams)
    ref = circ.ref_index if ref_index is None else ref_index
    if ws is None:
        ws = workspace(ctx, circ, hams, B, 0, theta.device)
    if out is None:
        out = torch.empty(B, dtype=torch.float64, device=theta.device)
    ctx.check(lib().vqe_energy(ctx.handle, circ.handle, nh, arr, B, ref, _ptr(theta), _ptr(out), _ptr(ws),
                               ws.numel(), _stream(theta.device)))
    return out


def energy_grad(ctx: Context, circ: Circuit, hams, theta: torch.Tensor, ref_index: int = None,
                ws: torch.Tensor = None, out_e: torch.Tensor = None, out_g: torch.Tensor = None):
    B = theta.shape[0]
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    arr, nh = _hams_array(hams)
    ref = circ.ref_index if ref_index is None else ref_index
    if ws is None:
        ws = workspace(ctx, circ, hams, B, 1, theta.device)
    if out_e is None:
        out_e = torch.empty(B, dtype=torch.float64, device=theta.device)
    if out_g is None:
        out_g = torch.empty(B, circ.n_params, dtype=torch.float64, device=theta.device)
    ctx.check(lib().vqe_energy_grad(ctx.handle, circ.handle, nh, arr, B, ref, _ptr(theta), _ptr(out_e),
                                    _ptr(out_g), _ptr(ws), ws.numel(), _stream(theta.device)))
    return out_e, out_g


def autotune(ctx: Context, circ: Circuit, hams, theta: torch.Tensor, want_grad: bool = True,
             ref_index: int = None) -> dict:
    """vqe_autotune: time candidate tiles, batch tile and workgroup cap for this
    (circuit, batch) on energy (+ gradient) calls and keep the fastest.  Size
    workspaces after tuning (the choice changes vqe_workspace_bytes)."""
    B = theta.shape[0]
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    arr, nh = _hams_array(hams)
    ref = circ.ref_index if ref_index is None else ref_index
    r = capi.TuneResult()
    ctx.check(lib().vqe_autotune(ctx.handle, circ.handle, nh, arr, B, ref, 1 if want_grad else 0, _ptr(theta),
                                 _stream(theta.device), ctypes.byref(r)))
    return {"k_fwd": r.k_fwd, "k_rev": r.k_rev, "c_low": r.c_low, "wg_max": r.wg_max,
            "batch_tile": int(r.batch_tile), "ms_default": r.ms_default, "ms_tuned": r.ms_tuned,
            "candidates": r.candidates}


def tune_set(ctx: Context, circ: Circuit, batch: int, want_grad: bool, k_fwd: int = 12, k_rev: int = 11,
             c_low: int = 3, wg_max: int = 8192, batch_tile: int = None):
    """vqe_tune_set: pin an execution configuration for (circuit, batch, mode)."""
    r = capi.TuneResult(k_fwd=k_fwd, k_rev=k_rev, c_low=c_low, wg_max=wg_max,
                        batch_tile=int(batch if batch_tile is None else batch_tile))
    ctx.check(lib().vqe_tune_set(ctx.handle, circ.handle, int(batch), 1 if want_grad else 0, ctypes.byref(r)))


def grad_shift(ctx: Context, circ: Circuit, hams, theta: torch.Tensor, ref_index: int = None,
               ws: torch.Tensor = None):
    """(E, dE/dtheta) by the parameter-shift rules (Algorithm 1), all shifted rows in one batch."""
    B = theta.shape[0]
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    arr, nh = _hams_array(hams)
    ref = circ.ref_index if ref_index is None else ref_index
    if ws is None:
        ws = workspace(ctx, circ, hams, B, 3, theta.device)
    e = torch.empty(B, dtype=torch.float64, device=theta.device)
    g = torch.empty(B, circ.n_params, dtype=torch.float64, device=theta.device)
    ctx.check(lib().vqe_grad_shift(ctx.handle, circ.handle, nh, arr, B, ref, _ptr(theta), _ptr(e), _ptr(g),
                                   _ptr(ws), ws.numel(), _stream(theta.device)))
    return e, g


def adam_step(ctx: Context, theta: torch.Tensor, m: torch.Tensor, v: torch.Tensor, grad: torch.Tensor, t: int,
              lr: float = 0.01, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    B, P = theta.shape
    for name, a in (("theta", theta), ("m", m), ("v", v), ("grad", grad)):
        _check_tensor(a, torch.float64, (B, P), name)
    ctx.check(lib().vqe_adam_step(ctx.handle, B, P, _ptr(theta), _ptr(m), _ptr(v), _ptr(grad), int(t), lr, b1,
                                  b2, eps, _stream(theta.device)))


def run(ctx: Context, circ: Circuit, hams, theta: torch.Tensor, iters: int, optimizer: str = "adam",
        lr: float = 0.01, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, ref_index: int = None,
        ws: torch.Tensor = None, energies: torch.Tensor = None) -> torch.Tensor:
    """Algorithm 1's loop for a batch: theta is updated in place.

    Returns energies [B, iters + 1] (before each step, then at the final theta).
    """
    B = theta.shape[0]
    _check_tensor(theta, torch.float64, (B, circ.n_params), "theta")
    arr, nh = _hams_array(hams)
    ref = circ.ref_index if ref_index is None else ref_index
    if ws is None:
        ws = workspace(ctx, circ, hams, B, 2, theta.device)
    if energies is None:
        energies = torch.empty(B, iters + 1, dtype=torch.float64, device=theta.device)
    opt = {"adam": capi.OPT_ADAM, "gd": capi.OPT_GD}[optimizer]
    ctx.check(lib().vqe_run(ctx.handle, circ.handle, nh, arr, B, ref, _ptr(theta), int(iters), opt, lr, b1, b2,
                            eps, _ptr(energies), _ptr(ws), ws.numel(), _stream(theta.device)))
    return energies


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------
class VQEEnergy(torch.autograd.Function):
    """E(theta) with the adjoint gradient computed by the library.

    ``VQEEnergy.apply(theta[B, P], ctx, circ, hams)`` returns E[B]; when theta
    requires grad the forward pass runs the adjoint sweep and keeps dE/dtheta
    for backward, which returns grad_E[:, None] * dE/dtheta.
    """

    @staticmethod
    def forward(fctx, theta, ctx, circ, hams):
        th = theta.detach().contiguous()
        if theta.requires_grad:
            e, g = energy_grad(ctx, circ, hams, th)
            fctx.save_for_backward(g)
        else:
            e = energy(ctx, circ, hams, th)
        return e

    @staticmethod
    def backward(fctx, grad_e):
        (g,) = fctx.saved_tensors
        return grad_e[:, None] * g, None, None, None


# ---------------------------------------------------------------------------
# schedule inspection
# ---------------------------------------------------------------------------
_GEOM = np.dtype([("n", "<i4"), ("k", "<i4"), ("c", "<i4"), ("nout", "<i4"), ("tpos", "u1", 16),
                  ("opos", "u1", 40)])
_PASS = np.dtype([("geom", _GEOM), ("op_begin", "<i4"), ("op_count", "<i4"), ("n_param_ops", "<i4"),
                  ("stage_begin", "<i4"), ("stage_count", "<i4"), ("fstage_begin", "<i4"), ("fstage_count", "<i4"),
                  ("pad", "<i4")])
_STAGE = np.dtype([("rpos", "u1", 4), ("cpos", "u1", 12), ("op_begin", "<i4"), ("op_count", "<i4"),
                   ("n_param_ops", "<i4"), ("nbits", "<i4"), ("cpack", "<u8"), ("rpack", "<u4"), ("pad2", "<u4")])
_SOP = np.dtype([("cmo", "<u8"), ("cvo", "<u8"), ("cmt", "<u4"), ("cvt", "<u4"), ("gate", "<i4"),
                 ("pgate", "<i4"), ("M", "u1"), ("lo", "u1"), ("cmr", "u1"), ("cvr", "u1"), ("swap", "u1"),
                 ("cls", "u1"), ("gen", "u1"), ("pad", "u1"), ("amask", "<u2"), ("pad2", "<u2", 3)])
_FSTAGE = np.dtype([("rpos", "u1", 4), ("cpos", "u1", 12), ("lr", "<u2", 16), ("lc", "<u2", 12), ("c0", "<u2"),
                    ("perm", "<u2"), ("na", "<i4"), ("cond_begin", "<i4"), ("cond_count", "<i4"), ("slot", "<i4"),
                    ("nb", "<i4"), ("phase_begin", "<i4"), ("phase_count", "<i4"), ("xbit", "<i4")])
_FCOND = np.dtype([("cmo", "<u8"), ("cvo", "<u8"), ("xmask", "<u4"), ("pad", "<u4")])
_FPHASE = np.dtype([("mask", "<u4"), ("cbit", "<u4"), ("gate", "<i4"), ("info", "<i4")])
_OP = np.dtype([("m", "<u4"), ("fixed_bits", "<u4"), ("cmask_out", "<u8"), ("cval_out", "<u8"),
                ("gate", "<i4"), ("pgate", "<i4"), ("cls", "<i2"), ("gen", "<i2"), ("nfix", "i1"),
                ("fixpos", "u1", 7), ("pad", "<u4")])
_SWEEP = np.dtype([("geom", _GEOM), ("grp_begin", "<i4"), ("grp_count", "<i4"), ("pad", "<i4", 2)])
_GROUP = np.dtype([("floc", "<u4"), ("pivot", "<u4"), ("ugroup", "<i4"), ("pad", "<i4")])
_TERM = np.dtype([("z", "<u8"), ("zloc", "<u4"), ("pad", "<u4"), ("w", "<f8")])
_WIDE = np.dtype([("f", "<u8"), ("pivot", "<i4"), ("ugroup", "<i4")])


def circuit_plan(ctx: Context, circ: Circuit, reverse: bool = False, stages: bool = False):
    """(passes, ops) structured arrays of the compiled pass schedule
    (plus (stages, stage_ops) when stages=True; with stages="fused":
    (passes, ops, fused_stages, fused_conds, slot_offsets, slot_gates, slot_info, phases))."""
    need = ctypes.c_size_t()
    ctx.check(lib().vqe_circ_plan_export(ctx.handle, circ.handle, int(reverse), None, 0, ctypes.byref(need)))
    buf = np.zeros(need.value, dtype=np.uint8)
    ctx.check(lib().vqe_circ_plan_export(ctx.handle, circ.handle, int(reverse), _hp(buf), buf.size,
                                         ctypes.byref(need)))
    hdr = buf[:32].view("<i4")
    npass, nops, nst, nsop = int(hdr[0]), int(hdr[1]), int(hdr[4]), int(hdr[5])
    assert hdr[2] == _GEOM.itemsize and hdr[3] == _OP.itemsize
    assert hdr[6] == _STAGE.itemsize and hdr[7] == _SOP.itemsize
    off = 32
    passes = buf[off:off + npass * _PASS.itemsize].view(_PASS)
    off += npass * _PASS.itemsize
    ops = buf[off:off + nops * _OP.itemsize].view(_OP)
    off += nops * _OP.itemsize
    st = buf[off:off + nst * _STAGE.itemsize].view(_STAGE)
    off += nst * _STAGE.itemsize
    sops = buf[off:off + nsop * _SOP.itemsize].view(_SOP)
    off += nsop * _SOP.itemsize
    if stages == "fused":
        fh = buf[off:off + 32].view("<i4")
        nfs, nfc, nsl, nsg, nph = int(fh[0]), int(fh[2]), int(fh[4]), int(fh[5]), int(fh[6])
        assert fh[1] == _FSTAGE.itemsize and fh[3] == _FCOND.itemsize and fh[7] == _FPHASE.itemsize
        off += 32
        fst = buf[off:off + nfs * _FSTAGE.itemsize].view(_FSTAGE)
        off += nfs * _FSTAGE.itemsize
        fco = buf[off:off + nfc * _FCOND.itemsize].view(_FCOND)
        off += nfc * _FCOND.itemsize
        soff = buf[off:off + (nsl + 1) * 4].view("<i4")
        off += (nsl + 1) * 4
        sgate = buf[off:off + nsg * 4].view("<i4")
        off += nsg * 4
        sinfo = buf[off:off + nsg * 4].view("<i4")
        off += nsg * 4
        fph = buf[off:off + nph * _FPHASE.itemsize].view(_FPHASE)
        return passes, ops, fst, fco, soff, sgate, sinfo, fph
    if stages:
        return passes, ops, st, sops
    return passes, ops


def hamiltonian_plan(ctx: Context, hams, batch: int = 1, for_gradient: bool = False):
    """dict of structured arrays describing the flip-group sweep schedule."""
    arr, nh = _hams_array(hams)
    need = ctypes.c_size_t()
    ctx.check(lib().vqe_ham_plan_export(ctx.handle, nh, arr, int(batch), int(for_gradient), None, 0,
                                        ctypes.byref(need)))
    buf = np.zeros(need.value, dtype=np.uint8)
    ctx.check(lib().vqe_ham_plan_export(ctx.handle, nh, arr, int(batch), int(for_gradient), _hp(buf), buf.size,
                                        ctypes.byref(need)))
    hdr = buf[:32].view("<i4")
    ns, ng, nu, ni, nt = (int(v) for v in hdr[:5])
    assert hdr[5] == _GEOM.itemsize and hdr[6] == _GROUP.itemsize and hdr[7] == _TERM.itemsize
    off = 32
    sweeps = buf[off:off + ns * _SWEEP.itemsize].view(_SWEEP)
    off += ns * _SWEEP.itemsize
    groups = buf[off:off + ng * _GROUP.itemsize].view(_GROUP)
    off += ng * _GROUP.itemsize
    toff = buf[off:off + ni * nu * 3 * 4].view("<i4").reshape(ni, nu, 3)
    off += ni * nu * 3 * 4
    terms = buf[off:off + nt * _TERM.itemsize].view(_TERM)
    off += nt * _TERM.itemsize
    nw, wsz = (int(v) for v in buf[off:off + 8].view("<i4"))
    assert wsz == _WIDE.itemsize
    off += 8
    wide = buf[off:off + nw * _WIDE.itemsize].view(_WIDE)
    return {"sweeps": sweeps, "groups": groups, "toff": toff, "terms": terms, "wide": wide, "n_union": nu,
            "n_inst": ni}
