"""The oracle: a plain, slow, obviously-correct CPU reference of the VQE hot path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package's smoke check and
the CPU-baseline leg of the benchmark may import this package.  The product
library never imports it, and this package imports nothing from the product.

Parts
-----
* ``statevec.c`` (built with gcc into ``_liboracle.so``): FP64 state-vector
  simulation by explicit gate matrices, term-by-term Pauli expectation with
  compensated summation, parameter-shift and plain adjoint gradients, Adam
  and the per-bond-length VQE loop (Eq. 2, Eqs. 4-5, Algorithm 1, Sections
  3.4 and 4.3 of arXiv 2601.09951).
* ``fermion.py``: the second-quantised Hamiltonian of Eq. (3) built as a
  dense matrix from Jordan-Wigner creation/annihilation matrices, and its
  Pauli decomposition by traces.

Every function states the passage it follows.  Parity of the 30/32-qubit
configurations is unpinned by this oracle (host memory), see the test notes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import fermion  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "statevec.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None

GATES = {
    "RX": 0, "RY": 1, "RZ": 2, "H": 3, "X": 4,
    "CNOT": 5, "CZ": 6, "SingleExcitation": 7, "DoubleExcitation": 8,
}


def build(force: bool = False) -> str:
    """Compile statevec.c with gcc (plain -O2, IEEE semantics, OpenMP for timing)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu99", "-fPIC", "-shared", "-fopenmp",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
            L.orc_set_threads.argtypes = [i32]
            L.orc_prepare.argtypes = [i32, u64, P]
            L.orc_apply_gate.argtypes = [i32, P, i32, P, f64, i32]
            L.orc_apply_gate.restype = i32
            L.orc_apply_generator.argtypes = [i32, P, i32, P]
            L.orc_apply_generator.restype = i32
            L.orc_apply_circuit.argtypes = [i32, P, i32, P, P, P, P, P]
            L.orc_apply_circuit.restype = i32
            L.orc_expect_pauli.argtypes = [i32, P, u64, u64, P, P]
            L.orc_expect.argtypes = [i32, P, i64, P, P, P, P, P]
            L.orc_apply_hamiltonian.argtypes = [i32, P, i64, P, P, P, P]
            L.orc_energy.argtypes = [i32, i32, P, P, P, P, i32, u64, i64, P, P, P, P, P, P]
            L.orc_energy.restype = i32
            L.orc_energy_grad.argtypes = [i32, i32, P, P, P, P, i32, u64, i64, P, P, P, P, i32, P, P]
            L.orc_energy_grad.restype = i32
            L.orc_adam_step.argtypes = [i32, P, P, P, P, i32, f64, f64, f64, f64]
            L.orc_vqe_run.argtypes = [i32, i32, P, P, P, P, i32, u64, i64, P, P, P, P, i32, i32,
                                      f64, f64, f64, f64, i32, P]
            L.orc_vqe_run.restype = i32
            _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class _Circ:
    def __init__(self, circ):
        self.n = circ.n
        self.kind = _c([GATES[k] for k in circ.kinds], np.int32)
        self.wires = _c(circ.wires, np.int32).reshape(-1, 4)
        self.pidx = _c(circ.param_idx, np.int32)
        self.fixed = _c(circ.fixed_angle, np.float64)
        self.n_gates = len(circ.kinds)
        self.n_params = int(circ.n_params)
        self.ref = int(circ.ref_index)


class _Ham:
    def __init__(self, ham):
        self.x = _c(ham.xmask, np.uint64)
        self.z = _c(ham.zmask, np.uint64)
        self.c = _c(ham.coeff, np.float64)
        self.T = int(self.c.shape[0])


# ---------------------------------------------------------------------------
# state-level helpers
# ---------------------------------------------------------------------------
def prepare(n: int, ref: int) -> np.ndarray:
    """The reference basis state e_ref (Eq. 4's |HF>)."""
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().orc_prepare(n, ref, _p(psi))
    return psi


def apply_gate(psi: np.ndarray, kind: str, wires, angle: float = 0.0, adjoint: bool = False) -> np.ndarray:
    """Apply one gate (explicit matrix) to a copy of psi."""
    out = _c(psi, np.complex128).copy()
    n = int(out.shape[0]).bit_length() - 1
    w = _c(list(wires) + [-1] * (4 - len(wires)), np.int32)
    rc = lib().orc_apply_gate(n, _p(out), GATES[kind], _p(w), float(angle), int(adjoint))
    if rc:
        raise ValueError("bad gate")
    return out


def apply_generator(psi: np.ndarray, kind: str, wires) -> np.ndarray:
    out = _c(psi, np.complex128).copy()
    n = int(out.shape[0]).bit_length() - 1
    w = _c(list(wires) + [-1] * (4 - len(wires)), np.int32)
    if lib().orc_apply_generator(n, _p(out), GATES[kind], _p(w)):
        raise ValueError("gate has no generator")
    return out


def state(circ, theta) -> np.ndarray:
    """psi(theta) = U(theta)|ref> (Eq. 4)."""
    C = _Circ(circ)
    th = _c(theta, np.float64)
    psi = prepare(C.n, C.ref)
    rc = lib().orc_apply_circuit(C.n, _p(psi), C.n_gates, _p(C.kind), _p(C.wires), _p(C.pidx),
                                 _p(C.fixed), _p(th))
    if rc:
        raise ValueError("bad circuit")
    return psi


def expect_pauli(psi: np.ndarray, x: int, z: int) -> complex:
    n = int(psi.shape[0]).bit_length() - 1
    re, im = ctypes.c_double(), ctypes.c_double()
    psi = _c(psi, np.complex128)
    lib().orc_expect_pauli(n, _p(psi), int(x), int(z), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def expect(psi: np.ndarray, ham) -> complex:
    """<psi|H|psi> term by term (Eq. 2)."""
    H = _Ham(ham)
    psi = _c(psi, np.complex128)
    n = int(psi.shape[0]).bit_length() - 1
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().orc_expect(n, _p(psi), H.T, _p(H.x), _p(H.z), _p(H.c), ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def apply_hamiltonian(psi: np.ndarray, ham) -> np.ndarray:
    H = _Ham(ham)
    psi = _c(psi, np.complex128)
    n = int(psi.shape[0]).bit_length() - 1
    out = np.empty_like(psi)
    lib().orc_apply_hamiltonian(n, _p(psi), H.T, _p(H.x), _p(H.z), _p(H.c), _p(out))
    return out


# ---------------------------------------------------------------------------
# problem-level entry points
# ---------------------------------------------------------------------------
def energy(circ, ham, theta) -> float:
    C, H = _Circ(circ), _Ham(ham)
    th = _c(theta, np.float64)
    e, ei = ctypes.c_double(), ctypes.c_double()
    rc = lib().orc_energy(C.n, C.n_gates, _p(C.kind), _p(C.wires), _p(C.pidx), _p(C.fixed),
                          C.n_params, C.ref, H.T, _p(H.x), _p(H.z), _p(H.c), _p(th),
                          ctypes.byref(e), ctypes.byref(ei))
    if rc:
        raise MemoryError("oracle allocation failed")
    return e.value


def energy_grad(circ, ham, theta, method: str = "adjoint"):
    """(E, dE/dtheta) by parameter shift ('shift') or the plain adjoint ('adjoint')."""
    C, H = _Circ(circ), _Ham(ham)
    th = _c(theta, np.float64)
    g = np.zeros(C.n_params, dtype=np.float64)
    e = ctypes.c_double()
    rc = lib().orc_energy_grad(C.n, C.n_gates, _p(C.kind), _p(C.wires), _p(C.pidx), _p(C.fixed),
                               C.n_params, C.ref, H.T, _p(H.x), _p(H.z), _p(H.c), _p(th),
                               {"shift": 0, "adjoint": 1}[method], ctypes.byref(e), _p(g))
    if rc:
        raise MemoryError("oracle allocation failed")
    return e.value, g


def adam_step(theta, m, v, g, t, lr=0.01, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays (Section 3.4; Kingma-Ba form)."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().orc_adam_step(theta.shape[0], _p(theta), _p(m), _p(v), _p(g), int(t), lr, b1, b2, eps)


def vqe_run(circ, ham, theta0, iters: int, optimizer: str = "adam", lr: float = 0.01,
            b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, grad: str = "adjoint"):
    """Algorithm 1's inner loop for one bond length.

    Returns (energies[iters + 1], theta_final): the energy before each of the
    ``iters`` optimiser steps, then the energy at the final parameters.
    """
    C, H = _Circ(circ), _Ham(ham)
    th = _c(theta0, np.float64).copy()
    out = np.zeros(iters + 1, dtype=np.float64)
    rc = lib().orc_vqe_run(C.n, C.n_gates, _p(C.kind), _p(C.wires), _p(C.pidx), _p(C.fixed),
                           C.n_params, C.ref, H.T, _p(H.x), _p(H.z), _p(H.c), _p(th), int(iters),
                           {"adam": 0, "gd": 1}[optimizer], lr, b1, b2, eps,
                           {"shift": 0, "adjoint": 1}[grad], _p(out))
    if rc:
        raise MemoryError("oracle allocation failed")
    return out, th
