"""Dense second-quantised Hamiltonian and its Pauli decomposition (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows arXiv 2601.09951, Section 3.2, Eq. (3):
    H = sum_{PQ} h_PQ a+_P a_Q + 1/2 sum_{PQRS} g_PQRS a+_P a+_Q a_R a_S,
mapped to qubits by the Jordan-Wigner transformation the paper names in
Sections 2.1 and 3.2.  Readings taken where the paper is silent:

* spin orbitals are interleaved (wire 2p = orbital p spin alpha, 2p+1 =
  spin beta), which is what puts both reference electrons of |1100> in the
  lowest spatial orbital with opposite spins (Section 3.3);
* two-electron integrals are chemist-notation (pq|rs) and enter as
  g_PQRS = (p s | q r) delta(spin P, spin S) delta(spin Q, spin R);
* |1> is an occupied mode, a+_P = Z_0 ... Z_{P-1} (X_P - i Y_P) / 2.

The operators are built as explicit 2^n x 2^n matrices (Kronecker products,
wire 0 the most significant factor) and H is decomposed into Pauli strings
by traces, c(x, z) = Tr(P(x, z)^dagger H) / 2^n.  Nothing here is symbolic:
it is the plain definition, slow and dense, for n <= 10.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

_I2 = np.eye(2, dtype=np.complex128)
_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_LOWER = np.array([[0, 1], [0, 0]], dtype=np.complex128)  # |0><1| removes an occupation


def _kron_all(mats):
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(out, m)
    return out


def annihilators(n_modes: int):
    """Dense a_P for P = 0..n_modes-1 (Jordan-Wigner, wire P = mode P)."""
    ops = []
    for P in range(n_modes):
        mats = [_Z] * P + [_LOWER] + [_I2] * (n_modes - P - 1)
        ops.append(_kron_all(mats))
    return ops


def spin_orbital_integrals(h1: np.ndarray, h2: np.ndarray):
    """Expand spatial integrals to interleaved spin orbitals.

    Returns (hP[P,Q], gP[P,Q,R,S]) with hP = h_pq delta(sP,sQ) and
    gP = (p s|q r) delta(sP,sS) delta(sQ,sR)."""
    n_orb = h1.shape[0]
    M = 2 * n_orb
    hP = np.zeros((M, M))
    gP = np.zeros((M, M, M, M))
    for P in range(M):
        for Q in range(M):
            if P % 2 == Q % 2:
                hP[P, Q] = h1[P // 2, Q // 2]
    for P in range(M):
        for Q in range(M):
            for R in range(M):
                for S in range(M):
                    if P % 2 == S % 2 and Q % 2 == R % 2:
                        gP[P, Q, R, S] = h2[P // 2, S // 2, Q // 2, R // 2]
    return hP, gP


def dense_hamiltonian(h1: np.ndarray, h2: np.ndarray, e_core: float = 0.0) -> np.ndarray:
    """Eq. (3) as a dense 2^n x 2^n matrix, n = 2 * n_orb."""
    hP, gP = spin_orbital_integrals(h1, h2)
    M = hP.shape[0]
    a = annihilators(M)
    ad = [x.conj().T for x in a]
    H = e_core * np.eye(1 << M, dtype=np.complex128)
    for P in range(M):
        for Q in range(M):
            if hP[P, Q] != 0.0:
                H += hP[P, Q] * (ad[P] @ a[Q])
    for P in range(M):
        for Q in range(M):
            if P == Q:
                continue  # a+_P a+_P = 0
            left = ad[P] @ ad[Q]
            for R in range(M):
                for S in range(M):
                    if R == S or gP[P, Q, R, S] == 0.0:
                        continue
                    H += 0.5 * gP[P, Q, R, S] * (left @ (a[R] @ a[S]))
    return H


def pauli_decompose(H: np.ndarray, tol: float = 1e-14):
    """Pauli coefficients of a dense Hermitian matrix by traces.

    With P(x, z)|b> = i^{|x&z|} (-1)^{|z&b|} |b^x>, the coefficient is
    c(x, z) = i^{-|x&z|} / 2^n * sum_b (-1)^{|z&b|} H[b^x, b]; the sum over b
    for all z at once is a Walsh-Hadamard transform of the x-th shifted
    diagonal.  Returns (xmask[T], zmask[T], coeff[T]) sorted by (x, z), with
    |c| <= tol dropped; raises if a kept coefficient is not real.
    """
    dim = H.shape[0]
    n = dim.bit_length() - 1
    W = scipy.linalg.hadamard(dim).astype(np.float64)
    b = np.arange(dim, dtype=np.int64)
    xs, zs, cs = [], [], []
    for x in range(dim):
        v = H[b ^ x, b]
        w = W @ v / dim
        for z in np.nonzero(np.abs(w) > tol)[0]:
            ny = bin(x & int(z)).count("1")
            c = w[z] * (1j ** (-ny))
            if abs(c.imag) > 1e-12 * max(1.0, abs(c.real)):
                raise ValueError(f"non-real Pauli coefficient {c} for x={x} z={z}")
            if abs(c.real) > tol:
                xs.append(x)
                zs.append(int(z))
                cs.append(c.real)
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
            np.array(cs, dtype=np.float64), n)


def qubit_hamiltonian(integrals, tol: float = 1e-14):
    """Integrals -> dense H (Eq. 3) -> Pauli sum, as a synth.PauliSum-like tuple."""
    H = dense_hamiltonian(integrals.h1, integrals.h2, integrals.e_core)
    x, z, c, n = pauli_decompose(H, tol)
    return _Sum(n, x, z, c)


class _Sum:
    """Minimal Pauli-sum record with the same fields as synth.PauliSum."""

    def __init__(self, n, x, z, c):
        self.n, self.xmask, self.zmask, self.coeff = n, x, z, c

    @property
    def n_terms(self):
        return int(self.coeff.shape[0])


def number_operator(n_modes: int) -> np.ndarray:
    a = annihilators(n_modes)
    return sum(x.conj().T @ x for x in a)


def sz_operator(n_modes: int) -> np.ndarray:
    a = annihilators(n_modes)
    out = np.zeros((1 << n_modes, 1 << n_modes), dtype=np.complex128)
    for P, x in enumerate(a):
        out += (0.5 if P % 2 == 0 else -0.5) * (x.conj().T @ x)
    return out
