"""Seeded synthetic inputs for the VQE hot path.

This module is shared by the oracle and by the GPU library's tests and
benchmarks.  It draws random numbers and lays out problem descriptions
(integrals, Pauli strings, gate lists, parameter vectors); it contains none
of the method's arithmetic: no Jordan-Wigner mapping, no gate matrices, no
expectation values.  Each side turns these descriptions into numbers with
code of its own.

Conventions shared by every consumer
------------------------------------
* A state on ``n`` qubits has ``2**n`` amplitudes.  Wire ``w`` is bit
  ``n-1-w`` of the amplitude index, so a ket printed as ``|w0 w1 ... >``
  reads as the binary expansion of its index (the Hartree-Fock ket
  ``|1100>`` of the paper's Section 3.3 is index 12 at n = 4).
* Pauli strings are given in symplectic form over amplitude-index bits:
  bit ``b`` of ``xmask`` is set when the string has X or Y on the wire
  that owns bit ``b``; bit ``b`` of ``zmask`` is set for Z or Y.
* Spin orbitals are interleaved: wire ``2p`` is spatial orbital ``p`` with
  spin alpha, wire ``2p+1`` is the same orbital with spin beta (the paper's
  Section 3.3 puts both electrons of the reference state in the lowest
  spatial orbital with opposite spins).
* Two-electron integrals are in chemist notation ``(pq|rs)`` with the
  usual 8-fold permutational symmetry.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Sequence, Tuple

import numpy as np

MASTER_SEED = 20260109

# Gate names understood by both sides.  Wires are listed in the order the
# gate definition uses them.
GATE_ARITY = {
    "RX": 1, "RY": 1, "RZ": 1, "H": 1, "X": 1,
    "CNOT": 2, "CZ": 2,
    "SingleExcitation": 2,
    "DoubleExcitation": 4,
}
PARAMETRIC = {"RX", "RY", "RZ", "SingleExcitation", "DoubleExcitation"}
# kinds whose matrices are real for every angle: from a basis state under a
# real Hamiltonian the state stays real
REAL_KINDS = {"RY", "H", "X", "CNOT", "CZ", "SingleExcitation", "DoubleExcitation"}


# ---------------------------------------------------------------------------
# data containers
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class PauliSum:
    """A real-coefficient Pauli sum on ``n`` qubits (index-bit masks)."""

    n: int
    xmask: np.ndarray  # uint64 [T]
    zmask: np.ndarray  # uint64 [T]
    coeff: np.ndarray  # float64 [T]

    @property
    def n_terms(self) -> int:
        return int(self.coeff.shape[0])

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.xmask, dtype=np.uint64).tobytes())
        h.update(np.ascontiguousarray(self.zmask, dtype=np.uint64).tobytes())
        h.update(np.ascontiguousarray(self.coeff, dtype=np.float64).tobytes())
        return h.hexdigest()[:16]


@dataclasses.dataclass
class Integrals:
    """Spatial-orbital integrals: ``h1[p,q]``, ``h2[p,q,r,s] = (pq|rs)``."""

    h1: np.ndarray
    h2: np.ndarray
    e_core: float = 0.0

    @property
    def n_orb(self) -> int:
        return int(self.h1.shape[0])


@dataclasses.dataclass
class Circuit:
    """An ansatz as a gate list.

    ``kinds[g]`` names gate ``g``; ``wires[g]`` holds its wires, padded
    with -1 to four entries; ``param_idx[g]`` is the index into the
    parameter vector (-1 for a fixed gate) and ``fixed_angle[g]`` the angle
    used when ``param_idx[g] == -1``.  ``ref_index`` is the amplitude index
    of the reference basis state the ansatz is applied to.
    """

    n: int
    kinds: List[str]
    wires: np.ndarray  # int32 [G, 4]
    param_idx: np.ndarray  # int32 [G]
    fixed_angle: np.ndarray  # float64 [G]
    n_params: int
    ref_index: int

    @property
    def n_gates(self) -> int:
        return len(self.kinds)

    def shape_key(self) -> str:
        h = hashlib.sha256()
        h.update(repr((self.n, tuple(self.kinds), self.n_params, self.ref_index)).encode())
        h.update(np.ascontiguousarray(self.wires, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.param_idx, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.fixed_angle, dtype=np.float64).tobytes())
        return h.hexdigest()[:16]


def _circuit(n: int, gates: Sequence[Tuple[str, Sequence[int], int, float]],
             n_params: int, ref_index: int) -> Circuit:
    G = len(gates)
    wires = np.full((G, 4), -1, dtype=np.int32)
    pidx = np.full(G, -1, dtype=np.int32)
    fixed = np.zeros(G, dtype=np.float64)
    kinds = []
    for g, (kind, ws, p, a) in enumerate(gates):
        if kind not in GATE_ARITY or len(ws) != GATE_ARITY[kind]:
            raise ValueError(f"bad gate {kind}{tuple(ws)}")
        kinds.append(kind)
        wires[g, : len(ws)] = ws
        pidx[g] = p
        fixed[g] = a
    return Circuit(n, kinds, wires, pidx, fixed, n_params, ref_index)


def basis_index(n: int, occupied_wires: Sequence[int]) -> int:
    """Amplitude index of the basis ket with ``occupied_wires`` set to 1."""
    idx = 0
    for w in occupied_wires:
        idx |= 1 << (n - 1 - w)
    return idx


def pauli_masks(n: int, ops: Sequence[Tuple[int, str]]) -> Tuple[int, int]:
    """Encode ``[(wire, 'X'|'Y'|'Z'), ...]`` as (xmask, zmask) over index bits."""
    x = z = 0
    for w, p in ops:
        b = 1 << (n - 1 - w)
        if p in "XY":
            x |= b
        if p in "ZY":
            z |= b
    return x, z


def pauli_label(n: int, x: int, z: int) -> str:
    """Printable label, wire 0 first (I/X/Y/Z per wire)."""
    out = []
    for w in range(n):
        b = 1 << (n - 1 - w)
        out.append({(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}[(int(bool(x & b)), int(bool(z & b)))])
    return "".join(out)


# ---------------------------------------------------------------------------
# grids
# ---------------------------------------------------------------------------
def bond_grid(count: int = 100, lo: float = 0.3, hi: float = 3.0) -> np.ndarray:
    """Bond lengths d_i = lo + (hi - lo) i / (count - 1) (angstrom)."""
    i = np.arange(count, dtype=np.float64)
    return lo + (hi - lo) * i / (count - 1)


def theta_grid(count: int = 100) -> np.ndarray:
    """Parameter scan theta_j = -pi + 2 pi j / count, j = 0..count-1."""
    j = np.arange(count, dtype=np.float64)
    return -math.pi + 2.0 * math.pi * j / count


# ---------------------------------------------------------------------------
# integrals
# ---------------------------------------------------------------------------
def _unique_h1(n_orb: int):
    return [(p, q) for p in range(n_orb) for q in range(p, n_orb)]


def _unique_h2(n_orb: int):
    pairs = [(p, q) for p in range(n_orb) for q in range(p + 1)]
    out = []
    for a, (p, q) in enumerate(pairs):
        for b, (r, s) in enumerate(pairs):
            if b <= a:
                out.append((p, q, r, s))
    return out


def _fill_h1(n_orb, entries, values):
    h1 = np.zeros((n_orb, n_orb))
    for (p, q), v in zip(entries, values):
        h1[p, q] = h1[q, p] = v
    return h1


def _fill_h2(n_orb, entries, values):
    h2 = np.zeros((n_orb,) * 4)
    for (p, q, r, s), v in zip(entries, values):
        for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
            h2[a, b, c, d] = v
    return h2


def _odd_parity(idx: Sequence[int]) -> bool:
    # spatial orbital p carries inversion parity (-1)^p; a matrix element
    # whose product of parities is odd vanishes for a centro-symmetric
    # two-orbital molecule such as H2.
    return sum(idx) % 2 == 1


def random_integrals(n_orb: int = 2, seed: int = MASTER_SEED, sigma: float = 0.5,
                     zero_odd_parity: bool = True) -> Integrals:
    """Random real symmetric integrals with 8-fold symmetry, N(0, sigma)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e1 = _unique_h1(n_orb)
    e2 = _unique_h2(n_orb)
    v1 = rng.normal(0.0, sigma, size=len(e1))
    v2 = rng.normal(0.0, sigma, size=len(e2))
    if zero_odd_parity:
        v1 = np.array([0.0 if _odd_parity(e) else v for e, v in zip(e1, v1)])
        v2 = np.array([0.0 if _odd_parity(e) else v for e, v in zip(e2, v2)])
    return Integrals(_fill_h1(n_orb, e1, v1), _fill_h2(n_orb, e2, v2), 0.0)


@dataclasses.dataclass
class SmoothIntegralModel:
    """Integrals that are smooth functions of a bond length ``d``.

    Every unique entry is a sum of three terms A_m phi_m(d); phi_m is a
    Gaussian exp(-(d-mu)^2 / 2w^2) or a Morse-like well
    (1 - exp(-a (d - mu)))^2 - 1, chosen per term by the seed.
    """

    n_orb: int
    e1: list
    e2: list
    kind1: np.ndarray
    par1: np.ndarray  # [n_e1, 3, 4] = A, mu, w, a
    kind2: np.ndarray
    par2: np.ndarray
    zero1: np.ndarray
    zero2: np.ndarray
    nuclear_shift: bool

    def at(self, d: float) -> Integrals:
        def evaluate(kind, par):
            A, mu, w, a = par[..., 0], par[..., 1], par[..., 2], par[..., 3]
            gauss = np.exp(-((d - mu) ** 2) / (2.0 * w * w))
            morse = (1.0 - np.exp(-a * (d - mu))) ** 2 - 1.0
            return np.sum(A * np.where(kind == 0, gauss, morse), axis=-1)

        v1 = np.where(self.zero1, 0.0, evaluate(self.kind1, self.par1))
        v2 = np.where(self.zero2, 0.0, evaluate(self.kind2, self.par2))
        e_core = 0.529177210903 / d if self.nuclear_shift else 0.0
        return Integrals(_fill_h1(self.n_orb, self.e1, v1),
                         _fill_h2(self.n_orb, self.e2, v2), e_core)


def smooth_integral_model(n_orb: int, seed: int = MASTER_SEED, zero_odd_parity=None,
                          nuclear_shift: bool = True) -> SmoothIntegralModel:
    if zero_odd_parity is None:
        zero_odd_parity = n_orb == 2
    rng = np.random.Generator(np.random.PCG64(seed))
    e1 = _unique_h1(n_orb)
    e2 = _unique_h2(n_orb)

    def draw(count):
        kind = rng.integers(0, 2, size=(count, 3))
        A = rng.normal(0.0, 0.5, size=(count, 3))
        mu = rng.uniform(0.5, 2.5, size=(count, 3))
        w = rng.uniform(0.2, 1.0, size=(count, 3))
        a = rng.uniform(0.5, 2.0, size=(count, 3))
        return kind, np.stack([A, mu, w, a], axis=-1)

    k1, p1 = draw(len(e1))
    k2, p2 = draw(len(e2))
    z1 = np.array([zero_odd_parity and _odd_parity(e) for e in e1], dtype=bool)
    z2 = np.array([zero_odd_parity and _odd_parity(e) for e in e2], dtype=bool)
    return SmoothIntegralModel(n_orb, e1, e2, k1, p1, k2, p2, z1, z2, nuclear_shift)


# ---------------------------------------------------------------------------
# random Pauli strings
# ---------------------------------------------------------------------------
def random_pauli_sum(n: int, n_terms: int, seed: int = MASTER_SEED,
                     max_weight: int = 4) -> PauliSum:
    """``n_terms`` distinct non-identity strings of weight <= max_weight.

    Weight w ~ U{1..max_weight}; w distinct wires uniformly; each factor
    uniform in {X, Y, Z}; duplicates are redrawn.  Coefficients are
    N(0, 1) / sqrt(n_terms).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    seen = set()
    xs, zs = [], []
    max_weight = min(max_weight, n)
    while len(xs) < n_terms:
        w = int(rng.integers(1, max_weight + 1))
        wires = rng.choice(n, size=w, replace=False)
        paulis = rng.integers(0, 3, size=w)
        x, z = pauli_masks(n, [(int(q), "XYZ"[int(p)]) for q, p in zip(wires, paulis)])
        if (x, z) in seen:
            continue
        seen.add((x, z))
        xs.append(x)
        zs.append(z)
    coeff = rng.normal(0.0, 1.0, size=n_terms) / math.sqrt(n_terms)
    return PauliSum(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), coeff)


# ---------------------------------------------------------------------------
# circuits
# ---------------------------------------------------------------------------
def h2_circuit() -> Circuit:
    """Hartree-Fock |1100> followed by one DoubleExcitation(theta) on (0,1,2,3)."""
    return _circuit(4, [("DoubleExcitation", (0, 1, 2, 3), 0, 0.0)], 1, basis_index(4, [0, 1]))


def ucc_circuit(n_qubits: int = 8, n_electrons: int = 2) -> Circuit:
    """All spin-conserving single and double excitations from the HF state.

    Occupied wires are 0..n_electrons-1 (interleaved spin orbitals).  All
    doubles (one alpha and one beta electron promoted, or two of equal
    spin) come first, then all singles.
    """
    occ = list(range(n_electrons))
    vir = list(range(n_electrons, n_qubits))
    gates = []
    p = 0
    # doubles: pairs of occupied -> pairs of virtual with the same total spin
    for i in range(len(occ)):
        for j in range(i + 1, len(occ)):
            for a in range(len(vir)):
                for b in range(a + 1, len(vir)):
                    o1, o2, v1, v2 = occ[i], occ[j], vir[a], vir[b]
                    if (o1 + o2) % 2 == (v1 + v2) % 2 and sorted([o1 % 2, o2 % 2]) == sorted([v1 % 2, v2 % 2]):
                        gates.append(("DoubleExcitation", (o1, o2, v1, v2), p, 0.0))
                        p += 1
    for o in occ:
        for v in vir:
            if o % 2 == v % 2:
                gates.append(("SingleExcitation", (o, v), p, 0.0))
                p += 1
    return _circuit(n_qubits, gates, p, basis_index(n_qubits, occ))


def hea_circuit(n: int, layers: int) -> Circuit:
    """Hardware-efficient ansatz from |0...0>.

    Each layer: RY on every wire (parameter 2*n*l + q), RZ on every wire
    (parameter 2*n*l + n + q), then CNOT(q -> q+1) for q = 0..n-2.
    """
    gates = []
    for l in range(layers):
        for q in range(n):
            gates.append(("RY", (q,), 2 * n * l + q, 0.0))
        for q in range(n):
            gates.append(("RZ", (q,), 2 * n * l + n + q, 0.0))
        for q in range(n - 1):
            gates.append(("CNOT", (q, q + 1), -1, 0.0))
    return _circuit(n, gates, 2 * n * layers, 0)


def random_circuit(n: int, n_gates: int, seed: int, kinds=None) -> Circuit:
    """A random mix of every supported gate kind, or of the given kinds (used
    by parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = [k for k in GATE_ARITY if GATE_ARITY[k] <= n and (kinds is None or k in kinds)]
    gates = []
    p = 0
    for _ in range(n_gates):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        ws = tuple(int(w) for w in rng.choice(n, size=GATE_ARITY[kind], replace=False))
        if kind in PARAMETRIC:
            if p > 0 and rng.random() < 0.2:
                gates.append((kind, ws, int(rng.integers(0, p)), 0.0))  # shared parameter
            else:
                gates.append((kind, ws, p, 0.0))
                p += 1
        else:
            gates.append((kind, ws, -1, 0.0))
    ref = int(rng.integers(0, 1 << n))
    return _circuit(n, gates, max(p, 1), ref)


def random_rotation_cnot_circuit(n: int, n_gates: int, seed: int) -> Circuit:
    """A random mix of RX, RY, RZ, H, X and CNOT (the gate set of hardware-
    efficient ansaetze), with some shared parameters."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kinds = ["RX", "RY", "RZ", "H", "X", "CNOT", "CNOT"]
    gates = []
    p = 0
    for _ in range(n_gates):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        ws = tuple(int(w) for w in rng.choice(n, size=GATE_ARITY[kind], replace=False))
        if kind in PARAMETRIC:
            if p > 0 and rng.random() < 0.2:
                gates.append((kind, ws, int(rng.integers(0, p)), 0.0))
            else:
                gates.append((kind, ws, p, 0.0))
                p += 1
        else:
            gates.append((kind, ws, -1, 0.0))
    ref = int(rng.integers(0, 1 << n))
    return _circuit(n, gates, max(p, 1), ref)


def random_graph(n: int, edge_prob: float, seed: int = MASTER_SEED) -> List[Tuple[int, int]]:
    """Erdos-Renyi graph G(n, p) as a list of edges (a, b), a < b, in order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < edge_prob]


def ring_graph(n: int, chords: int = 0, seed: int = MASTER_SEED) -> List[Tuple[int, int]]:
    """A ring on n vertices plus `chords` distinct random chords."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = {(min(q, (q + 1) % n), max(q, (q + 1) % n)) for q in range(n)}
    while len(edges) < n + chords:
        a, b = (int(v) for v in rng.choice(n, size=2, replace=False))
        edges.add((min(a, b), max(a, b)))
    return sorted(edges)


def qaoa_circuit(n: int, edges: Sequence[Tuple[int, int]], layers: int) -> Circuit:
    """QAOA ansatz for MaxCut from |0...0>: H on every wire, then per layer l
    the cost unitary prod_edges exp(-i theta_{2l} Z_a Z_b / 2) as
    CNOT(a, b) RZ(theta_{2l}) on b CNOT(a, b) (one parameter shared by all
    edges), and the mixer RX(theta_{2l+1}) on every wire (shared)."""
    gates = [("H", (q,), -1, 0.0) for q in range(n)]
    for l in range(layers):
        for a, b in edges:
            gates += [("CNOT", (a, b), -1, 0.0), ("RZ", (b,), 2 * l, 0.0), ("CNOT", (a, b), -1, 0.0)]
        for q in range(n):
            gates.append(("RX", (q,), 2 * l + 1, 0.0))
    return _circuit(n, gates, 2 * layers, 0)


def maxcut_hamiltonian(n: int, edges: Sequence[Tuple[int, int]], weights=None) -> PauliSum:
    """sum over edges of w_ab Z_a Z_b (diagonal: one flip group); its minimum
    is -(total weight) + 2 x (weight of the maximum cut)."""
    w = np.ones(len(edges)) if weights is None else np.asarray(weights, dtype=np.float64)
    xs, zs = [], []
    for a, b in edges:
        x, z = pauli_masks(n, [(a, "Z"), (b, "Z")])
        xs.append(x)
        zs.append(z)
    return PauliSum(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), w.copy())


def uniform_thetas(n_params: int, batch: int = 1, seed: int = MASTER_SEED) -> np.ndarray:
    """Parameters U(-pi, pi), shape [batch, n_params]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-math.pi, math.pi, size=(batch, n_params))


def random_state(n: int, seed: int) -> np.ndarray:
    """A normalised random complex128 state (for gate-level tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------
# served request stream
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    """One served evaluation: a state size, an ansatz, a Hamiltonian, parameters.

    Exactly one of ``integrals`` (chemistry models, mapped by the consumer) and
    ``pauli`` (random strings) is set.  ``arrival`` is seconds after the start.
    """

    rid: int
    n: int
    want_grad: bool
    circuit: Circuit
    theta: np.ndarray
    arrival: float
    integrals: Integrals = None
    pauli: PauliSum = None


SERVED_MIX = ((4, 0.40), (8, 0.25), (12, 0.15), (16, 0.10), (20, 0.06), (24, 0.04))


def served_requests(count: int, rate: float, seed: int = MASTER_SEED, mix=SERVED_MIX,
                    hea_layers: int = 4):
    """A Poisson stream of ``count`` requests at ``rate`` per second.

    n drawn from ``mix``; n = 4 and 8 use the smooth integral models at a
    random bond length (HF + DoubleExcitation, HF + all excitations), larger n
    use a hardware-efficient ansatz with ``hea_layers`` layers and T ~ U{15..500}
    random Pauli strings; parameters U(-pi, pi) (zero-centred small angles for
    the chemistry models); energy-only or energy + gradient with probability 1/2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = np.array([m[0] for m in mix])
    ps = np.array([m[1] for m in mix], dtype=float)
    ps = ps / ps.sum()
    models = {4: smooth_integral_model(2, seed=seed), 8: smooth_integral_model(4, seed=seed)}
    circuits = {4: h2_circuit(), 8: ucc_circuit(8, 2)}
    t = 0.0
    out = []
    for rid in range(count):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(ns, p=ps))
        want_grad = bool(rng.random() < 0.5)
        sub = int(rng.integers(0, 2 ** 31))
        if n in models:
            d = float(rng.uniform(0.3, 3.0))
            circ = circuits[n]
            theta = np.random.Generator(np.random.PCG64(sub)).uniform(-0.5, 0.5, size=circ.n_params)
            out.append(Request(rid, n, want_grad, circ, theta, t, integrals=models[n].at(d)))
        else:
            if n not in circuits:
                circuits[n] = hea_circuit(n, hea_layers)
            circ = circuits[n]
            T = int(rng.integers(15, 501))
            ham = random_pauli_sum(n, T, seed=sub)
            theta = uniform_thetas(circ.n_params, 1, seed=sub + 1)[0]
            out.append(Request(rid, n, want_grad, circ, theta, t, pauli=ham))
    return out
