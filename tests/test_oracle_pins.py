"""Pins of the oracle against facts that do not come from the oracle itself.

Every check here builds its expectation from mathematics, textbook closed
forms or brute force written in this file (dense Pauli matrices from
Kronecker products, matrix exponentials of generators, Slater rules,
fermionic sign counting over occupation bit-strings), never by calling the
oracle twice.  They are chosen so that a plausible slip in the oracle (a
dropped term, a wrong sign, a transposed wire order, a mis-read integral
index) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from oracle import fermion
from .qaoa_closed_form import qaoa1_zz_closed_form

I2 = np.eye(2, dtype=complex)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]], dtype=complex)
Z = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def kron_all(mats):
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(out, m)
    return out


def pauli_matrix(n, x, z):
    """Dense Pauli string from its per-wire letters (wire 0 = leftmost factor)."""
    return kron_all([PAULI[ch] for ch in synth.pauli_label(n, int(x), int(z))])


def pauli_sum_matrix(ham):
    n = ham.n
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for x, z, c in zip(ham.xmask, ham.zmask, ham.coeff):
        H += c * pauli_matrix(n, x, z)
    return H


def embed(n, wires, U):
    """Embed a k-qubit matrix acting on ``wires`` (first wire = most significant)."""
    k = len(wires)
    dim = 1 << n
    out = np.zeros((dim, dim), dtype=complex)
    rest = [w for w in range(n) if w not in wires]
    for b in range(dim):
        bits = [(b >> (n - 1 - w)) & 1 for w in range(n)]
        col_local = sum(bits[w] << (k - 1 - j) for j, w in enumerate(wires))
        for row_local in range(1 << k):
            nb = list(bits)
            for j, w in enumerate(wires):
                nb[w] = (row_local >> (k - 1 - j)) & 1
            r = sum(nb[w] << (n - 1 - w) for w in range(n))
            out[r, b] += U[row_local, col_local]
    assert all(True for _ in rest)
    return out


def ket(n, bits_str):
    v = np.zeros(1 << n, dtype=complex)
    v[int(bits_str, 2)] = 1
    return v


# ---------------------------------------------------------------------------
# generators, defined independently of the gate matrices
# ---------------------------------------------------------------------------
def generator(kind):
    if kind == "RX":
        return X
    if kind == "RY":
        return Y
    if kind == "RZ":
        return Z
    if kind == "SingleExcitation":
        return (np.kron(Y, X) - np.kron(X, Y)) / 2
    if kind == "DoubleExcitation":
        a, b = ket(4, "0011"), ket(4, "1100")
        return -1j * np.outer(a, b.conj()) + 1j * np.outer(b, a.conj())
    raise KeyError(kind)


FIXED = {
    "H": np.array([[1, 1], [1, -1]], dtype=complex) / math.sqrt(2),
    "X": X,
    # CNOT and CZ from their action on basis states: control = first wire
    "CNOT": np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=complex),
    "CZ": np.diag([1, 1, 1, -1]).astype(complex),
}


# ===========================================================================
# Jordan-Wigner construction
# ===========================================================================
@pytest.mark.parametrize("modes", [2, 4, 6])
def test_canonical_anticommutation(modes):
    a = fermion.annihilators(modes)
    Id = np.eye(1 << modes)
    for P in range(modes):
        for Q in range(modes):
            acomm = a[P] @ a[Q].conj().T + a[Q].conj().T @ a[P]
            np.testing.assert_allclose(acomm, Id if P == Q else 0 * Id, atol=1e-15)
            np.testing.assert_allclose(a[P] @ a[Q] + a[Q] @ a[P], 0 * Id, atol=1e-15)


def test_number_operator_is_occupation_of_wire():
    # |1> is occupied: a+_P a_P = (I - Z_P) / 2, so <1100|N|1100> = 2
    n = 4
    a = fermion.annihilators(n)
    for P in range(n):
        nP = a[P].conj().T @ a[P]
        ZP = kron_all([Z if w == P else I2 for w in range(n)])
        np.testing.assert_allclose(nP, (np.eye(16) - ZP) / 2, atol=1e-15)
    N = fermion.number_operator(n)
    hf = ket(4, "1100")
    assert abs(hf.conj() @ N @ hf - 2) < 1e-15


def _second_quantised_bruteforce(h1, h2, e_core):
    """H in the occupation basis by applying operator strings to bit-strings.

    Mode P is bit (M-1-P) of the basis index; a+_P / a_P pick up
    (-1)^(number of occupied modes Q < P).  Written without matrices.
    """
    n_orb = h1.shape[0]
    M = 2 * n_orb
    dim = 1 << M

    def occ(state, P):
        return (state >> (M - 1 - P)) & 1

    def apply(ops, state):
        # ops applied right-to-left: list of (P, dagger)
        sign = 1
        for P, dag in reversed(ops):
            if occ(state, P) == (1 if dag else 0):
                return 0, None
            parity = sum(occ(state, Q) for Q in range(P)) % 2
            sign *= -1 if parity else 1
            state ^= 1 << (M - 1 - P)
        return sign, state

    H = np.zeros((dim, dim))
    for s in range(dim):
        H[s, s] += e_core
        for P in range(M):
            for Q in range(M):
                if P % 2 != Q % 2:
                    continue
                v = h1[P // 2, Q // 2]
                sg, t = apply([(P, True), (Q, False)], s)
                if sg:
                    H[t, s] += v * sg
        for P, Q, R, S in itertools.product(range(M), repeat=4):
            if P % 2 != S % 2 or Q % 2 != R % 2:
                continue
            v = h2[P // 2, S // 2, Q // 2, R // 2]
            if v == 0.0:
                continue
            sg, t = apply([(P, True), (Q, True), (R, False), (S, False)], s)
            if sg:
                H[t, s] += 0.5 * v * sg
    return H


@pytest.mark.parametrize("n_orb,seed", [(2, 1), (3, 2)])
def test_dense_hamiltonian_matches_occupation_bruteforce(n_orb, seed):
    ints = synth.random_integrals(n_orb, seed=seed, zero_odd_parity=False)
    ints.e_core = 0.37
    H = fermion.dense_hamiltonian(ints.h1, ints.h2, ints.e_core)
    Hb = _second_quantised_bruteforce(ints.h1, ints.h2, ints.e_core)
    np.testing.assert_allclose(H, Hb, atol=1e-13)


def test_slater_rule_determinant_energies():
    # Textbook diagonal elements (Szabo-Ostlund): opposite spins in p, q
    # give h_pp + h_qq + J_pq; equal spins give h_pp + h_qq + J_pq - K_pq;
    # both spins in p give 2 h_pp + J_pp, with J_pq = (pp|qq), K_pq = (pq|qp).
    ints = synth.random_integrals(3, seed=11, zero_odd_parity=False)
    h, g = ints.h1, ints.h2
    H = fermion.dense_hamiltonian(h, g)
    n = 6

    def det(*wires):
        return synth.basis_index(n, wires)

    for p, q in [(0, 1), (0, 2), (1, 2)]:
        J = g[p, p, q, q]
        K = g[p, q, q, p]
        i = det(2 * p, 2 * q + 1)  # alpha in p, beta in q
        assert abs(H[i, i] - (h[p, p] + h[q, q] + J)) < 1e-13
        i = det(2 * p, 2 * q)  # alpha in p, alpha in q
        assert abs(H[i, i] - (h[p, p] + h[q, q] + J - K)) < 1e-13
    for p in range(3):
        i = det(2 * p, 2 * p + 1)
        assert abs(H[i, i] - (2 * h[p, p] + g[p, p, p, p])) < 1e-13


def test_quadratic_hamiltonian_spectrum_is_sums_of_orbital_energies():
    ints = synth.random_integrals(3, seed=5, zero_odd_parity=False)
    h = ints.h1
    H = fermion.dense_hamiltonian(h, np.zeros_like(ints.h2))
    eps = np.linalg.eigvalsh(h)
    spin_orb = np.concatenate([eps, eps])
    expected = sorted(sum(c) for k in range(7) for c in itertools.combinations(spin_orb, k))
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(H)), expected, atol=1e-12)


@pytest.mark.parametrize("n_orb,seed,zero", [(2, synth.MASTER_SEED, True), (2, 7, False), (3, 3, False)])
def test_pauli_decomposition_reconstructs_and_conserves(n_orb, seed, zero):
    ints = synth.random_integrals(n_orb, seed=seed, zero_odd_parity=zero)
    ints.e_core = -0.25
    Hd = fermion.dense_hamiltonian(ints.h1, ints.h2, ints.e_core)
    ham = fermion.qubit_hamiltonian(ints)
    Hp = pauli_sum_matrix(ham)
    np.testing.assert_allclose(Hp, Hd, atol=1e-13)
    np.testing.assert_allclose(Hp, Hp.conj().T, atol=1e-14)
    N = fermion.number_operator(2 * n_orb)
    Sz = fermion.sz_operator(2 * n_orb)
    np.testing.assert_allclose(Hp @ N - N @ Hp, 0, atol=1e-12)
    np.testing.assert_allclose(Hp @ Sz - Sz @ Hp, 0, atol=1e-12)


def test_h2_like_hamiltonian_has_fifteen_terms_in_two_flip_groups():
    ham = fermion.qubit_hamiltonian(synth.random_integrals(2, seed=synth.MASTER_SEED))
    assert ham.n_terms == 15
    labels = sorted(synth.pauli_label(4, int(x), int(z)) for x, z in zip(ham.xmask, ham.zmask))
    z_only = [l for l in labels if set(l) <= set("IZ")]
    assert len(z_only) == 11
    assert sum(1 for l in z_only if l.count("Z") == 1) == 4
    assert sum(1 for l in z_only if l.count("Z") == 2) == 6
    flips = {int(x) for x in ham.xmask}
    assert flips == {0, 0b1111}
    # with the odd-parity entries present the count grows (single-excitation strings)
    ham2 = fermion.qubit_hamiltonian(synth.random_integrals(2, seed=7, zero_odd_parity=False))
    assert ham2.n_terms > 15


# ===========================================================================
# gates
# ===========================================================================
@pytest.mark.parametrize("kind", ["RX", "RY", "RZ", "SingleExcitation", "DoubleExcitation"])
def test_parametric_gate_equals_exponential_of_generator(kind):
    n = 5
    rng = np.random.default_rng(3)
    k = synth.GATE_ARITY[kind]
    G = generator(kind)
    for trial in range(6):
        wires = [int(w) for w in rng.choice(n, size=k, replace=False)]
        a = float(rng.uniform(-4, 4))
        U = scipy.linalg.expm(-0.5j * a * G)
        psi = synth.random_state(n, seed=100 + trial)
        want = embed(n, wires, U) @ psi
        got = oracle.apply_gate(psi, kind, wires, a)
        np.testing.assert_allclose(got, want, atol=1e-13)
        back = oracle.apply_gate(got, kind, wires, a, adjoint=True)
        np.testing.assert_allclose(back, psi, atol=1e-13)
        # the generator the adjoint uses
        np.testing.assert_allclose(oracle.apply_generator(psi, kind, wires), embed(n, wires, G) @ psi, atol=1e-13)


@pytest.mark.parametrize("kind", ["H", "X", "CNOT", "CZ"])
def test_fixed_gates(kind):
    n = 4
    rng = np.random.default_rng(9)
    k = synth.GATE_ARITY[kind]
    for trial in range(5):
        wires = [int(w) for w in rng.choice(n, size=k, replace=False)]
        psi = synth.random_state(n, seed=200 + trial)
        np.testing.assert_allclose(oracle.apply_gate(psi, kind, wires), embed(n, wires, FIXED[kind]) @ psi,
                                   atol=1e-14)


def test_cnot_ladder_is_a_bit_exact_permutation():
    # CNOT(q -> q+1) for q = 0..n-2 on a basis state maps bit-strings to
    # their prefix XOR (wire order): a permutation, no arithmetic.
    n = 6
    for b in range(1 << n):
        bits = [(b >> (n - 1 - w)) & 1 for w in range(n)]
        psi = np.zeros(1 << n, dtype=complex)
        psi[b] = 1
        for q in range(n - 1):
            psi = oracle.apply_gate(psi, "CNOT", [q, q + 1])
        out = list(itertools.accumulate(bits, lambda u, v: u ^ v))
        idx = sum(v << (n - 1 - w) for w, v in enumerate(out))
        assert psi[idx] == 1 and np.count_nonzero(psi) == 1


def test_wire_zero_is_most_significant_bit():
    # <HF|Z_w|HF> = -1 on the occupied wires 0, 1 of |1100>, +1 on 2, 3
    psi = oracle.prepare(4, synth.basis_index(4, [0, 1]))
    assert synth.basis_index(4, [0, 1]) == 12
    for w, want in zip(range(4), [-1, -1, 1, 1]):
        x, z = synth.pauli_masks(4, [(w, "Z")])
        assert oracle.expect_pauli(psi, x, z) == want
    # RY(pi) on wire 0 flips the most significant bit
    psi = oracle.apply_gate(oracle.prepare(3, 0), "RY", [0], math.pi)
    assert abs(abs(psi[4]) - 1) < 1e-15


# ===========================================================================
# energies
# ===========================================================================
def test_pauli_phase_convention():
    # Y|0> = i|1>: the eigenstate (|0> + i|1>)/sqrt2 has <Y> = +1
    psi = np.array([1, 1j]) / math.sqrt(2)
    x, z = synth.pauli_masks(1, [(0, "Y")])
    assert abs(oracle.expect_pauli(psi, x, z) - 1) < 1e-15
    psi = np.array([1, 1]) / math.sqrt(2)
    x, z = synth.pauli_masks(1, [(0, "X")])
    assert abs(oracle.expect_pauli(psi, x, z) - 1) < 1e-15


def test_bloch_closed_forms_on_product_states():
    # RZ(b) RY(a)|0>: <Z> = cos a, <X> = sin a cos b, <Y> = sin a sin b
    rng = np.random.default_rng(1)
    n = 5
    a = rng.uniform(-3, 3, size=n)
    b = rng.uniform(-3, 3, size=n)
    psi = oracle.prepare(n, 0)
    for q in range(n):
        psi = oracle.apply_gate(psi, "RY", [q], a[q])
        psi = oracle.apply_gate(psi, "RZ", [q], b[q])
    for q in range(n):
        for P, want in (("Z", math.cos(a[q])), ("X", math.sin(a[q]) * math.cos(b[q])),
                        ("Y", math.sin(a[q]) * math.sin(b[q]))):
            x, z = synth.pauli_masks(n, [(q, P)])
            assert abs(oracle.expect_pauli(psi, x, z) - want) < 1e-14
    # two-body correlators of a product state factorise
    x, z = synth.pauli_masks(n, [(0, "X"), (3, "Y")])
    want = math.sin(a[0]) * math.cos(b[0]) * math.sin(a[3]) * math.sin(b[3])
    assert abs(oracle.expect_pauli(psi, x, z) - want) < 1e-14


@pytest.mark.parametrize("n,T,seed", [(3, 20, 1), (6, 60, 2), (8, 120, 3)])
def test_energy_and_h_psi_match_dense(n, T, seed):
    ham = synth.random_pauli_sum(n, T, seed=seed)
    Hd = pauli_sum_matrix(ham)
    for s in range(3):
        psi = synth.random_state(n, seed=seed * 10 + s)
        want = psi.conj() @ Hd @ psi
        got = oracle.expect(psi, ham)
        assert abs(got - want) < 1e-13
        assert abs(got.imag) < 1e-14
        np.testing.assert_allclose(oracle.apply_hamiltonian(psi, ham), Hd @ psi, atol=1e-13)


@pytest.mark.parametrize("n,seed", [(4, 1), (6, 2)])
def test_variational_bound(n, seed):
    # Eq. (2): E(theta) >= E_0 for every theta
    ham = synth.random_pauli_sum(n, 40, seed=seed)
    e0 = np.linalg.eigvalsh(pauli_sum_matrix(ham))[0]
    circ = synth.hea_circuit(n, 2)
    th = synth.uniform_thetas(circ.n_params, 20, seed=seed)
    for t in th:
        assert oracle.energy(circ, ham, t) >= e0 - 1e-12


def _c1_coefficients(ham):
    Hd = pauli_sum_matrix(ham).real
    A, B = 0b1100, 0b0011
    a = (Hd[A, A] + Hd[B, B]) / 2
    b = (Hd[A, A] - Hd[B, B]) / 2
    c = -Hd[A, B]
    return a, b, c, Hd


def test_c1_closed_form_energy_curve_and_sector_ground_state():
    # psi(theta) = cos(t/2)|1100> - sin(t/2)|0011>, so
    # E(t) = a + b cos t + c sin t with a, b, c from the 2x2 block of H.
    ham = fermion.qubit_hamiltonian(synth.random_integrals(2, seed=synth.MASTER_SEED))
    circ = synth.h2_circuit()
    a, b, c, Hd = _c1_coefficients(ham)
    for t in synth.theta_grid(100):
        e, g = oracle.energy_grad(circ, ham, [t], "adjoint")
        assert abs(e - (a + b * math.cos(t) + c * math.sin(t))) < 1e-12
        assert abs(g[0] - (-b * math.sin(t) + c * math.cos(t))) < 1e-12
    # span{|1100>, |0011>} is invariant under H, and its lower eigenvalue is the
    # ground energy of the two-electron S_z = 0 sector restricted to it.
    A, B = 0b1100, 0b0011
    for v in (A, B):
        col = Hd[:, v].copy()
        col[[A, B]] = 0
        assert np.max(np.abs(col)) < 1e-14
    emin = a - math.hypot(b, c)
    block = np.array([[Hd[A, A], Hd[A, B]], [Hd[B, A], Hd[B, B]]])
    assert abs(emin - np.linalg.eigvalsh(block)[0]) < 1e-13
    tstar = math.atan2(-c, -b)
    assert abs(oracle.energy(circ, ham, [tstar]) - emin) < 1e-12


# ===========================================================================
# gradients and the optimiser
# ===========================================================================
@pytest.mark.parametrize("n,seed", [(3, 1), (4, 2), (5, 3), (6, 4)])
def test_adjoint_equals_parameter_shift_on_random_circuits(n, seed):
    circ = synth.random_circuit(n, 25, seed=seed)
    ham = synth.random_pauli_sum(n, 30, seed=seed)
    th = synth.uniform_thetas(circ.n_params, 1, seed=seed)[0]
    e1, g1 = oracle.energy_grad(circ, ham, th, "adjoint")
    e2, g2 = oracle.energy_grad(circ, ham, th, "shift")
    assert abs(e1 - e2) < 1e-13
    np.testing.assert_allclose(g1, g2, atol=1e-11)
    # central finite differences as a sanity check only (truncation ~h^2)
    h = 1e-4
    for p in range(min(circ.n_params, 6)):
        tp, tm = th.copy(), th.copy()
        tp[p] += h
        tm[p] -= h
        fd = (oracle.energy(circ, ham, tp) - oracle.energy(circ, ham, tm)) / (2 * h)
        assert abs(fd - g1[p]) < 1e-6


def test_norm_preserved_and_circuit_reversible():
    n = 7
    circ = synth.random_circuit(n, 60, seed=9)
    th = synth.uniform_thetas(circ.n_params, 1, seed=9)[0]
    psi = oracle.state(circ, th)
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    for g in reversed(range(circ.n_gates)):
        w = [int(v) for v in circ.wires[g] if v >= 0]
        p = circ.param_idx[g]
        a = th[p] if p >= 0 else circ.fixed_angle[g]
        psi = oracle.apply_gate(psi, circ.kinds[g], w, a, adjoint=True)
    ref = np.zeros(1 << n, dtype=complex)
    ref[circ.ref_index] = 1
    np.testing.assert_allclose(psi, ref, atol=1e-12)


def test_adam_constant_gradient_closed_form():
    # With a constant gradient g, bias correction gives m_hat = g and
    # v_hat = g^2 at every step, so each step moves theta by -lr g/(|g|+eps).
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 8):
        before = theta.copy()
        oracle.adam_step(theta, m, v, g, t, lr=0.01)
        np.testing.assert_allclose(theta - before, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_varying_gradient_hand_computed():
    # Three steps with a gradient that changes sign and size, beta1 != beta2,
    # eps = 0, so that the moment recurrences (and which beta belongs to which
    # moment) decide the result.  Values worked by hand from Kingma and Ba's
    # Algorithm 1 with beta1 = 1/2, beta2 = 3/4, lr = 1/10, g = 1, -2, 3:
    #   t=1: m = 1/2,   v = 1/4,      m^ = 1,    v^ = 1        -> step -1/10
    #   t=2: m = -3/4,  v = 19/16,    m^ = -1,   v^ = 19/7     -> step +(1/10) sqrt(7/19)
    #   t=3: m = 9/8,   v = 201/64,   m^ = 9/7,  v^ = 201/37   -> step -(1/10)(9/7) sqrt(37/201)
    # With the betas swapped, step 2 would be +(1/10)(5/7)/sqrt(3) instead.
    want_steps = [-0.1, 0.1 * math.sqrt(7 / 19), -0.1 * (9 / 7) * math.sqrt(37 / 201)]
    want_m = [0.5, -0.75, 1.125]
    want_v = [0.25, 19 / 16, 201 / 64]
    theta, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t, g in enumerate([1.0, -2.0, 3.0], start=1):
        before = theta.copy()
        oracle.adam_step(theta, m, v, np.array([g]), t, lr=0.1, b1=0.5, b2=0.75, eps=0.0)
        assert abs((theta - before)[0] - want_steps[t - 1]) < 1e-15
        assert abs(m[0] - want_m[t - 1]) < 1e-15 and abs(v[0] - want_v[t - 1]) < 1e-15
    assert abs(theta[0] - sum(want_steps)) < 1e-15


def test_vqe_gd_loop_follows_closed_form_derivative():
    # Gradient descent driven by the closed-form derivative of the C1 curve.
    ham = fermion.qubit_hamiltonian(synth.random_integrals(2, seed=synth.MASTER_SEED))
    circ = synth.h2_circuit()
    a, b, c, _ = _c1_coefficients(ham)
    eta, iters = 0.2, 50
    t = 0.0
    want = []
    for _ in range(iters):
        want.append(a + b * math.cos(t) + c * math.sin(t))
        t -= eta * (-b * math.sin(t) + c * math.cos(t))
    want.append(a + b * math.cos(t) + c * math.sin(t))
    got, th = oracle.vqe_run(circ, ham, [0.0], iters, optimizer="gd", lr=eta)
    np.testing.assert_allclose(got, want, atol=1e-12)
    assert abs(th[0] - t) < 1e-11
    # and converges to the closed-form minimum
    assert abs(got[-1] - (a - math.hypot(b, c))) < 1e-6


def test_vqe_adam_loop_first_step_moves_by_learning_rate():
    ham = fermion.qubit_hamiltonian(synth.random_integrals(2, seed=synth.MASTER_SEED))
    circ = synth.h2_circuit()
    a, b, c, _ = _c1_coefficients(ham)
    e, th = oracle.vqe_run(circ, ham, [0.0], 1, optimizer="adam", lr=0.01)
    g0 = c  # dE/dt at t = 0
    assert abs(th[0] - (-0.01 * g0 / (abs(g0) + 1e-8))) < 1e-15
    assert abs(e[0] - (a + b)) < 1e-12


def test_thread_count_does_not_change_results():
    n = 13
    circ = synth.hea_circuit(n, 1)
    ham = synth.random_pauli_sum(n, 20, seed=4)
    th = synth.uniform_thetas(circ.n_params, 1, seed=4)[0]
    oracle.set_threads(1)
    e1, g1 = oracle.energy_grad(circ, ham, th)
    oracle.set_threads(4)
    try:
        e4, g4 = oracle.energy_grad(circ, ham, th)
    finally:
        oracle.set_threads(1)
    assert abs(e1 - e4) < 1e-12
    np.testing.assert_allclose(g1, g4, atol=1e-12)


@pytest.mark.parametrize("n,prob,seed", [(6, 0.6, 1), (8, 0.4, 2), (9, 0.5, 3)])
def test_qaoa_one_layer_matches_closed_form(n, prob, seed):
    """The QAOA MaxCut ansatz (H, CNOT-RZ-CNOT per edge with one shared angle,
    RX mixer with one shared angle) at one layer: every edge's <Z_u Z_v> and
    the MaxCut energy equal the published closed form; the energy's gradient
    equals central differences of the closed form (shared parameters summed)."""
    edges = synth.random_graph(n, prob, seed=seed)
    assert len(edges) >= 3
    circ = synth.qaoa_circuit(n, edges, 1)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        t = rng.uniform(-math.pi, math.pi, size=2)
        for (u, v) in edges:
            ham = synth.maxcut_hamiltonian(n, [(u, v)])
            got = oracle.energy(circ, ham, t)
            assert abs(got - qaoa1_zz_closed_form(edges, n, u, v, t[0], t[1])) < 1e-12
        ham = synth.maxcut_hamiltonian(n, edges)

        def closed(tc, tm):
            return sum(qaoa1_zz_closed_form(edges, n, a, b, tc, tm) for a, b in edges)

        e, g = oracle.energy_grad(circ, ham, t)
        assert abs(e - closed(*t)) < 1e-12
        h = 1e-5
        fd = [(closed(t[0] + h, t[1]) - closed(t[0] - h, t[1])) / (2 * h),
              (closed(t[0], t[1] + h) - closed(t[0], t[1] - h)) / (2 * h)]
        np.testing.assert_allclose(g, fd, atol=1e-8)
