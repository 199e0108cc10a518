"""The library's compiled schedules, executed by the CPU emulator, against the oracle.

Runs without a GPU: a host-only planning context (device -1) compiles the
circuits and Pauli sums exactly as the device path does, and
``kernel_emulator`` executes them with the kernels' index arithmetic.  This
pins the pass/sweep compilers and the kernels' pair and sign logic before
anything runs on the device.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import fermion

from . import kernel_emulator as emu

vqe = pytest.importorskip("paper_2601_09951_amd.vqe")


@pytest.fixture(scope="module")
def ctx():
    c = vqe.Context(-1)
    yield c
    c.close()


GEOMS = [(12, 11, 4), (6, 6, 2), (7, 6, 2), (8, 7, 3)]


def _grad_from_parts(circ, gpart):
    g = np.zeros(circ.n_params)
    pg = 0
    for gate in range(circ.n_gates):
        p = circ.param_idx[gate]
        if p >= 0:
            g[p] += gpart[pg]
            pg += 1
    return g


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("n,seed", [(3, 1), (6, 2), (9, 3), (10, 4)])
def test_forward_and_adjoint_schedules(ctx, geom, n, seed):
    ctx.set_tile(*geom)
    spec = synth.random_circuit(n, 40, seed=seed)
    ham = synth.random_pauli_sum(n, 25, seed=seed)
    th = synth.uniform_thetas(spec.n_params, 1, seed=seed)[0]
    C = vqe.Circuit.from_spec(ctx, spec)
    mats = emu.gate_matrices(spec, th)
    passes, ops = vqe.circuit_plan(ctx, C)
    ref = np.zeros(1 << n, dtype=complex)
    ref[spec.ref_index] = 1
    psi = emu.forward(passes, ops, ref, mats)
    want = oracle.state(spec, th)
    np.testing.assert_allclose(psi, want, atol=1e-13)

    H = vqe.Hamiltonian.from_sum(ctx, ham)
    for for_grad in (False, True):
        plan = vqe.hamiltonian_plan(ctx, H, 1, for_grad)
        e = emu.sweeps(plan, psi)
        assert abs(e - oracle.expect(psi, ham).real) < 1e-12
        lam, e2 = emu.sweeps(plan, psi, hpsi=True)
        np.testing.assert_allclose(lam, oracle.apply_hamiltonian(psi, ham), atol=1e-12)
        assert abs(e2 - e) < 1e-12

    rpasses, rops = vqe.circuit_plan(ctx, C, reverse=True)
    n_pg = int((spec.param_idx >= 0).sum())
    back, _, gpart = emu.reverse(rpasses, rops, psi, oracle.apply_hamiltonian(psi, ham), mats, n_pg)
    np.testing.assert_allclose(back, ref, atol=1e-12)
    _, g_or = oracle.energy_grad(spec, ham, th, "adjoint")
    np.testing.assert_allclose(_grad_from_parts(spec, gpart), g_or, atol=1e-11)


@pytest.mark.parametrize("n,k,c", [(12, 8, 3), (14, 9, 4), (11, 6, 2)])
def test_hea_schedules_multi_tile(ctx, n, k, c):
    ctx.set_tile(k, k, c)
    spec = synth.hea_circuit(n, 2)
    ham = synth.random_pauli_sum(n, 60, seed=n)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n)[0]
    C = vqe.Circuit.from_spec(ctx, spec)
    mats = emu.gate_matrices(spec, th)
    passes, ops = vqe.circuit_plan(ctx, C)
    assert len(passes) > 1
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = 1
    psi = emu.forward(passes, ops, ref, mats)
    np.testing.assert_allclose(psi, oracle.state(spec, th), atol=1e-12)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    plan = vqe.hamiltonian_plan(ctx, H, 1, False)
    assert len(plan["sweeps"]) > 1
    assert abs(emu.sweeps(plan, psi) - oracle.expect(psi, ham).real) < 1e-12
    plan = vqe.hamiltonian_plan(ctx, H, 1, True)
    lam, _ = emu.sweeps(plan, psi, hpsi=True)
    np.testing.assert_allclose(lam, oracle.apply_hamiltonian(psi, ham), atol=1e-12)
    rpasses, rops = vqe.circuit_plan(ctx, C, reverse=True)
    _, _, gpart = emu.reverse(rpasses, rops, psi, lam, mats, spec.n_params)
    _, g_or = oracle.energy_grad(spec, ham, th, "adjoint")
    np.testing.assert_allclose(_grad_from_parts(spec, gpart), g_or, atol=1e-11)


def test_batched_union_plan_per_instance_tables(ctx):
    ctx.set_tile(6, 6, 2)
    n = 8
    hams = [synth.random_pauli_sum(n, 20 + 5 * i, seed=40 + i) for i in range(3)]
    H = [vqe.Hamiltonian.from_sum(ctx, h) for h in hams]
    plan = vqe.hamiltonian_plan(ctx, H, 3, False)
    assert plan["n_inst"] == 3
    for i, h in enumerate(hams):
        psi = synth.random_state(n, seed=i)
        assert abs(emu.sweeps(plan, psi, inst=i) - oracle.expect(psi, h).real) < 1e-12


def test_library_jordan_wigner_matches_oracle(ctx):
    for n_orb, seed, zero in [(2, synth.MASTER_SEED, True), (2, 3, False), (3, 4, False), (4, 5, False)]:
        ints = synth.random_integrals(n_orb, seed=seed, zero_odd_parity=zero)
        ints.e_core = 0.123
        H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2, ints.e_core)
        x, z, c = H.terms()
        ref = fermion.qubit_hamiltonian(ints)
        assert np.array_equal(x, ref.xmask) and np.array_equal(z, ref.zmask)
        np.testing.assert_allclose(c, ref.coeff, atol=1e-13)
    # the H2-like model: 15 terms in 2 flip groups
    ints = synth.random_integrals(2, seed=synth.MASTER_SEED)
    H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2)
    assert H.n_terms == 15 and H.n_groups == 2


def test_library_rejects_bad_input(ctx):
    with pytest.raises(vqe.VQEError):
        vqe.Hamiltonian.from_pauli(ctx, 4, [1 << 5], [0], [1.0])
    with pytest.raises(vqe.VQEError):
        vqe.Hamiltonian.from_pauli(ctx, 4, [1], [0], [float("nan")])
    with pytest.raises(vqe.VQEError):
        vqe.Hamiltonian.from_pauli(ctx, 40, [1], [0], [1.0])
    with pytest.raises(vqe.VQEError):
        vqe.Circuit(ctx, 3, ["RY"], [[5, -1, -1, -1]], [0], n_params=1)
    with pytest.raises(vqe.VQEError):
        vqe.Circuit(ctx, 3, ["CNOT"], [[1, 1, -1, -1]], [-1], n_params=0)
    with pytest.raises(vqe.VQEError):
        vqe.Circuit(ctx, 3, ["CNOT"], [[0, 1, -1, -1]], [0], n_params=1)
    with pytest.raises(vqe.VQEError):
        vqe.Circuit(ctx, 3, [99], [[0, -1, -1, -1]], [-1], n_params=0)
    with pytest.raises(vqe.VQEError):
        vqe.Circuit(ctx, 3, ["RY"], [[0, -1, -1, -1]], [3], n_params=2)
    # device work is refused on a planning context
    spec = synth.h2_circuit()
    C = vqe.Circuit.from_spec(ctx, spec)
    from paper_2601_09951_amd import capi
    rc = capi.lib().vqe_prepare_reference(ctx.handle, 4, 1, 0, None, None)
    assert rc == capi.VQE_EUNSUPPORTED
    del C


def test_workspace_accounts_for_states(ctx):
    ctx.set_tile(12, 11, 4)
    n = 16
    spec = synth.hea_circuit(n, 1)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, synth.random_pauli_sum(n, 10, seed=1))
    state = (1 << n) * 16
    for B in (1, 4):
        w0 = vqe.workspace_bytes(ctx, C, H, B, 0)
        w1 = vqe.workspace_bytes(ctx, C, H, B, 1)
        w2 = vqe.workspace_bytes(ctx, C, H, B, 2)
        assert B * state <= w0 < B * state * 1.2
        assert 2 * B * state <= w1 < 2 * B * state * 1.2
        assert w2 > w1


@pytest.mark.parametrize("kind,n,k,c", [("random", 9, 8, 3), ("random", 10, 9, 4), ("hea", 12, 8, 3),
                                         ("hea", 13, 12, 4), ("ucc", 8, 8, 3), ("random", 12, 12, 4)])
def test_register_stage_schedules(ctx, kind, n, k, c):
    ctx.set_tile(k, min(k, 12), c)
    spec = {"random": lambda: synth.random_circuit(n, 60, seed=n),
            "hea": lambda: synth.hea_circuit(n, 2),
            "ucc": lambda: synth.ucc_circuit(8, 2)}[kind]()
    ham = synth.random_pauli_sum(n, 30, seed=n)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n)[0]
    C = vqe.Circuit.from_spec(ctx, spec)
    mats = emu.gate_matrices(spec, th)
    passes, ops, stages, sops = vqe.circuit_plan(ctx, C, stages=True)
    assert len(stages) > 0 and int(passes["stage_count"].sum()) == len(stages)
    assert len(sops) == len(ops)
    ref = np.zeros(1 << n, dtype=complex)
    ref[spec.ref_index] = 1
    psi = emu.forward_staged(passes, stages, sops, ref, mats)
    np.testing.assert_allclose(psi, oracle.state(spec, th), atol=1e-12)
    rp, rops, rst, rsops = vqe.circuit_plan(ctx, C, reverse=True, stages=True)
    n_pg = int((spec.param_idx >= 0).sum())
    back, _, gpart = emu.reverse_staged(rp, rst, rsops, psi, oracle.apply_hamiltonian(psi, ham), mats, n_pg)
    np.testing.assert_allclose(back, ref, atol=1e-12)
    _, g_or = oracle.energy_grad(spec, ham, th, "adjoint")
    np.testing.assert_allclose(_grad_from_parts(spec, gpart), g_or, atol=1e-11)


def _fused_spec(kind, n, k):
    if kind == "hea":
        return synth.hea_circuit(n, 2)
    if kind == "qaoa":
        return synth.qaoa_circuit(n, synth.ring_graph(n, n // 2, seed=n), 2)
    return synth.random_rotation_cnot_circuit(n, 90, seed=n + k)


@pytest.mark.parametrize("kind,n,k,c", [("hea", 12, 8, 3), ("hea", 13, 12, 4), ("hea", 14, 11, 4),
                                         ("rot", 10, 8, 2), ("rot", 12, 9, 4), ("rot", 13, 12, 4),
                                         ("rot", 14, 10, 4), ("qaoa", 12, 9, 3), ("qaoa", 14, 12, 3)])
def test_fused_stage_schedules(ctx, kind, n, k, c):
    """Fused forward stages (one 2x2 per qubit, CNOT / X folded into the
    store map) executed on the CPU reproduce the oracle's state."""
    ctx.set_tile(k, min(k, 12), c)
    spec = _fused_spec(kind, n, k)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n)[0]
    C = vqe.Circuit.from_spec(ctx, spec)
    mats = emu.gate_matrices(spec, th)
    passes, ops, fst, fco, soff, sg, si, fph = vqe.circuit_plan(ctx, C, stages="fused")
    assert int(passes["fstage_count"].sum()) == len(fst) > 0
    if kind == "hea":
        assert (passes["fstage_count"] > 0).all()
    ref = np.zeros(1 << n, dtype=complex)
    ref[spec.ref_index] = 1
    if kind == "qaoa":  # the RZ between a CNOT pair becomes a parity phase
        assert len(fph) > 0
    psi = emu.forward_fused(passes, ops, fst, fco, soff, sg, ref, mats, fph)
    np.testing.assert_allclose(psi, oracle.state(spec, th), atol=1e-12)


@pytest.mark.parametrize("kind,n,k,c", [("hea", 12, 8, 3), ("hea", 13, 11, 4), ("rot", 10, 8, 2),
                                         ("rot", 12, 9, 4), ("rot", 13, 11, 4), ("qaoa", 12, 9, 3),
                                         ("qaoa", 13, 11, 3)])
def test_fused_adjoint_schedules(ctx, kind, n, k, c):
    """Fused adjoint stages on the CPU: the reverse sweep returns to the
    reference state and its gradient equals the oracle's."""
    ctx.set_tile(k, k, c)
    spec = _fused_spec(kind, n, k)
    ham = synth.random_pauli_sum(n, 30, seed=n)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n)[0]
    C = vqe.Circuit.from_spec(ctx, spec)
    mats = emu.gate_matrices(spec, th)
    rp, rops, fst, fco, soff, sg, si, fph = vqe.circuit_plan(ctx, C, reverse=True, stages="fused")
    if kind == "qaoa":
        assert len(fph) > 0 and (fph["info"] >= 16).any()
    assert len(fst) > 0 and (fst["nb"] == 3).all()
    psi = oracle.state(spec, th)
    n_pg = int((spec.param_idx >= 0).sum())
    ref = np.zeros(1 << n, dtype=complex)
    ref[spec.ref_index] = 1
    _, g_or = oracle.energy_grad(spec, ham, th, "adjoint")
    for method in ("gates", "coef"):
        back, _, gpart = emu.reverse_fused(rp, rops, fst, fco, soff, sg, si, psi,
                                           oracle.apply_hamiltonian(psi, ham), mats, n_pg, method=method,
                                           phases=fph)
        np.testing.assert_allclose(back, ref, atol=1e-12)
        np.testing.assert_allclose(_grad_from_parts(spec, gpart), g_or, atol=1e-11)


def test_fused_adjoint_tile_limit(ctx):
    """Adjoint fused stages hold one 8-amplitude sub-cube per thread of a
    256-thread workgroup, so 12-bit reverse tiles take the staged path while
    the forward plan (16-amplitude sub-cubes) still fuses."""
    ctx.set_tile(12, 12, 4)
    spec = synth.hea_circuit(14, 2)
    C = vqe.Circuit.from_spec(ctx, spec)
    fwd = vqe.circuit_plan(ctx, C, stages="fused")[0]
    rev = vqe.circuit_plan(ctx, C, reverse=True, stages="fused")[0]
    assert int(fwd["fstage_count"].sum()) > 0
    assert int(rev["fstage_count"].sum()) == 0
    assert (rev["stage_count"] > 0).any()


@pytest.mark.parametrize("n,k,c,seed", [(12, 8, 3, 71), (13, 9, 2, 72), (10, 6, 2, 73)])
def test_wide_flip_groups(ctx, n, k, c, seed):
    """Strings of any weight: groups with more than k - c flip bits outside
    the low c bits pair over the whole state (wide groups); the schedule's
    energy and H psi still equal the oracle's."""
    ctx.set_tile(k, k, c)
    ham = synth.random_pauli_sum(n, 40, seed=seed, max_weight=n)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    psi = synth.random_state(n, seed=seed)
    low = (1 << c) - 1
    n_wide = len({int(x) for x in ham.xmask if bin(int(x) & ~low).count("1") > k - c})
    assert n_wide > 0
    for for_grad in (False, True):
        plan = vqe.hamiltonian_plan(ctx, H, 1, for_grad)
        assert len(plan["wide"]) == n_wide
        assert all(bin(int(w["f"]) & ~low).count("1") > k - c for w in plan["wide"])
        assert abs(emu.sweeps(plan, psi) - oracle.expect(psi, ham).real) < 1e-12
        lam, e2 = emu.sweeps(plan, psi, hpsi=True)
        np.testing.assert_allclose(lam, oracle.apply_hamiltonian(psi, ham), atol=1e-12)
    # only wide groups: no tile sweep at all
    wide_idx = [i for i, x in enumerate(ham.xmask) if bin(int(x) & ~low).count("1") > k - c]
    only = synth.PauliSum(n, ham.xmask[wide_idx], ham.zmask[wide_idx], ham.coeff[wide_idx])
    plan = vqe.hamiltonian_plan(ctx, vqe.Hamiltonian.from_sum(ctx, only), 1, True)
    assert len(plan["sweeps"]) == 0 and len(plan["wide"]) == n_wide
    lam, _ = emu.sweeps(plan, psi, hpsi=True)
    np.testing.assert_allclose(lam, oracle.apply_hamiltonian(psi, only), atol=1e-12)
