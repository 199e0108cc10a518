"""GPU parity: the HIP path through the C ABI against the oracle, element by element.

Tolerances (from the energy and gradient targets of the hot path): energies
1e-10 Ha absolute, gradients 1e-9, states 1e-12 per amplitude.  Every case
prints its name before touching the device.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import fermion

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E_TOL = 1e-10
G_TOL = 1e-9
S_TOL = 1e-12


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def vqe():
    from paper_2601_09951_amd import vqe as m
    return m


@pytest.fixture(scope="module")
def ctx(vqe):
    c = vqe.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(autouse=True)
def _default_tile(ctx):
    ctx.set_tile(12, 11, 3)  # the library's default tiles
    yield


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda:0").contiguous()


def test_library_is_the_hip_build(vqe):
    from paper_2601_09951_amd import capi
    import os
    L = capi.lib()
    assert os.path.basename(L._name) == "libvqe.so"
    for name in capi.EXPORTED:
        assert hasattr(L, name)


@pytest.mark.parametrize("n,B", [(1, 1), (4, 3), (13, 2), (20, 1)])
def test_prepare_reference(vqe, ctx, n, B):
    _say("prepare", n, B)
    psi = torch.full((B, 1 << n), 7 + 7j, dtype=torch.complex128, device="cuda:0")
    ref = (1 << n) - 1 if n > 1 else 1
    vqe.prepare_reference(ctx, n, B, ref, psi)
    torch.cuda.synchronize()
    host = psi.cpu().numpy()
    want = np.zeros((B, 1 << n), dtype=complex)
    want[:, ref] = 1
    assert np.array_equal(host, want)


GEOMS = [(12, 11, 3), (12, 11, 4), (6, 6, 2), (8, 7, 3)]


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (5, 2), (9, 3), (12, 4)])
def test_apply_ansatz_random_circuits(vqe, ctx, geom, n, seed):
    _say("apply", geom, n, seed)
    ctx.set_tile(*geom)
    spec = synth.random_circuit(n, 50, seed=seed)
    th = synth.uniform_thetas(spec.n_params, 2, seed=seed)
    C = vqe.Circuit.from_spec(ctx, spec)
    psi = torch.empty(2, 1 << n, dtype=torch.complex128, device="cuda:0")
    vqe.prepare_reference(ctx, n, 2, spec.ref_index, psi)
    vqe.apply_ansatz(ctx, C, dev(th), psi)
    torch.cuda.synchronize()
    got = psi.cpu().numpy()
    for b in range(2):
        np.testing.assert_allclose(got[b], oracle.state(spec, th[b]), atol=S_TOL)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("n,T,seed", [(1, 3, 0), (3, 10, 1), (7, 40, 2), (10, 80, 3), (14, 200, 4), (13, 600, 5)])
def test_expect_and_h_psi(vqe, ctx, geom, n, T, seed):
    _say("expect", geom, n, T, seed)
    ctx.set_tile(*geom)
    ham = synth.random_pauli_sum(n, min(T, 4 ** n - 1), seed=seed)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    states = np.stack([synth.random_state(n, seed=seed * 7 + b) for b in range(3)])
    psi = dev(states, torch.complex128)
    e = vqe.expect(ctx, H, psi)
    lam = vqe.apply_hamiltonian(ctx, H, psi)
    torch.cuda.synchronize()
    e = e.cpu().numpy()
    lam = lam.cpu().numpy()
    for b in range(3):
        assert abs(e[b] - oracle.expect(states[b], ham).real) < E_TOL
        np.testing.assert_allclose(lam[b], oracle.apply_hamiltonian(states[b], ham), atol=S_TOL)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("n,seed", [(2, 1), (6, 2), (10, 3), (13, 4)])
def test_energy_grad_random_circuits(vqe, ctx, geom, n, seed):
    _say("energy_grad", geom, n, seed)
    ctx.set_tile(*geom)
    spec = synth.random_circuit(n, 40, seed=seed)
    ham = synth.random_pauli_sum(n, min(30, 4 ** n - 1), seed=seed)
    B = 3
    th = synth.uniform_thetas(spec.n_params, B, seed=seed)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    e0 = vqe.energy(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    e, g, e0 = e.cpu().numpy(), g.cpu().numpy(), e0.cpu().numpy()
    for b in range(B):
        eo, go = oracle.energy_grad(spec, ham, th[b], "adjoint")
        assert abs(e[b] - eo) < E_TOL
        assert abs(e0[b] - eo) < E_TOL
        np.testing.assert_allclose(g[b], go, atol=G_TOL)


@pytest.mark.parametrize("n,k,c,seed", [(10, 8, 2, 1), (12, 9, 4, 2), (13, 12, 4, 3), (14, 10, 4, 4),
                                         (16, 12, 4, 5), (12, 12, 4, 6)])
def test_fused_forward_passes(vqe, ctx, n, k, c, seed):
    """Forward passes of rotation / X / H / CNOT circuits as fused stages
    (CNOT networks folded into data movement), batch of 2, against the oracle."""
    _say("fused", n, k, c, seed)
    ctx.set_tile(k, min(k, 12), c)
    spec = synth.random_rotation_cnot_circuit(n, 120, seed=seed)
    th = synth.uniform_thetas(spec.n_params, 2, seed=seed)
    C = vqe.Circuit.from_spec(ctx, spec)
    passes = vqe.circuit_plan(ctx, C, stages="fused")[0]
    assert int(passes["fstage_count"].sum()) > 0
    psi = torch.empty(2, 1 << n, dtype=torch.complex128, device="cuda:0")
    vqe.prepare_reference(ctx, n, 2, spec.ref_index, psi)
    vqe.apply_ansatz(ctx, C, dev(th), psi)
    torch.cuda.synchronize()
    got = psi.cpu().numpy()
    for b in range(2):
        np.testing.assert_allclose(got[b], oracle.state(spec, th[b]), atol=S_TOL)


@pytest.mark.parametrize("n,kr,c,seed", [(10, 8, 2, 11), (12, 9, 4, 12), (14, 11, 4, 13), (16, 11, 4, 14),
                                          (13, 10, 3, 15)])
def test_fused_adjoint_passes(vqe, ctx, n, kr, c, seed):
    """Energy and adjoint gradient of rotation / X / H / CNOT circuits with
    the adjoint passes as fused stages (per-qubit pair sums and gradient
    coefficients, CNOT networks as data movement), batch of 2, against the
    oracle."""
    _say("fused adjoint", n, kr, c, seed)
    ctx.set_tile(12, kr, c)
    spec = synth.random_rotation_cnot_circuit(n, 120, seed=seed)
    ham = synth.random_pauli_sum(n, 60, seed=seed)
    th = synth.uniform_thetas(spec.n_params, 2, seed=seed)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    passes = vqe.circuit_plan(ctx, C, reverse=True, stages="fused")[0]
    assert int(passes["fstage_count"].sum()) > 0
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for b in range(2):
        eo, go = oracle.energy_grad(spec, ham, th[b], "adjoint")
        assert abs(e[b] - eo) < E_TOL
        np.testing.assert_allclose(g[b], go, atol=G_TOL)


@pytest.mark.parametrize("staged", [2, 1, 0])
@pytest.mark.parametrize("n,k,c", [(14, 8, 3), (16, 12, 4), (17, 11, 4), (15, 13, 5)])
def test_hea_energy_grad_multi_tile(vqe, ctx, n, k, c, staged):
    _say("hea", n, k, c, "staged", staged)
    ctx.set_tile(k, min(k, 12), c)
    ctx.set_staged(staged)
    spec = synth.hea_circuit(n, 2)
    ham = synth.random_pauli_sum(n, 100, seed=n)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    ctx.set_staged(True)
    eo, go = oracle.energy_grad(spec, ham, th[0], "adjoint")
    assert abs(e.item() - eo) < E_TOL
    np.testing.assert_allclose(g.cpu().numpy()[0], go, atol=G_TOL)


@pytest.mark.parametrize("n,kf,kr,c", [(16, 12, 11, 3), (18, 10, 9, 3)])
def test_network_only_first_stage(vqe, ctx, n, kf, kr, c):
    """Passes whose first fused stage holds only a CNOT network (no gates, no
    phases) apply it while the tile is read in; the HEA's window passes have
    such stages, some with X conditioned on bits outside the tile.  The
    state, energy and gradient against the oracle."""
    _say("network-only first stage", n, kf, kr, c)
    ctx.set_tile(kf, kr, c)
    spec = synth.hea_circuit(n, 6)
    ham = synth.random_pauli_sum(n, 80, seed=n + 1)
    th = synth.uniform_thetas(spec.n_params, 1, seed=n + 1)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    folded = 0
    for rev in (False, True):
        passes, _, fst = vqe.circuit_plan(ctx, C, reverse=rev, stages="fused")[:3]
        for p in passes:
            if int(p["fstage_count"]) > 0:
                f0 = fst[int(p["fstage_begin"])]
                folded += int(f0["na"]) == 0 and int(f0["phase_count"]) == 0
    assert folded > 0  # the case exercises the folded tile read
    psi = torch.empty(1, 1 << n, dtype=torch.complex128, device="cuda")
    vqe.prepare_reference(ctx, n, 1, spec.ref_index, psi)
    vqe.apply_ansatz(ctx, C, dev(th), psi)
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    ctx.set_tile(12, 11, 3)
    np.testing.assert_allclose(psi.cpu().numpy()[0], oracle.state(spec, th[0]), atol=S_TOL)
    eo, go = oracle.energy_grad(spec, ham, th[0], "adjoint")
    assert abs(e.item() - eo) < E_TOL
    np.testing.assert_allclose(g.cpu().numpy()[0], go, atol=G_TOL)


def test_batched_per_instance_hamiltonians(vqe, ctx):
    _say("batched hams")
    n, B = 8, 5
    spec = synth.ucc_circuit(8, 2)
    model = synth.smooth_integral_model(4, seed=synth.MASTER_SEED)
    ds = synth.bond_grid(B)
    ints = [model.at(d) for d in ds]
    hams = [vqe.Hamiltonian.from_integrals(ctx, i.h1, i.h2, i.e_core) for i in ints]
    th = synth.uniform_thetas(spec.n_params, B, seed=3) * 0.3
    C = vqe.Circuit.from_spec(ctx, spec)
    e, g = vqe.energy_grad(ctx, C, hams, dev(th))
    torch.cuda.synchronize()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    for b in range(B):
        ho = fermion.qubit_hamiltonian(ints[b])
        eo, go = oracle.energy_grad(spec, ho, th[b], "adjoint")
        assert abs(e[b] - eo) < E_TOL
        np.testing.assert_allclose(g[b], go, atol=G_TOL)
        # alone == in the batch
        e1, g1 = vqe.energy_grad(ctx, C, hams[b], dev(th[b:b + 1]))
        torch.cuda.synchronize()
        assert abs(e1.item() - e[b]) < E_TOL
        np.testing.assert_allclose(g1.cpu().numpy()[0], g[b], atol=G_TOL)


def test_c1_energy_curve_and_gradient_descent(vqe, ctx):
    _say("c1")
    ints = synth.random_integrals(2, seed=synth.MASTER_SEED)
    ham = fermion.qubit_hamiltonian(ints)
    spec = synth.h2_circuit()
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2)
    thetas = synth.theta_grid(100)[:, None]
    e = vqe.energy(ctx, C, H, dev(thetas)).cpu().numpy()
    for j, t in enumerate(thetas[:, 0]):
        assert abs(e[j] - oracle.energy(spec, ham, [t])) < E_TOL
    want, th_o = oracle.vqe_run(spec, ham, [0.0], 50, optimizer="gd", lr=0.2)
    for mode in (0, 1):
        ctx.set_loop_mode(mode)
        th = dev(np.zeros((1, 1)))
        traj = vqe.run(ctx, C, H, th, 50, optimizer="gd", lr=0.2).cpu().numpy()[0]
        np.testing.assert_allclose(traj, want, atol=E_TOL)
        assert abs(th.item() - th_o[0]) < 1e-9
    ctx.set_loop_mode(0)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("n_orb", [2, 4])
def test_batched_pes_adam_trajectories(vqe, ctx, n_orb, mode):
    _say("pes", n_orb, "loop mode", mode)
    ctx.set_loop_mode(mode)
    B, iters = 100, 200 if n_orb == 2 else 60
    model = synth.smooth_integral_model(n_orb, seed=synth.MASTER_SEED)
    ds = synth.bond_grid(B)
    ints = [model.at(d) for d in ds]
    spec = synth.h2_circuit() if n_orb == 2 else synth.ucc_circuit(8, 2)
    C = vqe.Circuit.from_spec(ctx, spec)
    hams = [vqe.Hamiltonian.from_integrals(ctx, i.h1, i.h2, i.e_core) for i in ints]
    th = dev(np.zeros((B, spec.n_params)))
    traj = vqe.run(ctx, C, hams, th, iters).cpu().numpy()
    th_final = th.cpu().numpy()
    ctx.set_loop_mode(0)
    for b in range(0, B, 9 if n_orb == 2 else 33):
        ho = fermion.qubit_hamiltonian(ints[b])
        want, tho = oracle.vqe_run(spec, ho, np.zeros(spec.n_params), iters)
        np.testing.assert_allclose(traj[b], want, atol=E_TOL)
        np.testing.assert_allclose(th_final[b], tho, atol=1e-7)


def test_adam_step_kernel(vqe, ctx):
    _say("adam")
    rng = np.random.default_rng(0)
    B, P = 4, 7
    th, m, v = rng.normal(size=(B, P)), np.zeros((B, P)), np.zeros((B, P))
    T = [dev(a) for a in (th, m, v)]
    for t in range(1, 6):
        g = rng.normal(size=(B, P))
        vqe.adam_step(ctx, T[0], T[1], T[2], dev(g), t)
        for b in range(B):
            oracle.adam_step(th[b], m[b], v[b], g[b], t)
    torch.cuda.synchronize()
    np.testing.assert_allclose(T[0].cpu().numpy(), th, atol=1e-14)


def test_autograd_function(vqe, ctx):
    _say("autograd")
    spec = synth.hea_circuit(6, 2)
    ham = synth.random_pauli_sum(6, 30, seed=5)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th0 = synth.uniform_thetas(spec.n_params, 2, seed=5)
    th = dev(th0).requires_grad_(True)
    e = vqe.VQEEnergy.apply(th, ctx, C, H)
    (e * torch.tensor([1.0, -2.0], dtype=torch.float64, device="cuda:0")).sum().backward()
    g = th.grad.cpu().numpy()
    for b, w in enumerate([1.0, -2.0]):
        _, go = oracle.energy_grad(spec, ham, th0[b])
        np.testing.assert_allclose(g[b], w * go, atol=G_TOL)


def test_errors_do_not_launch(vqe, ctx):
    _say("errors")
    spec = synth.h2_circuit()
    C = vqe.Circuit.from_spec(ctx, spec)
    H8 = vqe.Hamiltonian.from_sum(ctx, synth.random_pauli_sum(8, 5, seed=1))
    with pytest.raises(vqe.VQEError):
        vqe.energy_grad(ctx, C, H8, dev(np.zeros((1, 1))))  # qubit count mismatch
    H4 = vqe.Hamiltonian.from_sum(ctx, synth.random_pauli_sum(4, 5, seed=1))
    ws = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(vqe.VQEError):
        vqe.energy_grad(ctx, C, H4, dev(np.zeros((1, 1))), ws=ws)  # workspace too small
    with pytest.raises(vqe.VQEError):
        vqe.energy(ctx, C, [H4, H4], dev(np.zeros((3, 1))))  # n_hams neither 1 nor B


@pytest.mark.parametrize("n,T,L,iters", [(6, 40, 2, 25), (10, 300, 1, 6), (3, 20, 2, 30), (7, 60, 2, 15),
                                           (8, 80, 2, 12)])
def test_persistent_loop_hamiltonian_forms(vqe, ctx, n, T, L, iters):
    # random strings carry imaginary phases (odd Y count): complex table at n = 3, 6, 7, 8;
    # at n = 10 the diagonal table does not fit LDS and the term form runs; at
    # n = 8 a one-qubit gate has 128 pairs, two per lane of the gate wave
    _say("persistent forms", n, T, L, iters)
    spec = synth.hea_circuit(n, L)
    ham = synth.random_pauli_sum(n, min(T, 4 ** n - 1), seed=n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th0 = synth.uniform_thetas(spec.n_params, 3, seed=n)
    out = {}
    for mode in (0, 1):
        ctx.set_loop_mode(mode)
        th = dev(th0)
        out[mode] = (vqe.run(ctx, C, H, th, iters).cpu().numpy(), th.cpu().numpy())
    ctx.set_loop_mode(0)
    for b in range(3):
        want, tho = oracle.vqe_run(spec, ham, th0[b], iters)
        for mode in (0, 1):
            np.testing.assert_allclose(out[mode][0][b], want, atol=E_TOL)
            np.testing.assert_allclose(out[mode][1][b], tho, atol=1e-7)


@pytest.mark.parametrize("n_orb,zero", [(2, True), (3, False), (4, False)])
def test_family_coefficients_on_device_match_oracle(vqe, ctx, n_orb, zero):
    # Eq. (3) -> Jordan-Wigner as a device sparse product vs the oracle's dense build
    _say("family", n_orb)
    ints = [synth.random_integrals(n_orb, seed=70 + i, zero_odd_parity=zero) for i in range(3)]
    for i, it in enumerate(ints):
        it.e_core = 0.1 * i
    fam = vqe.HamFamily(ctx, n_orb, 3)
    fam.set_integrals(dev(vqe.HamFamily.pack(ints)))
    torch.cuda.synchronize()
    for i, it in enumerate(ints):
        x, z, c = fam.member(i).terms()
        got = {(int(a), int(b)): v for a, b, v in zip(x, z, c) if abs(v) > 1e-14}
        ref = fermion.qubit_hamiltonian(it)
        want = {(int(a), int(b)): v for a, b, v in zip(ref.xmask, ref.zmask, ref.coeff)}
        assert got.keys() == want.keys()
        for k in want:
            assert abs(got[k] - want[k]) < 1e-13
    fam.close()


def test_family_pes_run_matches_oracle(vqe, ctx):
    _say("family pes")
    B, iters = 100, 200
    model = synth.smooth_integral_model(4, seed=synth.MASTER_SEED)
    ints = [model.at(float(d)) for d in synth.bond_grid(B)]
    spec = synth.ucc_circuit(8, 2)
    C = vqe.Circuit.from_spec(ctx, spec)
    fam = vqe.HamFamily(ctx, 4, B)
    fam.set_integrals(dev(vqe.HamFamily.pack(ints)))
    hams = fam.members(B)
    th = dev(np.zeros((B, spec.n_params)))
    traj = vqe.run(ctx, C, hams, th, iters).cpu().numpy()
    # new integrals into the same members: the next call sees them
    ints2 = [model.at(float(d) + 0.05) for d in synth.bond_grid(B)]
    fam.set_integrals(dev(vqe.HamFamily.pack(ints2)))
    th2 = dev(np.zeros((B, spec.n_params)))
    traj2 = vqe.run(ctx, C, hams, th2, 20).cpu().numpy()
    for b in (0, 37, 99):
        want, _ = oracle.vqe_run(spec, fermion.qubit_hamiltonian(ints[b]), np.zeros(spec.n_params), iters)
        np.testing.assert_allclose(traj[b], want, atol=E_TOL)
        want2, _ = oracle.vqe_run(spec, fermion.qubit_hamiltonian(ints2[b]), np.zeros(spec.n_params), 20)
        np.testing.assert_allclose(traj2[b], want2, atol=E_TOL)
    del hams
    fam.close()


@pytest.mark.parametrize("case", ["h2", "ucc", "random6", "hea12"])
def test_parameter_shift_gradient_on_device(vqe, ctx, case):
    # Algorithm 1's gradient on the device equals the oracle's parameter shift and the adjoint
    _say("shift", case)
    if case == "h2":
        ints = synth.random_integrals(2, seed=synth.MASTER_SEED)
        spec, ham = synth.h2_circuit(), fermion.qubit_hamiltonian(ints)
        H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2)
        th = synth.theta_grid(8)[:, None]
    elif case == "ucc":
        ints = synth.smooth_integral_model(4).at(0.9)
        spec, ham = synth.ucc_circuit(8, 2), fermion.qubit_hamiltonian(ints)
        H = vqe.Hamiltonian.from_integrals(ctx, ints.h1, ints.h2, ints.e_core)
        th = synth.uniform_thetas(spec.n_params, 3, seed=4) * 0.4
    elif case == "random6":
        spec, ham = synth.random_circuit(6, 30, seed=8), synth.random_pauli_sum(6, 40, seed=8)
        H = vqe.Hamiltonian.from_sum(ctx, ham)
        th = synth.uniform_thetas(spec.n_params, 2, seed=8)
    else:
        spec, ham = synth.hea_circuit(12, 2), synth.random_pauli_sum(12, 80, seed=12)
        H = vqe.Hamiltonian.from_sum(ctx, ham)
        th = synth.uniform_thetas(spec.n_params, 1, seed=12)
    C = vqe.Circuit.from_spec(ctx, spec)
    e, g = vqe.grad_shift(ctx, C, H, dev(th))
    ea, ga = vqe.energy_grad(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    e, g, ea, ga = e.cpu().numpy(), g.cpu().numpy(), ea.cpu().numpy(), ga.cpu().numpy()
    for b in range(th.shape[0]):
        eo, go = oracle.energy_grad(spec, ham, th[b], "shift")
        assert abs(e[b] - eo) < E_TOL
        np.testing.assert_allclose(g[b], go, atol=G_TOL)
        np.testing.assert_allclose(g[b], ga[b], atol=G_TOL)


def _real_pauli_sum(n, n_groups, seed):
    """X/Z strings only (no Y factor, so every coefficient stays real), with
    exactly n_groups distinct flip masks (the identity group included)."""
    rng = np.random.default_rng(seed)
    flips = [0]
    while len(flips) < n_groups:
        f = int(rng.integers(1, 1 << n))
        if f not in flips:
            flips.append(f)
    xs, zs = [], []
    for f in flips:
        seen = set()
        for _ in range(int(rng.integers(1, 4))):
            z = int(rng.integers(0, 1 << n)) & ~f
            if (f == 0 and z == 0) or z in seen:
                continue
            seen.add(z)
            xs.append(f)
            zs.append(z)
    c = rng.normal(size=len(xs)) / np.sqrt(len(xs))
    return synth.PauliSum(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), c)


@pytest.mark.parametrize("n_groups", [60, 90])
def test_persistent_loop_register_rows(vqe, ctx, n_groups):
    # 8 qubits, a real Hamiltonian and gates of at most 64 pairs: with at most
    # 64 flip groups the loop keeps each amplitude's Hamiltonian row in
    # registers (60: the last block of eight partly padding); with 90 groups
    # the table does not fit and the general persistent loop runs
    _say("register rows", n_groups)
    spec = synth.ucc_circuit(8, 2)
    ham = _real_pauli_sum(8, n_groups, seed=n_groups)
    assert len(set(int(v) for v in ham.xmask)) == n_groups
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th0 = synth.uniform_thetas(spec.n_params, 3, seed=n_groups)
    th = dev(th0)
    iters = 20
    ctx.profile(reset=True)
    ctx.set_profiling(True)  # records which persistent kernel variant ran
    traj = vqe.run(ctx, C, H, th, iters).cpu().numpy()
    ran = set(ctx.profile(reset=True))
    ctx.set_profiling(False)
    # 90 groups: the 8-qubit table (96 x 256 doubles) exceeds the LDS
    want_kernel = ("k_small_fast (real state, register rows)" if n_groups <= 64
                   else "k_small_run (persistent loop)")
    assert want_kernel in ran, ran
    tho_gpu = th.cpu().numpy()
    for b in range(3):
        want, tho = oracle.vqe_run(spec, ham, th0[b], iters)
        np.testing.assert_allclose(traj[b], want, atol=E_TOL)
        np.testing.assert_allclose(tho_gpu[b], tho, atol=1e-7)


@pytest.mark.parametrize("n,n_gates,n_groups,iters,imag", [
    (3, 14, 5, 30, False), (6, 30, 24, 20, False), (7, 30, 40, 15, False),
    (8, 24, 50, 12, False),  # one-qubit gates at 8 qubits: two pair slots per lane
    (6, 30, 0, 20, True),    # strings with odd Y counts: a complex Hamiltonian keeps the complex state
])
def test_persistent_loop_real_state(vqe, ctx, n, n_gates, n_groups, iters, imag):
    # circuits of RY, H, X, CNOT, CZ and the excitations from a random basis
    # state under a real Hamiltonian: the loop runs on real amplitudes
    _say("real state", n, n_gates, n_groups, iters, imag)
    spec = synth.random_circuit(n, n_gates, seed=90 + n, kinds=synth.REAL_KINDS)
    assert set(spec.kinds) <= synth.REAL_KINDS
    assert n < 8 or any(k in ("RY", "H", "X") for k in spec.kinds)
    if imag:
        ham = synth.random_pauli_sum(n, 40, seed=90 + n)
        assert any(bin(int(x) & int(z)).count("1") % 2 for x, z in zip(ham.xmask, ham.zmask))
    else:
        ham = _real_pauli_sum(n, n_groups, seed=90 + n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th0 = synth.uniform_thetas(spec.n_params, 3, seed=90 + n)
    th = dev(th0)
    ctx.profile(reset=True)
    ctx.set_profiling(True)  # records which persistent kernel variant ran
    traj = vqe.run(ctx, C, H, th, iters).cpu().numpy()
    ran = set(ctx.profile(reset=True))
    ctx.set_profiling(False)
    want_kernel = ("k_small_fast (persistent loop, table)" if imag
                   else "k_small_fast (real state, table)")
    assert want_kernel in ran, ran
    tho_gpu = th.cpu().numpy()
    for b in range(3):
        want, tho = oracle.vqe_run(spec, ham, th0[b], iters)
        np.testing.assert_allclose(traj[b], want, atol=E_TOL)
        np.testing.assert_allclose(tho_gpu[b], tho, atol=1e-7)


def test_real_state_loop_equals_complex_loop(vqe, ctx):
    # the 8-qubit scan problem on real amplitudes against the same problem
    # forced onto complex amplitudes by a trailing fixed RZ(0) (an identity
    # of a complex gate kind; the complex loop, or the general one where its
    # tables do not fit): same trajectories up to rounding order
    _say("real vs complex loop")
    B, iters = 8, 60
    model = synth.smooth_integral_model(4, seed=synth.MASTER_SEED)
    ints = [model.at(float(d)) for d in synth.bond_grid(B)]
    spec = synth.ucc_circuit(8, 2)
    spec_c = synth.Circuit(spec.n, list(spec.kinds) + ["RZ"],
                           np.vstack([spec.wires, np.array([[3, -1, -1, -1]], dtype=np.int32)]),
                           np.append(spec.param_idx, np.int32(-1)).astype(np.int32),
                           np.append(spec.fixed_angle, 0.0), spec.n_params, spec.ref_index)
    hams = [vqe.Hamiltonian.from_integrals(ctx, i.h1, i.h2, i.e_core) for i in ints]
    out = {}
    for name, sp in (("real", spec), ("complex", spec_c)):
        C = vqe.Circuit.from_spec(ctx, sp)
        th = dev(np.zeros((B, sp.n_params)))
        ctx.profile(reset=True)
        ctx.set_profiling(True)
        traj = vqe.run(ctx, C, hams, th, iters).cpu().numpy()
        out[name] = (traj, th.cpu().numpy(), set(ctx.profile(reset=True)))
        ctx.set_profiling(False)
    assert "k_small_fast (real state, register rows)" in out["real"][2], out["real"][2]
    assert not any("real state" in k for k in out["complex"][2]), out["complex"][2]  # complex128 amplitudes
    np.testing.assert_allclose(out["real"][0], out["complex"][0], atol=1e-11, rtol=0)
    np.testing.assert_allclose(out["real"][1], out["complex"][1], atol=1e-10, rtol=0)
    want, tho = oracle.vqe_run(spec, fermion.qubit_hamiltonian(ints[3]), np.zeros(spec.n_params), iters)
    np.testing.assert_allclose(out["real"][0][3], want, atol=E_TOL)


@pytest.mark.parametrize("n,tiles,seed", [(14, (12, 11, 3), 81), (15, (9, 9, 3), 82), (16, (12, 11, 3), 83)])
def test_any_weight_pauli_strings(vqe, ctx, n, tiles, seed):
    """Strings of weight up to n (flip groups too wide for any tile run as
    whole-state pair sweeps): energy, adjoint and parameter-shift gradients,
    H psi and per-instance Hamiltonians against the oracle."""
    _say("wide groups", n, tiles, seed)
    ctx.set_tile(*tiles)
    k, c = tiles[1], tiles[2]
    spec = synth.hea_circuit(n, 1)
    hams = [synth.random_pauli_sum(n, 30, seed=seed + b, max_weight=n) for b in range(2)]
    low = (1 << c) - 1
    assert any(bin(int(x) & ~low).count("1") > k - c for x in hams[0].xmask)
    th = synth.uniform_thetas(spec.n_params, 2, seed=seed)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = [vqe.Hamiltonian.from_sum(ctx, h) for h in hams]
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    e0 = vqe.energy(ctx, C, H, dev(th))
    es, gs = vqe.grad_shift(ctx, C, H[0], dev(th[:1]))
    psi = dev(np.stack([oracle.state(spec, th[b]) for b in range(2)]), torch.complex128)
    lam = vqe.apply_hamiltonian(ctx, H, psi)
    torch.cuda.synchronize()
    for b in range(2):
        eo, go = oracle.energy_grad(spec, hams[b], th[b], "adjoint")
        assert abs(e[b].item() - eo) < E_TOL
        assert abs(e0[b].item() - eo) < E_TOL
        np.testing.assert_allclose(g[b].cpu().numpy(), go, atol=G_TOL)
        np.testing.assert_allclose(lam[b].cpu().numpy(), oracle.apply_hamiltonian(psi[b].cpu().numpy(), hams[b]),
                                   atol=S_TOL)
        if b == 0:
            assert abs(es[0].item() - eo) < E_TOL
            np.testing.assert_allclose(gs[0].cpu().numpy(), go, atol=G_TOL)


def test_only_wide_groups(vqe, ctx):
    """A Hamiltonian whose every flip group is too wide for a tile (no tile
    sweep at all): lambda and the energy slot start from zero."""
    n = 14
    _say("only wide groups", n)
    ctx.set_tile(12, 11, 3)
    low = 7
    rng = np.random.Generator(np.random.PCG64(5))
    xs, zs = [], []
    while len(xs) < 6:
        x = int(rng.integers(0, 1 << n))
        if bin(x & ~low).count("1") > 11 - 3 and x not in xs:
            xs.append(x)
            zs.append(int(rng.integers(0, 1 << n)))
    ham = synth.PauliSum(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), rng.normal(size=6))
    spec = synth.hea_circuit(n, 1)
    th = synth.uniform_thetas(spec.n_params, 1, seed=6)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    assert len(vqe.hamiltonian_plan(ctx, H, 1, True)["sweeps"]) == 0
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    e0 = vqe.energy(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    eo, go = oracle.energy_grad(spec, ham, th[0], "adjoint")
    assert abs(e.item() - eo) < E_TOL
    assert abs(e0.item() - eo) < E_TOL
    np.testing.assert_allclose(g.cpu().numpy()[0], go, atol=G_TOL)
