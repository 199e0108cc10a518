"""Launch graphs, batch tiles and the autotuner against the oracle.

Graph replay: a launch sequence captured on its second identical call and
replayed afterwards gives the same energies and gradients as the eager
sequence, with the parameters and the Hamiltonian coefficients changed by
content between replays (the graph reads them from the same buffers), and
with eager work and synchronisations between the replays.  Batch tiles: a
batch run as ragged chunks equals the oracle per instance.  The autotuner's
choice evaluates to the oracle's energy and gradient.  Tolerances: energies
1e-10, gradients 1e-9, Adam trajectories 1e-7 (theta) / 1e-10 (energies).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import fermion

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E_TOL = 1e-10
G_TOL = 1e-9


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
def _defaults(ctx):
    ctx.set_tile(12, 11, 3)
    ctx.set_graphs(True)
    ctx.set_loop_mode(0)
    ctx.clear_tuning()
    yield


def test_energy_grad_graph_replays_match_eager(vqe, ctx):
    n = 14
    spec = synth.hea_circuit(n, 2)
    ham = synth.random_pauli_sum(n, 60, seed=7)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    B = 3
    th = torch.empty(B, spec.n_params, dtype=torch.float64, device="cuda:0")
    ws = vqe.workspace(ctx, C, H, B, 1)
    e = torch.empty(B, dtype=torch.float64, device="cuda:0")
    g = torch.empty(B, spec.n_params, dtype=torch.float64, device="cuda:0")
    before = ctx.graph_stats()
    for rep in range(5):
        _say(f"graph replay {rep}, n = {n}, batch {B}")
        thetas = synth.uniform_thetas(spec.n_params, B, seed=300 + rep)
        th.copy_(torch.from_numpy(thetas))  # new content, same buffer
        vqe.energy_grad(ctx, C, H, th, ws=ws, out_e=e, out_g=g)
        torch.cuda.synchronize()
        got_e, got_g = e.cpu().numpy().copy(), g.cpu().numpy().copy()
        # eager work between the replays: the same evaluation with other buffers
        e2, g2 = vqe.energy_grad(ctx, C, H, th.clone())
        torch.cuda.synchronize()
        assert np.max(np.abs(got_e - e2.cpu().numpy())) <= 1e-12
        assert np.max(np.abs(got_g - g2.cpu().numpy())) <= 1e-12
        for b in range(B) if rep in (0, 4) else ():
            eo, go = oracle.energy_grad(spec, ham, thetas[b], "adjoint")
            assert abs(got_e[b] - eo) < E_TOL
            assert np.max(np.abs(got_g[b] - go)) < G_TOL
    after = ctx.graph_stats()
    assert after["captures"] >= before["captures"] + 1
    assert after["launches"] >= before["launches"] + 4


def test_energy_graph_sees_new_family_coefficients(vqe, ctx):
    """Family members' weights are refreshed inside the graph: new integrals
    between replays give the new energies."""
    model = synth.smooth_integral_model(4, seed=synth.MASTER_SEED)
    ds = synth.bond_grid(6)
    spec = synth.ucc_circuit(8, 2)
    C = vqe.Circuit.from_spec(ctx, spec)
    fam = vqe.HamFamily(ctx, 4, 3)
    hams = fam.members(3)
    thetas = synth.uniform_thetas(spec.n_params, 3, seed=5) * 0.3
    th = torch.tensor(thetas, device="cuda:0")
    ws = vqe.workspace(ctx, C, hams, 3, 0)
    e = torch.empty(3, dtype=torch.float64, device="cuda:0")
    for rep in range(4):
        _say(f"family graph replay {rep}")
        ints = [model.at(float(d)) for d in ds[(rep % 2) * 3:(rep % 2) * 3 + 3]]
        fam.set_integrals(torch.tensor(vqe.HamFamily.pack(ints), dtype=torch.float64, device="cuda:0"))
        vqe.energy(ctx, C, hams, th, ws=ws, out=e)
        torch.cuda.synchronize()
        for b in range(3):
            eo = oracle.energy(spec, fermion.qubit_hamiltonian(ints[b]), thetas[b])
            assert abs(e[b].item() - eo) < E_TOL, (rep, b)
    assert ctx.graph_stats()["launches"] >= 2


@pytest.mark.parametrize("graphs", [True, False])
def test_per_step_loop_matches_oracle(vqe, ctx, graphs):
    """vqe_run's per-step loop (one graph per step when graphs are on) against
    the oracle's Adam trajectory."""
    ctx.set_graphs(graphs)
    ctx.set_loop_mode(1)
    n, iters, B = 10, 12, 3
    spec = synth.hea_circuit(n, 2)
    hams_s = [synth.random_pauli_sum(n, 30, seed=40 + b) for b in range(B)]
    C = vqe.Circuit.from_spec(ctx, spec)
    hams = [vqe.Hamiltonian.from_sum(ctx, h) for h in hams_s]
    th0 = synth.uniform_thetas(spec.n_params, B, seed=9)
    th = torch.tensor(th0, device="cuda:0")
    _say(f"per-step loop, graphs {graphs}")
    traj = vqe.run(ctx, C, hams, th, iters).cpu().numpy()
    for b in range(B):
        eo, tho = oracle.vqe_run(spec, hams_s[b], th0[b], iters)
        assert np.max(np.abs(traj[b] - eo)) < E_TOL, b
        assert np.max(np.abs(th[b].cpu().numpy() - tho)) < 1e-7, b


@pytest.mark.parametrize("shared", [True, False])
def test_batch_tiles_match_oracle(vqe, ctx, shared):
    """A batch of 8 run as launch chunks of 3, 3 and 2 instances."""
    n, B = 12, 8
    spec = synth.hea_circuit(n, 2)
    hs = [synth.random_pauli_sum(n, 40, seed=60 + (0 if shared else b)) for b in range(B)]
    C = vqe.Circuit.from_spec(ctx, spec)
    hams = vqe.Hamiltonian.from_sum(ctx, hs[0]) if shared else [vqe.Hamiltonian.from_sum(ctx, h) for h in hs]
    thetas = synth.uniform_thetas(spec.n_params, B, seed=61)
    th = torch.tensor(thetas, device="cuda:0")
    for want in (False, True):
        vqe.tune_set(ctx, C, B, want, k_fwd=10, k_rev=9, c_low=3, batch_tile=3)
    ws1 = vqe.workspace(ctx, C, hams, B, 1)
    ws_tuned = vqe.workspace_bytes(ctx, C, hams, B, 1)
    _say(f"batch tile 3 of {B}, shared H {shared}, workspace {ws1.numel()} B")
    for rep in range(3):  # eager, capture, replay
        e, g = vqe.energy_grad(ctx, C, hams, th, ws=ws1)
        e0 = vqe.energy(ctx, C, hams, th)
        torch.cuda.synchronize()
        for b in range(B) if rep != 1 else ():
            eo, go = oracle.energy_grad(spec, hs[b], thetas[b], "adjoint")
            assert abs(e[b].item() - eo) < E_TOL, (rep, b)
            assert abs(e0[b].item() - eo) < E_TOL, (rep, b)
            assert np.max(np.abs(g[b].cpu().numpy() - go)) < G_TOL, (rep, b)
    ctx.clear_tuning()
    assert vqe.workspace_bytes(ctx, C, hams, B, 1) > ws_tuned  # the chunked workspace holds 3 states, not 8


def test_batch_tiles_in_the_per_step_loop(vqe, ctx):
    ctx.set_loop_mode(1)
    n, B, iters = 9, 5, 8
    spec = synth.hea_circuit(n, 2)
    hs = [synth.random_pauli_sum(n, 25, seed=80 + b) for b in range(B)]
    C = vqe.Circuit.from_spec(ctx, spec)
    hams = [vqe.Hamiltonian.from_sum(ctx, h) for h in hs]
    vqe.tune_set(ctx, C, B, True, k_fwd=8, k_rev=8, c_low=3, batch_tile=2)
    th0 = synth.uniform_thetas(spec.n_params, B, seed=81)
    th = torch.tensor(th0, device="cuda:0")
    _say("per-step loop with batch tile 2 of 5")
    traj = vqe.run(ctx, C, hams, th, iters).cpu().numpy()
    for b in range(B):
        eo, tho = oracle.vqe_run(spec, hs[b], th0[b], iters)
        assert np.max(np.abs(traj[b] - eo)) < E_TOL, b
        assert np.max(np.abs(th[b].cpu().numpy() - tho)) < 1e-7, b


def test_autotune_choice_matches_oracle(vqe, ctx):
    n, B = 12, 4
    spec = synth.hea_circuit(n, 4)
    ham = synth.random_pauli_sum(n, 80, seed=90)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    thetas = synth.uniform_thetas(spec.n_params, B, seed=91)
    th = torch.tensor(thetas, device="cuda:0")
    _say("autotune n = 12, batch 4")
    r = vqe.autotune(ctx, C, H, th, want_grad=True)
    _say(f"tuned {r}")
    assert r["candidates"] >= 5
    assert r["ms_tuned"] <= r["ms_default"] * 1.05
    assert 8 <= r["k_fwd"] <= 12 and 8 <= r["k_rev"] <= 12 and 1 <= r["batch_tile"] <= B
    e, g = vqe.energy_grad(ctx, C, H, th)
    torch.cuda.synchronize()
    for b in range(B):
        eo, go = oracle.energy_grad(spec, ham, thetas[b], "adjoint")
        assert abs(e[b].item() - eo) < E_TOL
        assert np.max(np.abs(g[b].cpu().numpy() - go)) < G_TOL
