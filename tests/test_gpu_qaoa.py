"""QAOA MaxCut on the device (the diagonal-only Hamiltonian path and circuits
of H, CNOT, RZ and RX with parameters shared across gates):

* energy and adjoint gradient against the oracle at sizes it finishes
  (several tile geometries, a batch of parameter points);
* the persistent Adam loop against the oracle's;
* one layer at 22 qubits against the published closed form of
  <Z_u Z_v> (oracle parity unpinned at that size; the closed form and its
  central differences pin energy and gradient instead).
"""
import math

import numpy as np
import pytest

import oracle
import synth

from .qaoa_closed_form import qaoa1_zz_closed_form

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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0").contiguous()


@pytest.mark.parametrize("n,layers,tiles", [(10, 3, (12, 11, 3)), (13, 2, (9, 9, 3)), (14, 2, (12, 10, 4))])
def test_qaoa_energy_grad_matches_oracle(vqe, ctx, n, layers, tiles):
    _say("qaoa energy_grad", n, layers, tiles)
    ctx.set_tile(*tiles)
    edges = synth.ring_graph(n, n // 2, seed=n)
    spec = synth.qaoa_circuit(n, edges, layers)
    ham = synth.maxcut_hamiltonian(n, edges, weights=np.linspace(0.5, 1.5, len(edges)))
    th = synth.uniform_thetas(spec.n_params, 2, seed=n)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    e0 = vqe.energy(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    e, g, e0 = e.cpu().numpy(), g.cpu().numpy(), e0.cpu().numpy()
    ctx.set_tile(12, 11, 3)
    for b in range(2):
        eo, go = oracle.energy_grad(spec, ham, th[b], "adjoint")
        assert abs(e[b] - eo) < E_TOL
        assert abs(e0[b] - eo) < E_TOL
        np.testing.assert_allclose(g[b], go, atol=G_TOL)


def test_qaoa_persistent_adam_loop(vqe, ctx):
    _say("qaoa adam loop")
    n, iters = 8, 30
    edges = synth.ring_graph(n, 4, seed=5)
    spec = synth.qaoa_circuit(n, edges, 2)
    ham = synth.maxcut_hamiltonian(n, edges)
    th0 = synth.uniform_thetas(spec.n_params, 3, seed=5)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)
    th = dev(th0)
    traj = vqe.run(ctx, C, H, th, iters).cpu().numpy()
    thf = th.cpu().numpy()
    for b in range(3):
        want, tho = oracle.vqe_run(spec, ham, th0[b], iters)
        np.testing.assert_allclose(traj[b], want, atol=E_TOL)
        np.testing.assert_allclose(thf[b], tho, atol=1e-7)


def test_qaoa_one_layer_closed_form_at_22_qubits(vqe, ctx):
    n = 22
    _say("qaoa closed form", n)
    edges = synth.random_graph(n, 0.15, seed=22)
    spec = synth.qaoa_circuit(n, edges, 1)
    ham = synth.maxcut_hamiltonian(n, edges)
    C = vqe.Circuit.from_spec(ctx, spec)
    H = vqe.Hamiltonian.from_sum(ctx, ham)

    def closed(tc, tm):
        return sum(qaoa1_zz_closed_form(edges, n, a, b, tc, tm) for a, b in edges)

    th = np.array([[0.37, -1.21], [-2.3, 0.8]])
    e, g = vqe.energy_grad(ctx, C, H, dev(th))
    torch.cuda.synchronize()
    e, g = e.cpu().numpy(), g.cpu().numpy()
    h = 1e-5
    for b in range(2):
        tc, tm = th[b]
        assert abs(e[b] - closed(tc, tm)) < 1e-10
        fd = [(closed(tc + h, tm) - closed(tc - h, tm)) / (2 * h), (closed(tc, tm + h) - closed(tc, tm - h)) / (2 * h)]
        np.testing.assert_allclose(g[b], fd, atol=1e-7)
    del C, H
    torch.cuda.empty_cache()
