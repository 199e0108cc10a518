"""Served results: every request's energy (and gradient) is the same alone and
in the mix, within the energy / gradient tolerances, and matches the oracle."""
import numpy as np
import pytest

import oracle
import synth
from oracle import fermion

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

MIX = ((4, 0.4), (8, 0.3), (12, 0.2), (16, 0.1))


@pytest.fixture(scope="module")
def mods():
    from paper_2601_09951_amd import serve, vqe
    return serve, vqe


@pytest.fixture(scope="module")
def ctx(mods):
    c = mods[1].Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _alone(vqe, ctx, r):
    spec = r.circuit
    C = vqe.Circuit.from_spec(ctx, spec)
    if r.integrals is not None:
        H = vqe.Hamiltonian.from_integrals(ctx, r.integrals.h1, r.integrals.h2, r.integrals.e_core)
    else:
        H = vqe.Hamiltonian.from_sum(ctx, r.pauli)
    th = torch.tensor(r.theta[None, :], dtype=torch.float64, device="cuda:0")
    e, g = vqe.energy_grad(ctx, C, H, th)
    torch.cuda.synchronize()
    return e.item(), g.cpu().numpy()[0]


@pytest.mark.parametrize("budget", [32 << 30, 6 << 20])
def test_served_equals_alone(mods, ctx, budget):
    serve, vqe = mods
    print("[case] served mix, budget", budget, flush=True)
    reqs = synth.served_requests(80, 400.0, seed=11, mix=MIX)
    srv = serve.Server(serve.LibvqeExecutor(ctx), mem_budget=budget, max_batch=32)
    # every request has arrived when serving starts, so batches form whatever the GPU's speed
    res = srv.run(reqs, realtime=False)
    assert [r.rid for r in res] == [q.rid for q in sorted(reqs, key=lambda q: q.rid)]
    assert 0 < srv.stats["peak_bytes"] <= budget  # admission never exceeds the device-memory budget
    if budget >= (1 << 30):
        assert srv.stats["max_batch_seen"] > 1
    for q, r in zip(sorted(reqs, key=lambda q: q.rid), res):
        e, g = _alone(vqe, ctx, q)
        assert abs(r.energy - e) < 1e-10
        if q.want_grad:
            np.testing.assert_allclose(r.grad, g, atol=1e-9)
        else:
            assert r.grad is None


def test_served_matches_oracle_on_a_sample(mods, ctx):
    serve, vqe = mods
    print("[case] served vs oracle", flush=True)
    reqs = synth.served_requests(40, 400.0, seed=12, mix=MIX)
    res = serve.Server(serve.LibvqeExecutor(ctx)).run(reqs)
    by = {r.rid: r for r in res}
    for q in reqs[:12]:
        ham = fermion.qubit_hamiltonian(q.integrals) if q.integrals is not None else q.pauli
        eo, go = oracle.energy_grad(q.circuit, ham, q.theta, "adjoint")
        assert abs(by[q.rid].energy - eo) < 1e-10
        if q.want_grad:
            np.testing.assert_allclose(by[q.rid].grad, go, atol=1e-9)


def test_plain_path_matches(mods, ctx):
    serve, vqe = mods
    print("[case] plain path", flush=True)
    reqs = synth.served_requests(20, 1000.0, seed=13, mix=MIX)
    plain = serve.run_plain(ctx, reqs, realtime=False)
    served = serve.Server(serve.LibvqeExecutor(ctx)).run(reqs)
    for a, b in zip(plain, served):
        assert abs(a.energy - b.energy) < 1e-10


def test_short_requests_finish_while_a_long_batch_runs(mods, ctx):
    """Continuous batching on the device: while a batch of 24-qubit energy +
    gradient requests is in flight, single 4-qubit requests launched after it
    complete (their own completion events fire) before it does, and their
    results equal the same requests evaluated alone."""
    serve, vqe = mods
    print("[case] short requests beside a long batch", flush=True)
    ex = serve.LibvqeExecutor(ctx)
    big = [r for r in synth.served_requests(600, 1000.0, seed=21) if r.n == 24 and r.want_grad][:8]
    small = synth.served_requests(24, 1000.0, seed=22, mix=((4, 1.0),))
    assert len(big) == 8

    def run_one(r):
        k = serve.Server._class(r)
        hs = [ex.hamiltonian(r)]
        return k, hs, ex.launch(k, [r], hs, ex.batch_bytes(k, [r], hs))

    k, hs, h = run_one(small[0])  # warm the small class (plans, code objects)
    ex.collect(h)
    ex.release(hs[0])
    kb = serve.Server._class(big[0])
    hb = [ex.hamiltonian(r) for r in big]
    hbig = ex.launch(kb, big, hb, ex.batch_bytes(kb, big, hb))
    before, got = 0, []
    for r in small[1:]:
        k, hs, h = run_one(r)
        h["event"].synchronize()  # waits for this request's own stream only
        if not ex.done(hbig):
            before += 1
        got.append((r, ex.collect(h)))
        ex.release(hs[0])
    big_done_last = not ex.done(hbig) or before == len(small) - 1
    ex.collect(hbig)
    for hm in hb:
        ex.release(hm)
    ex.close()
    for r, (e, g) in got:
        if r.want_grad:
            e1, g1 = _alone(vqe, ctx, r)
            assert abs(e[0] - e1) < 1e-10
            np.testing.assert_allclose(g[0], g1, atol=1e-9)
    print(f"[case] {before} of {len(small) - 1} short requests finished before the long batch "
          f"(long batch still running at the end: {big_done_last})", flush=True)
    assert before >= 1, "every short request waited for the long batch"
