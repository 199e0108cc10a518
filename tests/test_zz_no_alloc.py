"""The allocation-free entry point vqe_apply_ansatz_noalloc, through the C ABI,
against vqe_apply_ansatz on the same inputs: two calls in a row, the second
with a smaller batch (the static array keeps the first call's contents), and
a batch too large for the array is rejected with an error naming the limit.
States must agree to 1e-12 per amplitude (the two share their kernels)."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S_TOL = 1e-12


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mods():
    from paper_2601_09951_amd import capi, vqe
    return capi, vqe


@pytest.fixture(scope="module")
def ctx(mods):
    c = mods[1].Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _call(L, fn, ctx, C, theta, psi):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return getattr(L, fn)(ctx.handle, C.handle, ctypes.c_int64(psi.shape[0]), ctypes.c_void_p(theta.data_ptr()),
                          ctypes.c_void_p(psi.data_ptr()), s)


def _ref_states(L, ctx, n, B, ref):
    psi = torch.empty(B, 1 << n, dtype=torch.complex128, device="cuda:0")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.vqe_prepare_reference(ctx.handle, n, ctypes.c_int64(B), ctypes.c_uint64(ref),
                                   ctypes.c_void_p(psi.data_ptr()), s) == 0
    return psi


@pytest.mark.parametrize("case", ["hea14", "ucc8"])
def test_noalloc_matches_apply_ansatz(mods, ctx, case):
    capi, vqe = mods
    L = capi.lib()
    if case == "hea14":
        spec = synth.hea_circuit(14, 3)  # several passes of fused stages
    else:
        spec = synth.ucc_circuit(8, 2)   # excitation gates: single-pass op lists
    C = vqe.Circuit.from_spec(ctx, spec)
    for call, B in enumerate((6, 2)):  # the second call is smaller
        _say(f"noalloc {case}: call {call + 1}, batch {B}")
        th = torch.tensor(synth.uniform_thetas(spec.n_params, B, seed=100 + call), device="cuda:0")
        want = _ref_states(L, ctx, spec.n, B, C.ref_index)
        got = _ref_states(L, ctx, spec.n, B, C.ref_index)
        assert _call(L, "vqe_apply_ansatz", ctx, C, th, want) == 0
        assert _call(L, "vqe_apply_ansatz_noalloc", ctx, C, th, got) == 0, L.vqe_last_error(ctx.handle)
        torch.cuda.synchronize()
        err = (got - want).abs().max().item()
        assert err <= S_TOL, (case, call, err)
        norms = torch.linalg.vector_norm(got, dim=1).cpu().numpy()
        np.testing.assert_allclose(norms, 1.0, atol=1e-12)
    C.close()


def test_noalloc_rejects_a_batch_beyond_the_array(mods, ctx):
    capi, vqe = mods
    L = capi.lib()
    spec = synth.hea_circuit(12, 12)
    C = vqe.Circuit.from_spec(ctx, spec)
    per_inst_min = spec.n_gates * 64  # the array holds at least every gate's matrix per instance
    B = capi.NOALLOC_SCRATCH_BYTES // per_inst_min + 1
    _say(f"noalloc over the limit: batch {B}")
    th = torch.zeros(B, spec.n_params, dtype=torch.float64, device="cuda:0")
    psi = _ref_states(L, ctx, spec.n, B, 0)
    before = psi.clone()
    rc = _call(L, "vqe_apply_ansatz_noalloc", ctx, C, th, psi)
    assert rc == capi.VQE_EINVAL
    msg = L.vqe_last_error(ctx.handle).decode()
    assert "static scratch" in msg and "at most" in msg, msg
    torch.cuda.synchronize()
    assert torch.equal(psi, before)  # nothing was enqueued
    C.close()
