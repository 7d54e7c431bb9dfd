"""The map and refinement entry points captured into a HIP graph on their
first call with an eccentricity and a step count no other call has used:
they allocate nothing and never synchronise (the stage values are computed
on the GPU, the tableau is a compile-time constant), so the capture needs no
warm-up call.  Every replay, after in-place changes of the inputs and eager
work in between, equals the eager calls; the eager results match the oracle
(Sec. 4.1 map, Sec. 7 mismatch, tangent and adjoint)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MU = 2.528e-5
E_NEW = 0.0094 + 3.137e-5       # used by no other test, so nothing can have been prepared for it
STEPS = 372


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def test_capture_on_first_call_with_new_e(ms):
    import torch
    pr = synth.planted_refinement(5, 23, lambda x, n: oracle.rk8_map(x, MU, E_NEW, STEPS, n))
    K = len(pr.patches_s)
    rng = np.random.default_rng(4)
    x = torch.tensor(pr.roots + rng.uniform(-1e-4, 1e-4, pr.roots.shape), device="cuda")
    U = torch.tensor(np.repeat(ms.patch_row(pr.patch_u)[None, :], K, axis=0), device="cuda")
    S = torch.tensor(np.stack([ms.patch_row(p) for p in pr.patches_s]), device="cuda")
    fwd, bwd = ms.MapParams(MU, E_NEW, STEPS, 3), ms.MapParams(MU, E_NEW, STEPS, -3)
    z = torch.tensor(synth.random_states(200, 9, synth.UNSTABLE_BASE, 1e-3), device="cuda")
    zp = torch.tensor(synth.pm_random_states(150, 10, E_NEW + 1e-6, synth.UNSTABLE_BASE, 1e-3), device="cuda")

    def work():
        outs = []
        for mode, ck in ((ms.MS_REFINE_RESIDUAL, 1), (ms.MS_REFINE_TANGENT, 1), (ms.MS_REFINE_ADJOINT, 50)):
            o = ms.refine_grad(x, U, S, fwd, bwd, mode, ck)
            outs += [o[k] for k in ("f", "r", "grad", "J") if k in o]
        outs.append(ms.propagate(z, MU, E_NEW + 2e-6, STEPS + 1, 2))
        outs.append(ms.pertbp_map(zp, MU, E_NEW + 1e-6, STEPS + 3, -1))
        return outs

    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            captured = work()                  # the first calls with these parameters
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for rep in range(3):
        x.add_(1e-6 * (rep + 1))
        z.add_(1e-5)
        zp.add_(-1e-5)
        junk.add_(1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = work()
        torch.cuda.synchronize()
        for i, (c, e) in enumerate(zip(captured, eager)):
            assert torch.equal(c, e), (rep, i)
    # the eager results against the oracle
    xs = x.cpu().numpy()
    f0, r0, J0, g0 = (np.concatenate(v) for v in zip(*[
        oracle.mismatch(xs[k:k + 1], pr.patch_u, pr.patches_s[k], MU, E_NEW, STEPS, 3, -3) for k in range(K)]))
    f_res, r_res, f_tan, r_tan, g_tan, J_tan, f_adj, r_adj, g_adj = (t.cpu().numpy() for t in eager[:9])
    for f in (f_res, f_tan, f_adj):
        assert np.max(np.abs(f - f0)) <= 1e-10
    gs = max(1e-12, np.max(np.abs(g0)))
    assert np.max(np.abs(J_tan - J0)) <= 1e-10 * max(1.0, np.max(np.abs(J0)))
    assert np.max(np.abs(g_tan - g0)) <= 1e-10 * gs and np.max(np.abs(g_adj - g0)) <= 1e-10 * gs
    y = eager[9].cpu().numpy()
    assert np.max(np.abs(y - oracle.rk8_map(z.cpu().numpy(), MU, E_NEW + 2e-6, STEPS + 1, 2))) <= 1e-10
    yp = eager[10].cpu().numpy()
    assert np.max(np.abs(yp - oracle.pertbp_map(zp.cpu().numpy(), MU, E_NEW + 1e-6, STEPS + 3, -1))) <= 1e-10


def _tolerance(ref, perturbed):
    """1e-10 of the scale, plus the map's own conditioning: 1e3 times the
    oracle's response to a 1e-15 relative change of its inputs.  At 5 steps
    per period over 3 periods the discrete map amplifies such a change to
    ~1e-7, so rounding-level differences (device cos in the stage values,
    fused multiply-adds) cannot agree to 1e-10 there; a wrong stage index
    changes the force by up to 10% at some stage and is far above this."""
    return 1e-10 * max(1.0, np.max(np.abs(ref))) + 1e3 * np.max(np.abs(perturbed - ref))


@pytest.mark.parametrize("steps", [5, 7, 31, 32, 33, 100])
def test_maps_at_step_counts_around_the_stage_chunk(ms, steps):
    """Step counts below, at and just above the number of steps whose stage
    values a block computes at a time, over several periods (the stage index
    wraps inside a chunk), against the oracle."""
    import torch
    z = synth.random_states(130, steps, synth.UNSTABLE_BASE, 1e-3)
    for n in (3, -2):
        got = ms.propagate(torch.tensor(z, device="cuda"), MU, 0.05, steps, n).cpu().numpy()
        ref = oracle.rk8_map(z, MU, 0.05, steps, n)
        tol = _tolerance(ref, oracle.rk8_map(z * (1.0 + 1e-15), MU, 0.05, steps, n))
        assert np.max(np.abs(got - ref)) <= tol, (n, np.max(np.abs(got - ref)), tol)
    zp = synth.pm_random_states(130, steps, 0.05, synth.UNSTABLE_BASE, 1e-3)
    got = ms.pertbp_map(torch.tensor(zp, device="cuda"), MU, 0.05, steps, 3).cpu().numpy()
    ref = oracle.pertbp_map(zp, MU, 0.05, steps, 3)
    tol = _tolerance(ref, oracle.pertbp_map(zp * (1.0 + 1e-15), MU, 0.05, steps, 3))
    assert np.max(np.abs(got - ref)) <= tol, (np.max(np.abs(got - ref)), tol)
