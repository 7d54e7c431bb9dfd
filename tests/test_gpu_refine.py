"""GPU parity of the refinement kernels (paper Sec. 7) through the C ABI:
mismatch, tangent Jacobian, discrete-adjoint gradient with checkpoints,
damped Newton, and the autograd wrapper, against the oracle's mismatch (whose
Jacobian comes from the variational equations) and its damped Newton, on
planted problems whose roots are known."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

MU, ECC = 2.528e-5, 0.0094


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def planted(K, seed, steps):
    return synth.planted_refinement(K, seed, lambda x, n: oracle.rk8_map(x, MU, ECC, steps, n))


def rows(ms, pr):
    K = len(pr.patches_s)
    U = np.repeat(ms.patch_row(pr.patch_u)[None, :], K, axis=0)
    S = np.stack([ms.patch_row(p) for p in pr.patches_s])
    return U, S


def maps(ms, steps, e=ECC, n=3):
    return ms.MapParams(MU, e, steps, n), ms.MapParams(MU, e, steps, -n)


def oracle_mismatch(pr, params, steps, e=ECC):
    out = [oracle.mismatch(params[k:k + 1], pr.patch_u, pr.patches_s[k], MU, e, steps, 3, -3)
           for k in range(params.shape[0])]
    return tuple(np.concatenate([o[i] for o in out]) for i in range(4))   # f, r, J, grad


def starts(pr, seed, spread=1e-4):
    rng = np.random.default_rng(seed)
    return pr.roots + rng.uniform(-spread, spread, size=pr.roots.shape)


def np_(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("steps,K", [(400, 6), (4000, 3)])
def test_residual_tangent_adjoint_match_oracle(ms, steps, K):
    pr = planted(K, 1, steps)
    x = starts(pr, 11)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    f0, r0, J0, g0 = oracle_mismatch(pr, x, steps)
    res = ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_RESIDUAL)
    tan = ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_TANGENT)
    adj = ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 100)
    for out in (res, tan, adj):
        assert np.max(np.abs(np_(out["f"]) - f0)) <= 1e-10
        assert np.max(np.abs(np_(out["r"]) - r0)) <= 1e-10 * max(1.0, np.max(r0))
    jscale = max(1.0, np.max(np.abs(J0)))
    assert np.max(np.abs(np_(tan["J"]) - J0)) <= 1e-10 * jscale
    gscale = max(1e-12, np.max(np.abs(g0)))
    assert np.max(np.abs(np_(tan["grad"]) - g0)) <= 1e-10 * gscale
    assert np.max(np.abs(np_(adj["grad"]) - g0)) <= 1e-10 * gscale
    # transpose consistency: the adjoint gradient equals 2 J^T f from the tangent
    assert np.max(np.abs(np_(adj["grad"]) - np_(tan["grad"]))) <= 1e-11 * gscale


def test_adjoint_does_not_depend_on_checkpoint_interval(ms):
    """Store-all (one step per segment), the default interval, an interval
    that does not divide the step count, one segment, and an interval longer
    than the run give the same bits."""
    steps = 400
    pr = planted(4, 2, steps)
    x = starts(pr, 12)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    ref = np_(ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 1)["grad"])
    for ck in (7, 100, 1200, 5000):
        g = np_(ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, ck)["grad"])
        assert np.array_equal(g, ref), ck


def test_adjoint_against_central_differences(ms):
    """dr/d(th1, s1, th2, s2, e) at unrefined hits (|f| ~ 1e-4) against central
    differences of the GPU residual with h = 1e-6."""
    steps = 400
    pr = planted(3, 3, steps)
    x = starts(pr, 13)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    g = np_(ms.refine_grad(x, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 100)["grad"])
    h = 1e-6
    for j in range(4):
        d = np.zeros(4); d[j] = h
        rp = np_(ms.refine_grad(x + d, U, S, fwd, bwd, ms.MS_REFINE_RESIDUAL)["r"])
        rm = np_(ms.refine_grad(x - d, U, S, fwd, bwd, ms.MS_REFINE_RESIDUAL)["r"])
        fd = (rp - rm) / (2 * h)
        assert np.max(np.abs(fd - g[:, j])) <= 1e-7 * np.max(np.abs(g[:, j])), j
    fp_, bp_ = maps(ms, steps, ECC + h)
    fm_, bm_ = maps(ms, steps, ECC - h)
    rp = np_(ms.refine_grad(x, U, S, fp_, bp_, ms.MS_REFINE_RESIDUAL)["r"])
    rm = np_(ms.refine_grad(x, U, S, fm_, bm_, ms.MS_REFINE_RESIDUAL)["r"])
    fd = (rp - rm) / (2 * h)
    assert np.max(np.abs(fd - g[:, 4])) <= 1e-7 * np.max(np.abs(g[:, 4]))


def test_shared_patches_equal_replicated_patches(ms):
    steps = 400
    pr = planted(1, 4, steps)
    K = 5
    rng = np.random.default_rng(14)
    x = pr.roots + rng.uniform(-1e-4, 1e-4, size=(K, 4))
    U1 = ms.patch_row(pr.patch_u)
    S1 = ms.patch_row(pr.patches_s[0])
    fwd, bwd = maps(ms, steps)
    a = ms.refine_grad(x, U1, S1, fwd, bwd, ms.MS_REFINE_TANGENT)
    b = ms.refine_grad(x, np.repeat(U1[None], K, 0), np.repeat(S1[None], K, 0), fwd, bwd, ms.MS_REFINE_TANGENT)
    for k in ("f", "r", "J", "grad"):
        assert np.array_equal(np_(a[k]), np_(b[k])), k


@pytest.mark.parametrize("steps", [400, 4000])
def test_newton_matches_oracle(ms, steps):
    K = 6 if steps == 400 else 3
    pr = planted(K, 5, steps)
    x0 = starts(pr, 15)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    xg, fg, rg, sg, tg = (np_(t) for t in ms.refine_newton(x0, U, S, fwd, bwd, max_trials=30, tol=1e-12))
    xo, fo, ro, so, to = oracle.damped_newton(x0, pr.patch_u, pr.patches_s, MU, ECC, steps, 3, -3,
                                              max_trials=30, tol=1e-12)
    assert np.array_equal(sg, so)
    assert np.all(sg == 0)
    assert np.array_equal(tg, to)
    assert np.max(np.abs(xg - xo)) <= 1e-10
    assert np.max(np.abs(xg - pr.roots)) <= 1e-10
    assert np.all(rg <= 1e-24)


def test_newton_far_starts_and_limits(ms):
    """Far starts: the step is halved until r decreases.  Rounding can steer
    the GPU and the oracle iterations apart there, so rows are compared only
    where both converged to the same root."""
    steps = 400
    pr = planted(4, 6, steps)
    x0 = starts(pr, 16, 3e-2)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    xg, fg, rg, sg, tg = (np_(t) for t in ms.refine_newton(x0, U, S, fwd, bwd, max_trials=60))
    xo, fo, ro, so, to = oracle.damped_newton(x0, pr.patch_u, pr.patches_s, MU, ECC, steps, 3, -3, max_trials=60)
    assert set(sg.tolist()) <= {0, 1, 2} and np.all(tg <= 60)
    assert np.all(rg[sg == 0] <= 1e-24)
    both = (sg == 0) & (so == 0)
    same = both & (np.max(np.abs(xg - xo), axis=1) < 1e-6)
    assert np.max(np.abs(xg[same] - xo[same])) <= 1e-10 if same.any() else True
    # one trial only
    xg, fg, rg, sg, tg = (np_(t) for t in ms.refine_newton(x0, U, S, fwd, bwd, max_trials=1))
    assert np.all(sg == 1) and np.all(tg == 1)
    # a zero patch direction makes the first column of Df exactly zero
    Ub = U.copy(); Ub[:, 4:8] = 0.0
    xg, fg, rg, sg, tg = (np_(t) for t in ms.refine_newton(x0, Ub, S, fwd, bwd, max_trials=5))
    assert np.all(sg == 3) and np.all(tg == 0) and np.array_equal(xg, x0)


def test_autograd_function_uses_the_adjoint(ms):
    import torch
    steps = 400
    pr = planted(4, 7, steps)
    x = torch.tensor(starts(pr, 17), dtype=torch.float64, device="cuda", requires_grad=True)
    e = torch.tensor(ECC, dtype=torch.float64, requires_grad=True)
    U, S = rows(ms, pr)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device="cuda")
    r = ms.mismatch_r(x, e, U, S, MU, steps, 3, -3, 100)
    (w * r).sum().backward()
    fwd, bwd = maps(ms, steps)
    g = np_(ms.refine_grad(x.detach(), U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 100)["grad"])
    wn = np_(w)
    assert np.array_equal(np_(x.grad), wn[:, None] * g[:, :4])
    assert abs(float(e.grad) - float(np.sum(wn * g[:, 4]))) <= 1e-12 * max(1e-30, abs(float(e.grad)))
    _, r0, _, _ = oracle_mismatch(pr, np_(x), steps)
    assert np.max(np.abs(np_(r) - r0)) <= 1e-10


def test_refine_edge_cases(ms):
    import ctypes as C
    import torch
    pr = planted(2, 8, 400)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, 400)
    # no hits
    out = ms.refine_grad(np.zeros((0, 4)), U[:0], S[:0], fwd, bwd, ms.MS_REFINE_ADJOINT)
    assert out["grad"].shape == (0, 5)
    xo, *_ = ms.refine_newton(np.zeros((0, 4)), U[:0], S[:0], fwd, bwd)
    assert xo.shape == (0, 4)
    # different mu on the two sides
    with pytest.raises(ms.MSearchError) as ei:
        ms.refine_grad(pr.roots, U, S, fwd, ms.MapParams(MU * 2, ECC, 400, -3), ms.MS_REFINE_RESIDUAL)
    assert ei.value.code == ms.MS_E_ARG
    # adjoint without a checkpoint interval
    with pytest.raises(ms.MSearchError):
        ms.refine_grad(pr.roots, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 0)
    # workspace too small (direct call through the C ABI)
    x = torch.tensor(pr.roots, dtype=torch.float64, device="cuda")
    u = torch.tensor(U, device="cuda"); s = torch.tensor(S, device="cuda")
    f = torch.empty((2, 4), dtype=torch.float64, device="cuda")
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    rc = ms.lib().refine_grad(C.c_void_p(x.data_ptr()), 2, C.c_void_p(u.data_ptr()), C.c_void_p(s.data_ptr()), 1,
                              C.byref(fwd), C.byref(bwd), 100, ms.MS_REFINE_RESIDUAL, C.c_void_p(f.data_ptr()),
                              None, None, None, C.c_void_p(ws.data_ptr()), 64, None)
    assert rc == ms.MS_E_WORKSPACE


def test_planted_family_at_full_steps_sampled(ms):
    """128 planted problems at 4000 steps per period (the workload the bench
    times): the GPU Newton converges on all of them to the planted roots and
    the adjoint agrees with the oracle on a sample."""
    steps, K = 4000, 128
    pr = planted(K, 9, steps)
    x0 = starts(pr, 19)
    U, S = rows(ms, pr)
    fwd, bwd = maps(ms, steps)
    xg, fg, rg, sg, tg = (np_(t) for t in ms.refine_newton(x0, U, S, fwd, bwd, max_trials=30))
    assert np.all(sg == 0)
    assert np.max(np.abs(xg - pr.roots)) <= 1e-10
    adj = np_(ms.refine_grad(x0, U, S, fwd, bwd, ms.MS_REFINE_ADJOINT, 100)["grad"])
    for k in (0, 63, 127):
        f0, r0, J0, g0 = oracle.mismatch(x0[k:k + 1], pr.patch_u, pr.patches_s[k], MU, ECC, steps, 3, -3)
        assert np.max(np.abs(adj[k] - g0[0])) <= 1e-10 * max(1e-12, np.max(np.abs(g0)))
