"""The map, matrix, theta shift and chart entry points captured into one graph
on the caller's stream (after a first call has built their tables): every
replay, with eager device work and synchronisations between the replays and
new input values each time, equals the eager calls on the same inputs."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

MU, ECC = 2.527e-5, 0.0094


@pytest.fixture(scope="module")
def ms():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_14814_amd as ms
    ms.lib()
    return ms


def test_capture_and_replay(ms):
    import torch
    rng = np.random.default_rng(5)
    z = torch.tensor(synth.pm_random_states(300, 1, ECC, synth.UNSTABLE_BASE, 1e-3), device="cuda")
    rows = torch.tensor(rng.standard_normal((40, 256, 4)), device="cuda")
    rho = torch.tensor(rng.uniform(-2, 2, 40), device="cuda")
    th = 2 * np.pi * np.arange(64) / 64
    coeffs = np.stack([np.outer(np.cos(k * th), rng.standard_normal(4)) / (k + 1) for k in range(6)])
    chart = ms.FourierTaylor(coeffs)
    qt = torch.tensor(rng.uniform(0, 6, 100), device="cuda")
    qs = torch.tensor(rng.uniform(-0.5, 0.5, 100), device="cuda")

    def work():
        a = ms.pertbp_map(z, MU, ECC, 200, 1)
        b = ms.pertbp_map_stm(z, MU, ECC, 200, -1)
        c = ms.theta_shift(rows, rho, 1)
        d = chart.partials(qt, qs)
        return [a, b[0], b[1], c, *d]

    work()                                   # builds the stage, twiddle tables
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        with torch.cuda.graph(g, stream=stream):
            outs = work()
    torch.cuda.current_stream().wait_stream(stream)
    torch.cuda.synchronize()
    for rep in range(3):
        # eager work between replays: new inputs, written in place
        z.add_(1e-4 * (rep + 1))
        rows.mul_(1.0 + 0.01 * rep)
        rho.add_(0.1)
        qt.add_(0.05)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = work()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), rep
