"""The thesis's benchmark operator (Section 5.1.2): 2D diffusion, first
order in time, on the GPU vs the FP64 oracle, at every space order the
thesis sweeps, with ragged tiles, and at its two grid sizes in the launch
shape the benchmark times (a few steps, every point compared)."""
import numpy as np
import pytest

import oracle
from gpu_common import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu


def _hat(nx, ny, seed):
    """Seeded hat initial condition (2 inside a random box, 1 outside), as in
    the Devito tutorial's init_hat (Section 2.1.1), plus a little noise."""
    rng = np.random.default_rng(seed)
    u = np.ones((ny, nx))
    x0, y0 = rng.integers(nx // 4, nx // 2), rng.integers(ny // 4, ny // 2)
    u[y0:y0 + ny // 4, x0:x0 + nx // 4] = 2.0
    return u + 0.05 * rng.standard_normal((ny, nx))


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
@pytest.mark.parametrize("time_block", [0, 1, 3, 16])
def test_diffusion_parity(so, time_block):
    """203 x 141 (ragged 64 x 64 tiles), 121 steps: the automatic choice, one
    step per launch, 3 per launch, or as many as the tile halo allows
    (16 / (so/2), with a shorter last launch)."""
    need_gpu()
    from paper_1906_10811_amd import diffusion
    nx, ny, h = 203, 141, (1.0 / 202, 1.0 / 140)
    g = oracle.Grid((nx, ny), h, (0.0, 0.0), so)
    nu = 0.5
    dt = 0.8 * oracle.diffusion_critical_dt(g, nu)
    u0 = _hat(nx, ny, so)
    want = oracle.diffusion(g, u0, nu, dt, 121)
    got = diffusion(torch.from_numpy(u0).float().cuda(), h, so, nu, dt, 121, time_block=time_block)
    torch.cuda.synchronize()
    e = rel_l2(got.cpu().numpy(), want)
    print("diffusion so=%d time_block=%d rel L2 %.3e" % (so, time_block, e))
    assert e <= 1e-5


_FULL_WANT = {}   # oracle result of the current size, shared by both launch forms


@pytest.mark.parametrize("time_block", [1, 16])
@pytest.mark.parametrize("n", [2500, 10000])
def test_diffusion_full_size(n, time_block):
    need_gpu()
    from paper_1906_10811_amd import diffusion
    so = 8
    h = (1.0 / (n - 1), 1.0 / (n - 1))
    g = oracle.Grid((n, n), h, (0.0, 0.0), so)
    nu = 0.5
    dt = 0.8 * oracle.diffusion_critical_dt(g, nu)
    u0 = _hat(n, n, 3).astype(np.float32)
    nt = 5
    got = diffusion(torch.from_numpy(u0).cuda(), h, so, nu, dt, nt, time_block=time_block)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    if n not in _FULL_WANT:
        _FULL_WANT.clear()
        _FULL_WANT[n] = oracle.diffusion(g, u0.astype(np.float64), nu, dt, nt)
    e = rel_l2(got, _FULL_WANT[n])
    print("diffusion %d^2 so 8, %d steps, time_block %d: rel L2 %.3e" % (n, nt, time_block, e))
    assert e <= 1e-5


def test_diffusion_rejects_unstable_dt():
    need_gpu()
    from paper_1906_10811_amd import FDError, diffusion
    g = oracle.Grid((64, 64), (1.0, 1.0), (0.0, 0.0), 4)
    lim = oracle.diffusion_critical_dt(g, 0.5)
    u = torch.zeros((64, 64), device="cuda")
    with pytest.raises(FDError) as e:
        diffusion(u, (1.0, 1.0), 4, 0.5, 1.01 * lim, 5)
    assert e.value.code == -2
    diffusion(u, (1.0, 1.0), 4, 0.5, 0.99 * lim, 5)
