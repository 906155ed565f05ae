"""Edge and degenerate cases of the GPU path against the FP64 oracle: no
time steps, grids smaller than the stencil, sparse points on every corner
of a grid without damping layer (multilinear and windowed sinc, most sinc
nodes cut), a zero wavelet, the receiver-table capacity, and the extreme
z-chunk lengths of the 3D launch (one plane; the 256-plane maximum)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import case, gpu_forward, gpu_grid, need_gpu, oracle_forward, rel_l2, torch

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _corners(c):
    ext = [(n - 1) * hh for n, hh in zip(c["shape"], c["spacing"])]
    nd = len(ext)
    return np.array([[o + (e if (k >> a) & 1 else 0.0) for a, (o, e) in enumerate(zip(c["origin"], ext))]
                     for k in range(1 << nd)])


def test_zero_steps_keep_the_given_state():
    need_gpu()
    c = case((30, 22, 17), 8, 3, 5, seed=2)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(0)
    u0 = torch.from_numpy(rng.standard_normal(c["og"].array_shape).astype(np.float32)).to(dev)
    um = torch.from_numpy(rng.standard_normal(c["og"].array_shape).astype(np.float32)).to(dev)
    wav = torch.empty((0, 1), dtype=torch.float32, device=dev)
    rec, (u, up) = g.forward(c["src"], wav, c["rec"], c["dt"], u0=u0, u_prev=um, save_state=True)
    torch.cuda.synchronize()
    assert rec.shape == (0, len(c["rec"]))
    assert torch.equal(u, u0) and torch.equal(up, um)


@pytest.mark.parametrize("shape,so,sinc", [((2, 3, 2), 16, 0), ((2, 3, 2), 16, 8), ((3, 2), 16, 8), ((5, 4), 2, 1)])
def test_grid_smaller_than_the_stencil(shape, so, sinc):
    """No damping layer, radius up to 8 on 2 or 3 points per axis: every
    neighbour read lands in the zero halo; sources and receivers on corners."""
    need_gpu()
    c = case(shape, so, 0, 40, seed=4, nsrc=1, nrec=1)
    cs = _corners(c)
    c["src"] = [tuple(cs[0])]
    c["rec"] = cs
    c["sinc"] = sinc
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("tiny %s so=%d sinc=%d: traces %.3e field %.3e" % (shape, so, sinc, e_rec, e_u), flush=True)
    assert e_rec <= TOL and e_u <= TOL


@pytest.mark.parametrize("sinc", [0, 4])
def test_points_on_every_corner(sinc):
    """25 x 19 x 13 without layer: a source on one corner and a receiver on
    each of the 8 corners (multilinear: the last-line rule on every axis;
    sinc: the node window cut on three sides, the weights a delta because a
    corner is a grid point)."""
    need_gpu()
    c = case((25, 19, 13), 8, 0, 60, seed=6, nsrc=1, nrec=1)
    cs = _corners(c)
    c["src"] = [tuple(cs[7])]
    c["rec"] = cs
    c["sinc"] = sinc
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("corners sinc=%d: traces %.3e field %.3e" % (sinc, e_rec, e_u), flush=True)
    assert e_rec <= TOL and e_u <= TOL


def test_zero_wavelet_gives_exact_zeros():
    need_gpu()
    c = case((40, 33, 21), 8, 4, 30, seed=3, nsrc=2, nrec=9)
    c["wav"] = np.zeros_like(c["wav"])
    _, (rec, state) = gpu_forward(c, save_state=True)
    assert torch.count_nonzero(rec).item() == 0 and torch.count_nonzero(state[0]).item() == 0


def test_receiver_table_capacity():
    """The default table holds 4096 receivers (all of them checked against
    the oracle); one more is rejected and the grid keeps working."""
    need_gpu()
    from paper_1906_10811_amd import FDError
    c = case((90, 70), 4, 4, 40, seed=8, nsrc=1, nrec=4096)
    want, *_ = oracle_forward(c)
    g = gpu_grid(c)
    _, rec = gpu_forward(c, grid=g)
    e = rel_l2(rec.cpu().numpy(), want)
    print("4096 receivers: %.3e" % e, flush=True)
    assert e <= TOL
    dev = torch.device("cuda:0")
    more = np.concatenate([c["rec"], c["rec"][:1]])
    with pytest.raises(FDError):
        g.forward(c["src"], torch.from_numpy(c["wav"]).to(dev), more, c["dt"])
    _, rec2 = gpu_forward(c, grid=g)
    assert torch.equal(rec, rec2)


@pytest.mark.parametrize("shape,zchunk", [((30, 20, 24), 1), ((20, 18, 560), 512), ((20, 18, 560), 2000)])
def test_extreme_z_chunks(shape, zchunk):
    """One plane per workgroup (every plane a chunk start, warm-up only), the
    longest chunk the kernel stages (512 planes, then a ragged 52), and a
    request beyond it, which is clamped to 512."""
    need_gpu()
    c = case(shape, 8, 2, 30, seed=9, nsrc=2, nrec=7)
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, grid=gpu_grid(c, zchunk=zchunk), save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("zchunk %d on %s: traces %.3e field %.3e" % (zchunk, shape, e_rec, e_u), flush=True)
    assert e_rec <= TOL and e_u <= TOL


def test_shots_without_sources_or_receivers():
    """No sources (an initial-value problem from a caller's u^0 = u^{-1}) and
    no receivers (only the final state) against the oracle; the adjoint of
    an empty receiver set is zero and of an empty source set is empty."""
    need_gpu()
    c = case((44, 36, 30), 8, 5, 50, seed=31, nsrc=1, nrec=7)
    dev = torch.device("cuda:0")
    x = np.linspace(-1.0, 1.0, c["og"].array_shape[2])
    bump = np.exp(-((x[None, None, :] ** 2 + np.linspace(-1, 1, c["og"].array_shape[1])[None, :, None] ** 2
                     + np.linspace(-1, 1, c["og"].array_shape[0])[:, None, None] ** 2) / 0.05))
    no_src = dict(c, src=np.zeros((0, 3)), wav=np.zeros((c["nt"], 0), dtype=np.float32))
    want, u_nt, _, _ = oracle_forward(no_src, u0=bump, u_prev=bump)
    g = gpu_grid(c)
    u0 = torch.from_numpy(bump.astype(np.float32)).to(dev)
    rec, (u, _) = g.forward(no_src["src"], torch.zeros((c["nt"], 0), device=dev), c["rec"], c["dt"],
                            u0=u0, u_prev=u0, save_state=True)
    torch.cuda.synchronize()
    assert rec.shape == (c["nt"], len(c["rec"]))
    assert rel_l2(rec.cpu().numpy(), want) <= TOL
    assert rel_l2(u.cpu().numpy(), u_nt) <= TOL
    want2, u2, _, _ = oracle_forward(c)
    rec0, (v, _) = g.forward(c["src"], torch.from_numpy(c["wav"]).to(dev), np.zeros((0, 3)), c["dt"],
                             save_state=True)
    torch.cuda.synchronize()
    assert rec0.shape == (c["nt"], 0)
    assert rel_l2(v.cpu().numpy(), u2) <= TOL
    res = torch.zeros((c["nt"], 0), device=dev)
    fa = g.adjoint(c["src"], np.zeros((0, 3)), res, c["dt"])
    fb = g.adjoint(np.zeros((0, 3)), c["rec"], torch.ones((c["nt"], len(c["rec"])), device=dev), c["dt"])
    torch.cuda.synchronize()
    assert fa.shape == (c["nt"], 1) and not bool(fa.any())
    assert fb.shape == (c["nt"], 0)
    g.close()
