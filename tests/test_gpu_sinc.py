"""Kaiser-windowed sinc sources and receivers (Hicks 2002) on the GPU
against the FP64 oracle with the same weights: forward traces and final
field, the adjoint, the gradient, the shot server, and the layouts that
stress the per-tile injection tables (nodes dropped at the edge of the
padded grid, sources sharing nodes across tile boundaries, a tile's plane
list longer than a workgroup).  Gate: relative L2 <= 1e-5 (float32
arithmetic), for the gradient as well."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (assert_field, assert_traces, case, gpu_forward, gpu_grid, need_gpu, oracle_forward,
                        rel_l2, torch)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _edge_points(c, r):
    """Move one source and one receiver to within a cell of opposite corners
    of the physical grid, so that with a thin layer some of their 2r nodes
    per axis fall outside the padded grid."""
    ext = [(n - 1) * hh for n, hh in zip(c["shape"], c["spacing"])]
    lo = tuple(o + 0.37 * hh for o, hh in zip(c["origin"], c["spacing"]))
    hi = tuple(o + e - 0.41 * hh for o, e, hh in zip(c["origin"], ext, c["spacing"]))
    c["src"][0] = lo
    c["rec"][0] = hi
    c["rec"][1] = lo


@pytest.mark.parametrize("shape,so,r", [((67, 133), 4, 1), ((67, 133), 8, 4), ((67, 133), 16, 8),
                                        ((70, 37, 29), 4, 2), ((70, 37, 29), 8, 4), ((70, 37, 29), 12, 3)])
def test_sinc_forward_parity(shape, so, r):
    need_gpu()
    c = case(shape, so, 2, 60, seed=so + r, nsrc=3, nrec=9)
    c["sinc"] = r
    _edge_points(c, r)
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("sinc %dD so=%d r=%d: traces %.3e field %.3e" % (len(shape), so, r, e_rec, e_u), flush=True)
    assert e_rec <= TOL and e_u <= TOL


def test_sinc_many_sources_across_tiles():
    """80 sources in a line along x that crosses x tiles, straddling a y tile
    boundary (padded y = 16), r = 4: up to 64 x 8 distinct nodes in one
    tile's plane, more than one per lane of the scattering workgroup, and
    nodes shared by neighbouring sources.  200 receivers over two planes."""
    need_gpu()
    c = case((150, 40, 30), 8, 3, 40, seed=5, nsrc=1, nrec=1)
    h, o = c["spacing"], c["origin"]
    y = o[1] + (16 - 3 - 0.45) * h[1]          # padded y 15.55: nodes 12..19 in two y tiles
    c["src"] = [(o[0] + 1.3 + 1.61 * k * h[0], y, o[2] + 11.3 * h[2]) for k in range(80)]
    c["wav"] = np.stack([synth.ricker(c["nt"], c["dt"], 0.12 / c["dt"] / 4, t0=1.2 * 4 * c["dt"] / 0.12)
                         * (1.0 + 0.01 * k) for k in range(80)], axis=1).astype(np.float32)
    rng = np.random.default_rng(3)
    ext = [(n - 1) * hh for n, hh in zip(c["shape"], h)]
    c["rec"] = np.array([[o[0] + rng.uniform(0, 1) * ext[0], o[1] + rng.uniform(0, 1) * ext[1],
                          o[2] + (5.5 if k % 2 else 20.2) * h[2]] for k in range(200)])
    c["sinc"] = 4
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, grid=gpu_grid(c, max_src=80), save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("sinc many sources: traces %.3e field %.3e" % (e_rec, e_u), flush=True)
    assert e_rec <= TOL and e_u <= TOL


@pytest.mark.parametrize("shape,r", [((67, 71), 4), ((40, 33, 26), 3)])
def test_sinc_adjoint_parity(shape, r):
    need_gpu()
    c = case(shape, 8, 3, 50, seed=9, nsrc=2, nrec=12)
    c["sinc"] = r
    _edge_points(c, r)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    rng = np.random.default_rng(4)
    res = rng.standard_normal((c["nt"], len(c["rec"])))
    want, _ = oracle.adjoint(og, vp, sig, c["dt"], c["nt"], c["src"], c["rec"], res, sinc_radius=r)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    got = g.adjoint(c["src"], c["rec"], torch.from_numpy(res.astype(np.float32)).to(dev), c["dt"])
    torch.cuda.synchronize()
    e = rel_l2(got.cpu().numpy(), want)
    print("sinc adjoint %dD r=%d: %.3e" % (len(shape), r, e), flush=True)
    assert e <= TOL


def test_sinc_gradient_parity():
    """fd_gradient with sinc points vs the oracle's gradient and misfit."""
    need_gpu()
    c = case((34, 29, 25), 8, 4, 160, seed=8, nsrc=1, nrec=6)
    c["sinc"] = 3
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    v_true = vp.copy()
    v_true[8:26, 8:30, 8:34] *= 1.1
    wav = c["wav"].astype(np.float64)
    d_obs, *_ = oracle.forward(og, v_true, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], sinc_radius=3)
    J, grad, _ = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], d_obs, sinc_radius=3)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    mis, gm, _, _ = g.gradient(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"],
                               torch.from_numpy(d_obs.astype(np.float32)).to(dev), c["dt"], checkpoint_every=13)
    torch.cuda.synchronize()
    eJ = abs(float(mis.item()) - J) / J
    eg = rel_l2(gm.cpu().numpy(), grad)
    print("sinc gradient: misfit %.3e grad %.3e" % (eJ, eg), flush=True)
    assert eJ <= TOL
    assert_field(gm.cpu().numpy(), grad, TOL, "sinc gradient")


def test_sinc_binomial_gradient_nodes_outside_the_grid():
    """Binomial schedule with sinc nodes outside the padded grid (radius 4 >
    nbl 2, points within a cell of the grid's corners): the last trace row
    is sampled from the bracket step's out-of-place output, where a dropped
    node reads the zero column with weight 0.  The workspace is carved from
    memory that held NaN, so a column left unzeroed would poison the traces,
    misfit and gradient.  Against the oracle and the fixed interval."""
    need_gpu()
    c = case((30, 27, 23), 8, 2, 90, seed=31, nsrc=1, nrec=6)
    c["sinc"] = 4
    _edge_points(c, 4)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    v_true = 1.1 * vp   # a residual of the traces' own size (points at the corners: no local block)
    wav = c["wav"].astype(np.float64)
    d_obs, *_ = oracle.forward(og, v_true, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], sinc_radius=4)
    J, grad, rec_o = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], d_obs, sinc_radius=4)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    obs = torch.from_numpy(d_obs.astype(np.float32)).to(dev)
    w = torch.from_numpy(c["wav"]).to(dev)
    ws = g.gradient_workspace_bytes(c["nt"], len(c["rec"]), binomial_slots=3)
    poison = torch.full((ws // 4 + 4096,), float("nan"), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    del poison   # the caching allocator hands this block to the gradient's workspace
    m1, g1, r1, _ = g.gradient(c["src"], w, c["rec"], obs, c["dt"], binomial_slots=3)
    m2, g2, r2, _ = g.gradient(c["src"], w, c["rec"], obs, c["dt"], checkpoint_every=20)
    torch.cuda.synchronize()
    assert np.isfinite(m1.item()) and abs(m1.item() - J) <= TOL * J
    assert_traces(r1.cpu().numpy(), rec_o, TOL, "sinc binomial")
    assert_field(g1.cpu().numpy(), grad, TOL, "sinc binomial gradient")
    assert torch.equal(r1, r2) and torch.equal(g1, g2)


def test_sinc_through_server():
    need_gpu()
    from paper_1906_10811_amd import Server
    c = case((40, 36, 30), 8, 5, 80, seed=12, nsrc=1, nrec=16)
    want, *_ = oracle_forward(dict(c, sinc=4))
    srv = Server(1 << 30, max_slots=2)
    out, info = srv.wait(srv.submit(shape=c["shape"], spacing=c["spacing"], origin=c["origin"],
                                    space_order=c["so"], nbl=c["nbl"], vp=c["v"], src_xyz=c["src"],
                                    wavelet=c["wav"], rec_xyz=c["rec"], dt=c["dt"], sinc_radius=4),
                         timeout=120.0)
    srv.close()
    e = rel_l2(out, want)
    print("sinc via server: %.3e" % e, flush=True)
    assert info["status"] == 0 and e <= TOL


def test_sinc_rejects_bad_radius():
    need_gpu()
    from paper_1906_10811_amd import FDError
    c = case((20, 20), 4, 2, 10, seed=1)
    for r in (-1, 9):
        with pytest.raises(FDError):
            gpu_grid(c, sinc_radius=r)
