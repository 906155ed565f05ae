"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Gate (float32 arithmetic): relative L2 error <= 1e-5 over all receivers x
samples and over the final wavefield, and element-wise bars beside it: each
receiver's trace and each field's largest pointwise error (gpu_common).
Gradient and misfit: 1e-5 as well.  Cases span several x/y tiles and
z chunks with ragged tails, every space order 2..16, damping layers,
off-grid sources and receivers, and 2D and 3D grids.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import (assert_field, assert_traces, case, gpu_forward, gpu_grid, need_gpu, oracle_forward,
                        rel_l2, torch)

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _print(name, **kv):
    print(name, " ".join("%s=%.3e" % (k, v) if isinstance(v, float) else "%s=%s" % (k, v)
                         for k, v in kv.items()), flush=True)


def test_acoustic2d_101_workload():
    """2D 101x101, so 4, v 1.5 km/s, 200 steps, Courant 0.4, on-grid source
    and receivers: traces and final field vs the FP64 oracle."""
    need_gpu()
    w = synth.workload("acoustic2d_101")
    c = dict(shape=w["shape"], spacing=w["spacing"], origin=w["origin"], so=w["space_order"],
             nbl=w["nbl"], nt=w["nt"], v=synth.velocity(w), src=w["src"], rec=w["rec"], dt=w["dt"],
             wav=synth.wavelets(w))
    c["og"] = oracle.Grid(c["shape"], c["spacing"], c["origin"], c["so"], c["nbl"])
    want, u_nt, _, _ = oracle_forward(c)
    g, (rec, state) = gpu_forward(c, save_state=True)
    assert_traces(rec.cpu().numpy(), want, TOL, "acoustic2d_101")
    assert_field(state[0].cpu().numpy(), u_nt, TOL, "acoustic2d_101")


@pytest.mark.parametrize("so", [2, 4, 6, 8, 10, 12, 14, 16])
@pytest.mark.parametrize("zchunk", [0, 7])
@pytest.mark.parametrize("tile_x", [64, 32, 96])
def test_3d_every_space_order(so, zchunk, tile_x):
    """One step per launch.  70x37x29 + 5-point layer (80 x 47 x 39 padded): 64 x 16 tiles give 2
    x tiles and 3 y tiles, 32 x 32 tiles 3 and 2, all ragged; the mixed
    shape (96) one 64 x 16 column of 3 tiles and a 16-point strip of two
    32 x 32 tiles (so 14 and 16: 32 x 32 throughout); z chunks of 7 or
    automatic; 3 sources, 9 receivers, 60 steps."""
    need_gpu()
    c = case((70, 37, 29), so, 5, 60, seed=so, nsrc=3, nrec=9)
    want, u_nt, _, _ = oracle_forward(c)
    g = gpu_grid(c, zchunk=zchunk, tile_x=tile_x, time_block=1)
    _, (rec, state) = gpu_forward(c, grid=g, save_state=True)
    assert_traces(rec.cpu().numpy(), want, TOL, "3d so=%d zchunk=%d tile_x=%d" % (so, zchunk, tile_x))
    assert_field(state[0].cpu().numpy(), u_nt, TOL, "3d so=%d zchunk=%d tile_x=%d" % (so, zchunk, tile_x))


@pytest.mark.parametrize("so", [4, 16])
def test_2d_ragged(so):
    need_gpu()
    c = case((67, 133), so, 6, 150, seed=3, nsrc=2, nrec=11)
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, save_state=True)
    assert_traces(rec.cpu().numpy(), want, TOL, "2d so=%d" % so)
    assert_field(state[0].cpu().numpy(), u_nt, TOL, "2d so=%d" % so)


def test_nx_not_multiple_of_four_and_shared_corners():
    """nx' = 67 (partial 4-point groups); two sources in the same cell and a
    receiver on the last grid line (cell N-2, fraction 1)."""
    need_gpu()
    c = case((61, 19, 23), 8, 3, 50, seed=7, nsrc=1, nrec=5)
    s0 = c["src"][0]
    c["src"] = [s0, (s0[0] + 1.0, s0[1] + 0.5, s0[2] - 0.7)]
    c["wav"] = np.concatenate([c["wav"], 0.5 * c["wav"]], axis=1)
    ext = [(n - 1) * hh for n, hh in zip(c["shape"], c["spacing"])]
    c["rec"][0] = [o + e for o, e in zip(c["origin"], ext)]
    want, u_nt, _, _ = oracle_forward(c)
    _, (rec, state) = gpu_forward(c, save_state=True)
    assert_traces(rec.cpu().numpy(), want, TOL, "ragged nx")
    assert_field(state[0].cpu().numpy(), u_nt, TOL, "ragged nx")


def test_initial_state_and_resume_bitwise():
    """Running 40 + 30 steps with the saved state equals 70 steps bitwise,
    and an initial state given by the caller matches the oracle."""
    need_gpu()
    c = case((40, 33, 26), 8, 4, 70, seed=11, nsrc=1, nrec=6)
    dev = torch.device("cuda:0")
    g = gpu_grid(c)
    wav = torch.from_numpy(c["wav"]).to(dev)
    full = g.forward(c["src"], wav, c["rec"], c["dt"])
    r1, st = g.forward(c["src"], wav[:40].contiguous(), c["rec"], c["dt"], save_state=True)
    r2 = g.forward(c["src"], wav[40:].contiguous(), c["rec"], c["dt"], u0=st[0], u_prev=st[1])
    torch.cuda.synchronize()
    both = torch.cat([r1, r2]).cpu().numpy()
    assert np.array_equal(both, full.cpu().numpy())
    rng = np.random.default_rng(2)
    u0 = rng.standard_normal(c["og"].array_shape) * 1e-3
    um = u0 * 0.99
    c["nt"] = 25
    c["wav"] = c["wav"][:25].copy()
    want, u_nt, _, _ = oracle_forward(c, u0=u0, u_prev=um)
    rec, state = g.forward(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"], c["dt"],
                           u0=torch.from_numpy(u0).float().to(dev), u_prev=torch.from_numpy(um).float().to(dev),
                           save_state=True)
    torch.cuda.synchronize()
    assert_traces(rec.cpu().numpy(), want, TOL, "caller state")
    assert_field(state[0].cpu().numpy(), u_nt, TOL, "caller state")


def test_adjoint_parity_and_dot_product():
    """fd_adjoint vs the oracle's O11 on a random residual, and the dot test
    <F w, r> = <w, F^T r> in float32: with r = F w for band-limited w (the
    inner product is then not a cancellation of random signs) the relative
    gap is <= 1e-6; for white-noise w, r the gap is measured against
    |F w| |r|, the scale of the rounding in either product."""
    need_gpu()
    c = case((48, 37, 30), 8, 5, 70, seed=5, nsrc=2, nrec=8)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(1)
    w = rng.standard_normal((c["nt"], 2)).astype(np.float32)
    r = rng.standard_normal((c["nt"], 8)).astype(np.float32)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    want, _ = oracle.adjoint(og, vp, sig, c["dt"], c["nt"], c["src"], c["rec"], r.astype(np.float64))
    got = g.adjoint(c["src"], c["rec"], torch.from_numpy(r).to(dev), c["dt"])
    Fw = g.forward(c["src"], torch.from_numpy(w).to(dev), c["rec"], c["dt"])
    torch.cuda.synchronize()
    e = rel_l2(got.cpu().numpy(), want)
    fw = Fw.cpu().numpy().astype(np.float64)
    lhs = float(np.sum(fw * r))
    rhs = float(np.sum(w.astype(np.float64) * got.cpu().numpy()))
    dot_white = abs(lhs - rhs) / (np.linalg.norm(fw) * np.linalg.norm(r))
    # band-limited wavelets, r = F w
    wb = c["wav"]
    Fb = g.forward(c["src"], torch.from_numpy(wb).to(dev), c["rec"], c["dt"])
    FtFb = g.adjoint(c["src"], c["rec"], Fb, c["dt"])
    torch.cuda.synchronize()
    fb = Fb.cpu().numpy().astype(np.float64)
    a1 = float(np.sum(fb * fb))
    a2 = float(np.sum(wb.astype(np.float64) * FtFb.cpu().numpy()))
    dot = abs(a1 - a2) / abs(a1)
    _print("adjoint", rel=e, dot=dot, dot_white=dot_white)
    assert_traces(got.cpu().numpy(), want, TOL, "adjoint F^T r")
    assert dot <= 1e-6
    assert dot_white <= 1e-6


def _gradient_case():
    """200 steps, so 8, damped heterogeneous medium; the observed data come
    from a model 10% faster in a block on the wave path, so the residual is
    far above float32 rounding."""
    c = case((34, 29, 25), 8, 4, 200, seed=8, nsrc=1, nrec=6)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    v_true = vp.copy()
    v_true[8:26, 8:30, 8:34] *= 1.1
    d_obs, *_ = oracle.forward(og, v_true, sig, c["dt"], c["nt"], c["src"], c["wav"].astype(np.float64), c["rec"])
    return c, vp, sig, d_obs.astype(np.float32)


@pytest.mark.parametrize("K", [7, 500])
def test_gradient_parity(K):
    """fd_gradient vs the oracle's O12 gradient and misfit (checkpoint
    interval 7 gives ragged segments; 500 > nt keeps every field)."""
    need_gpu()
    c, vp, sig, d_obs = _gradient_case()
    og = c["og"]
    J, grad, _ = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], c["wav"].astype(np.float64),
                                 c["rec"], d_obs.astype(np.float64))
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    mis, gm, rec, _ = g.gradient(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"],
                                 torch.from_numpy(d_obs).to(dev), c["dt"], checkpoint_every=K)
    torch.cuda.synchronize()
    eJ = abs(float(mis.item()) - J) / J
    eg = rel_l2(gm.cpu().numpy(), grad)
    _print("gradient K=%d" % K, J=J, eJ=eJ, grad=eg)
    assert eJ <= TOL
    assert_field(gm.cpu().numpy(), grad, TOL, "gradient K=%d" % K)
    # with respect to the velocity: the library applies dm/dv = -2 / v^3
    _, gv, _, _ = g.gradient(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"],
                             torch.from_numpy(d_obs).to(dev), c["dt"], checkpoint_every=K, wrt_velocity=True)
    torch.cuda.synchronize()
    assert_field(gv.cpu().numpy(), grad * (-2.0 / vp ** 3), TOL, "gradient wrt v K=%d" % K)


def test_gradient_parity_so14():
    """Space order 14, where the bracket mode runs the z queue that rotates
    by index (2r + 1 = 15 planes, the plane loop unrolled 15 times): fixed
    interval 13 (ragged last segment) and every bracket resident, against
    the oracle's gradient; the two schedules agree bitwise."""
    need_gpu()
    c = case((30, 27, 23), 14, 4, 120, seed=21, nsrc=1, nrec=6)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    v_true = vp.copy()
    v_true[8:20, 8:22, 8:26] *= 1.1
    wav = c["wav"].astype(np.float64)
    d_obs, *_ = oracle.forward(og, v_true, sig, c["dt"], c["nt"], c["src"], wav, c["rec"])
    J, grad, _ = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], d_obs)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    obs = torch.from_numpy(d_obs.astype(np.float32)).to(dev)
    w = torch.from_numpy(c["wav"]).to(dev)
    m1, g1, _, _ = g.gradient(c["src"], w, c["rec"], obs, c["dt"], checkpoint_every=13)
    m2, g2, _, _ = g.gradient(c["src"], w, c["rec"], obs, c["dt"], checkpoint_every=c["nt"])
    torch.cuda.synchronize()
    eJ = abs(float(m1.item()) - J) / J
    eg = rel_l2(g1.cpu().numpy(), grad)
    _print("gradient so 14", eJ=eJ, grad=eg, schedules_bitwise=int(torch.equal(g1, g2)))
    assert eJ <= TOL
    assert_field(g1.cpu().numpy(), grad, TOL, "gradient so 14")
    assert torch.equal(m1, m2) and torch.equal(g1, g2)


@pytest.mark.parametrize("K", [9, 1000])
def test_gradient_parity_2d(K):
    """The 2D kernel's bracket and imaging epilogues: fd_gradient on a 2D
    damped case vs the oracle (ragged segments, and every bracket kept)."""
    need_gpu()
    c = case((61, 47), 8, 5, 180, seed=12, nsrc=1, nrec=9)
    og = c["og"]
    vp = oracle.pad_velocity(og, c["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    v_true = vp.copy()
    v_true[15:35, 20:45] *= 1.1
    wav = c["wav"].astype(np.float64)
    d_obs, *_ = oracle.forward(og, v_true, sig, c["dt"], c["nt"], c["src"], wav, c["rec"])
    J, grad, _ = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], wav, c["rec"], d_obs)
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    mis, gm, _, _ = g.gradient(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"],
                               torch.from_numpy(d_obs.astype(np.float32)).to(dev), c["dt"], checkpoint_every=K)
    torch.cuda.synchronize()
    eJ = abs(float(mis.item()) - J) / J
    eg = rel_l2(gm.cpu().numpy(), grad)
    _print("gradient 2d K=%d" % K, J=J, eJ=eJ, grad=eg)
    assert eJ <= TOL
    assert_field(gm.cpu().numpy(), grad, TOL, "gradient 2d K=%d" % K)


def test_gradient_resident_brackets_equal_recompute():
    """checkpoint_every >= nt keeps every bracket from the forward pass (no
    recompute); the result is bitwise the recomputing schedule's."""
    need_gpu()
    c, vp, sig, d_obs = _gradient_case()
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    obs = torch.from_numpy(d_obs).to(dev)
    m1, g1, r1, a1 = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=13, want_src_adj=True)
    m2, g2, r2, a2 = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=c["nt"], want_src_adj=True)
    torch.cuda.synchronize()
    _print("resident brackets", grad_bitwise=int(torch.equal(g1, g2)), traces_bitwise=int(torch.equal(r1, r2)))
    assert torch.equal(r1, r2) and torch.equal(m1, m2) and torch.equal(g1, g2) and torch.equal(a1, a2)


def test_gradient_on_a_side_stream_reuses_its_workspace():
    """fd_gradient enqueued on a caller's stream: the result equals the
    current-stream result, and a later call on that stream reuses the
    workspace block whichever stream is current at the call (a block that
    belongs to another stream would not be handed out again)."""
    need_gpu()
    c, vp, sig, d_obs = _gradient_case()
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    obs = torch.from_numpy(d_obs).to(dev)
    m0, g0, _, _ = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=c["nt"])
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    m1, g1, _, _ = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=c["nt"], stream=side)
    torch.cuda.synchronize()
    reserved = torch.cuda.memory_reserved()
    with torch.cuda.stream(side):
        m2, g2, _, _ = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=c["nt"], stream=side)
    torch.cuda.synchronize()
    ws = g.gradient_workspace_bytes(c["nt"], len(c["rec"]), checkpoint_every=c["nt"])
    grown = torch.cuda.memory_reserved() - reserved
    _print("side stream", workspace=ws, reserved_growth=grown)
    # the small outputs may open a new pool segment on the side stream; a
    # second workspace would add at least its own size
    assert grown < ws // 2
    assert torch.equal(m0, m1) and torch.equal(g0, g1) and torch.equal(m1, m2) and torch.equal(g1, g2)


@pytest.mark.parametrize("slots", [0, 3, 9])
def test_gradient_binomial_schedule(slots):
    """The binomial checkpoint schedule (snapshot slots 0, 3, 9): misfit,
    gradient, traces and F^T residual against the oracle's O12 / O11, and
    against the fixed-interval schedule (the same kernels compute the same
    levels, only the order of recomputation differs)."""
    need_gpu()
    c, vp, sig, d_obs = _gradient_case()
    og = c["og"]
    wav64 = c["wav"].astype(np.float64)
    J, grad, rec_o = oracle.gradient(og, vp, sig, c["dt"], c["nt"], c["src"], wav64, c["rec"],
                                     d_obs.astype(np.float64))
    adj_o, _ = oracle.adjoint(og, vp, sig, c["dt"], c["nt"], c["src"], c["rec"], rec_o - d_obs.astype(np.float64))
    g = gpu_grid(c)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    obs = torch.from_numpy(d_obs).to(dev)
    m1, g1, r1, a1 = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=50, want_src_adj=True)
    m2, g2, r2, a2 = g.gradient(c["src"], wav, c["rec"], obs, c["dt"], binomial_slots=slots, want_src_adj=True)
    torch.cuda.synchronize()
    eg = rel_l2(g2.cpu().numpy(), g1.cpu().numpy())
    _print("binomial slots=%d" % slots, grad=eg, misfit=abs(m2.item() - m1.item()) / m1.item(),
           traces_bitwise=int(torch.equal(r1, r2)), grad_bitwise=int(torch.equal(g1, g2)))
    assert abs(m2.item() - J) <= TOL * J
    assert_field(g2.cpu().numpy(), grad, TOL, "binomial slots=%d gradient" % slots)
    assert_traces(r2.cpu().numpy(), rec_o, TOL, "binomial slots=%d" % slots)
    assert_traces(a2.cpu().numpy(), adj_o, TOL, "binomial slots=%d F^T r" % slots)
    assert torch.equal(r1, r2)
    assert abs(m2.item() - m1.item()) <= 1e-14 * m1.item()
    assert eg <= 1e-12
    assert rel_l2(a2.cpu().numpy(), a1.cpu().numpy()) <= 1e-12


def test_gradient_finite_differences_on_gpu():
    """<g_m, dm> from fd_gradient against central differences of the misfit
    computed by fd_forward on the padded grid, float32 throughout.  The data
    are zero, so the residual is the traces themselves and the float32
    rounding of J stays far below its change under the perturbation."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    c, vp, sig, _ = _gradient_case()
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    obs = torch.zeros((c["nt"], len(c["rec"])), dtype=torch.float32, device=dev)

    # sigma_max held fixed: its default follows v_max, which the perturbation moves
    smax = oracle.sigma_max_default(c["og"], float(vp.max()))

    def grid(v):
        return Grid(c["shape"], c["spacing"], torch.from_numpy(v.astype(np.float32)).to(dev), space_order=c["so"],
                    nbl=c["nbl"], origin=c["origin"], vp_padded=True, damp_max=smax)

    def J(v):
        g = grid(v)
        rec = g.forward(c["src"], wav, c["rec"], c["dt"])
        torch.cuda.synchronize()
        r = rec.double()
        return 0.5 * float((r * r).sum())

    g0 = grid(vp)
    _, gm, _, _ = g0.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=50)
    torch.cuda.synchronize()
    gm = gm.cpu().numpy()
    m0 = 1.0 / vp ** 2
    rng = np.random.default_rng(4)
    dm = m0 * 0.02 * rng.standard_normal(m0.shape)
    eps = 0.5
    fd = (J(1.0 / np.sqrt(m0 + eps * dm)) - J(1.0 / np.sqrt(m0 - eps * dm))) / (2 * eps)
    an = float(np.sum(gm * dm))
    _print("gradient FD", fd=fd, an=an, rel=abs(fd - an) / abs(an))
    assert abs(fd - an) <= 1e-3 * abs(an)


def test_errors_are_reported():
    need_gpu()
    from paper_1906_10811_amd import FDError, _lib
    c = case((20, 18, 16), 4, 2, 10, seed=1)
    g = gpu_grid(c, max_rec=8)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    with pytest.raises(FDError) as e:
        g.forward(c["src"], wav, c["rec"], 1.001 * g.critical_dt)
    assert e.value.code == _lib.FD_ERR_UNSTABLE
    with pytest.raises(FDError) as e:
        g.forward([(-1.0, 0.0, 0.0)], wav, c["rec"], c["dt"])
    assert e.value.code == _lib.FD_ERR_ARG
    with pytest.raises(FDError) as e:
        g.forward(c["src"], wav, np.zeros((9, 3)) + 10.0, c["dt"])
    assert e.value.code == _lib.FD_ERR_ARG
    # the grid still works after rejected calls
    _, rec = gpu_forward(c, grid=g)
    want, *_ = oracle_forward(c)
    assert_traces(rec.cpu().numpy(), want, TOL, "after errors")
    with pytest.raises(FDError) as e:
        g.gradient(c["src"], wav, c["rec"], torch.zeros((c["nt"], len(c["rec"])), device=dev), c["dt"],
                   checkpoint_every=-3)
    assert e.value.code == _lib.FD_ERR_ARG
