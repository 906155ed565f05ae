"""The three further forms against the FP64 oracle: 16-bit wavefield storage
(error stated per storage type), the differentiable modelling operator
behind torch.autograd, and full-size runs in the launch configuration the
benchmark times."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu


def _grf_case(shape=(72, 66, 60), nbl=12, nt=400, so=8, seed=1):
    h = (10.0, 10.0, 10.0)
    v = synth.grf_model(shape, h, seed=seed)
    dt = 0.4 * 10.0 / synth.VMAX
    src = [((shape[0] - 1) * 5.0 + 5.0, (shape[1] - 1) * 5.0 + 5.0, 20.0)]
    rec = synth.line_receivers(40, 0.0, (shape[0] - 1) * 10.0, ((shape[1] - 1) * 5.0, 20.0), 3)
    wav = synth.ricker(nt, dt, 15.0).astype(np.float32)[:, None]
    return dict(shape=shape, h=h, v=v, dt=dt, src=src, rec=rec, wav=wav, nbl=nbl, so=so, nt=nt)


def test_reduced_precision_storage_error_vs_fp64():
    """GRF medium, so 8, 400 steps.  FP32 meets the 1e-5 gate; F16 (scaled
    automatically) and BF16 storage keep FP32 arithmetic and their trace
    error against the FP64 oracle is reported and bounded.  With a weak
    source (1e-4), unscaled half precision loses the field to underflow and
    a matching amp_scale restores it."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    c = _grf_case()
    g0 = oracle.Grid(c["shape"], c["h"], (0.0, 0.0, 0.0), c["so"], c["nbl"])
    vp = oracle.pad_velocity(g0, c["v"])
    sig = oracle.damping(g0, oracle.sigma_max_default(g0, float(vp.max())))
    want, *_ = oracle.forward(g0, vp, sig, c["dt"], c["nt"], c["src"], c["wav"].astype(np.float64), c["rec"])
    dev = torch.device("cuda:0")
    auto = 2.0 ** round(math.log2(1000.0 / (c["dt"] ** 2 * float(vp.max()) ** 2)))
    errs = {}
    for label, st, scale, amp in (("f32", "f32", 0.0, 1.0), ("f16 auto", "f16", 0.0, 1.0),
                                  ("bf16", "bf16", 0.0, 1.0), ("f16 weak, scale 1", "f16", 1.0, 1e-4),
                                  ("f16 weak, scale 1e4*auto", "f16", 1e4 * auto, 1e-4)):
        g = Grid(c["shape"], c["h"], torch.from_numpy(c["v"]).to(dev), space_order=c["so"], nbl=c["nbl"],
                 storage=st, amp_scale=scale)
        rec = g.forward(c["src"], torch.from_numpy(c["wav"] * amp).to(dev), c["rec"], c["dt"])
        torch.cuda.synchronize()
        errs[label] = rel_l2(rec.cpu().numpy() / amp, want)
        g.close()
    print("storage error vs FP64 oracle:", {k: "%.2e" % v for k, v in errs.items()})
    assert errs["f32"] <= 1e-5
    assert errs["f16 auto"] <= 5e-3
    assert errs["bf16"] <= 5e-2
    assert errs["f16 weak, scale 1"] > 10 * errs["f16 weak, scale 1e4*auto"]
    assert errs["f16 weak, scale 1e4*auto"] <= 5e-3


@pytest.mark.parametrize("sinc", [0, 3])
def test_autograd_modeling_matches_oracle_gradient(sinc):
    """loss = 1/2 |F(v, w) - d|^2 through torch.autograd: d loss/d v equals
    the oracle's O12 gradient chained through m = 1/v^2, and d loss/d w
    equals the oracle's adjoint of the residual."""
    need_gpu()
    from paper_1906_10811_amd import modeling
    shape, h, so, nbl, nt = (30, 26, 22), (10.0, 10.0, 10.0), 4, 4, 160
    g0 = oracle.Grid(shape, h, (0.0, 0.0, 0.0), so, nbl)
    v = synth.layered_model(shape, h, seed=4)
    vp = oracle.pad_velocity(g0, v)
    sig = oracle.damping(g0, oracle.sigma_max_default(g0, float(vp.max())))
    dt = 0.4 * 10.0 / synth.VMAX
    src = [(145.0, 125.0, 20.0)]
    rec = synth.line_receivers(8, 0.0, 290.0, (125.0, 20.0), 3)
    wav = synth.ricker(nt, dt, 30.0)[:, None]
    v_true = vp.copy()
    v_true[8:20, :, :] *= 1.08
    d_obs, *_ = oracle.forward(g0, v_true, sig, dt, nt, src, wav, rec, sinc_radius=sinc)
    J, g_m, rec0 = oracle.gradient(g0, vp, sig, dt, nt, src, wav, rec, d_obs, sinc_radius=sinc)
    r = rec0 - d_obs
    g_w, _ = oracle.adjoint(g0, vp, sig, dt, nt, src, rec, r, sinc_radius=sinc)
    dev = torch.device("cuda:0")
    vt = torch.tensor(vp, dtype=torch.float32, device=dev, requires_grad=True)
    wt = torch.tensor(wav, dtype=torch.float32, device=dev, requires_grad=True)
    out = modeling(vt, wt, shape, h, so, nbl, src, rec, dt, checkpoint_every=30, sinc_radius=sinc)
    loss = 0.5 * ((out.double() - torch.tensor(d_obs, device=dev)) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    g_v_want = g_m * (-2.0 / vp ** 3)
    ev = rel_l2(vt.grad.cpu().numpy(), g_v_want)
    ew = rel_l2(wt.grad.cpu().numpy(), g_w)
    eJ = abs(float(loss.item()) - J) / J
    print("autograd sinc=%d: loss %.3e, dv %.3e, dw %.3e" % (sinc, eJ, ev, ew))
    # the wavelet gradient is F^T of a float32 residual that is ~10x smaller
    # than the traces it is the difference of: gradient-class gate 1e-4
    assert eJ <= 1e-4 and ev <= 1e-4 and ew <= 1e-4


def _smooth_state(shape_np, seed):
    """Seeded smooth random field (dense padded), for full-size runs whose
    first steps must already carry signal everywhere."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(shape_np).astype(np.float32)
    # separable 3-point smoothing, twice
    for _ in range(2):
        for ax in range(3):
            f = (np.roll(f, 1, ax) + 2 * f + np.roll(f, -1, ax)) / 4
    return f


@pytest.mark.parametrize("name,shape", [("layered3d_256", None), ("grf3d_512", (512, 512, 512)),
                                        ("gradient3d_200", None)])
def test_full_size_in_bench_launch_shape(name, shape):
    """The benchmark's grids (336^3, 592^3 and 280^3 padded, so 8) in their
    automatic launch shape (64 x 16 tiles with a last column of 32 x 32: 16,
    16 and 24 points wide): a few steps from a smooth random state with a
    source firing at its peak, every point of the final field and every
    trace sample against the oracle run on the whole grid."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    w = synth.workload(name, model="layered", nt=4)
    nt = 4 if shape else 6
    h = w["spacing"]
    v = synth.layered_model(w["shape"], h, seed=w["seed"])
    g0 = oracle.Grid(tuple(w["shape"]), h, (0.0, 0.0, 0.0), 8, w["nbl"])
    u0 = _smooth_state(g0.array_shape, 3)
    um = (0.999 * u0).astype(np.float32)
    wav = synth.ricker(nt, w["dt"], 15.0, t0=0.0).astype(np.float32)[:, None] * 1e3
    dev = torch.device("cuda:0")
    g = Grid(w["shape"], h, torch.from_numpy(v).to(dev), space_order=8, nbl=w["nbl"])
    rec, (u_nt, _) = g.forward(w["src"], torch.from_numpy(wav).to(dev), w["rec"], w["dt"],
                               u0=torch.from_numpy(u0).to(dev), u_prev=torch.from_numpy(um).to(dev),
                               save_state=True)
    torch.cuda.synchronize()
    got_u = u_nt.cpu().numpy()
    got_rec = rec.cpu().numpy()
    g.close()
    del u_nt
    vp = oracle.pad_velocity(g0, v)
    sig = oracle.damping(g0, oracle.sigma_max_default(g0, float(vp.max())))
    want_rec, want_u, _, _ = oracle.forward(g0, vp, sig, w["dt"], nt, w["src"], wav.astype(np.float64), w["rec"],
                                            u0=u0, u_prev=um)
    eu = rel_l2(got_u, want_u)
    er = rel_l2(got_rec, want_rec)
    print("full size %s (%s padded), %d steps: field %.3e, traces %.3e" % (name, g0.padded, nt, eu, er))
    assert eu <= 1e-5 and er <= 1e-5


def test_full_size_gradient_schedules_agree():
    """gradient3d_200 as the benchmark runs it (280^3 padded, so 8, 800
    steps, mixed tiles): checkpoints every 50 steps, every bracket resident,
    and the binomial schedule with 16 snapshot slots give bitwise the same
    misfit, gradient and traces."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    w = synth.workload("gradient3d_200")
    v_true = synth.velocity(w)
    v0 = synth.smooth_model(v_true, w["spacing"], 100.0)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(synth.wavelets(w)).to(dev)
    gt = Grid(w["shape"], w["spacing"], torch.from_numpy(v_true).to(dev), space_order=8, nbl=w["nbl"])
    d_obs = gt.forward(w["src"], wav, w["rec"], w["dt"])
    torch.cuda.synchronize()
    gt.close()
    g = Grid(w["shape"], w["spacing"], torch.from_numpy(v0).to(dev), space_order=8, nbl=w["nbl"])
    assert g.tile_strip == 24
    m1, g1, r1, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], checkpoint_every=w["checkpoint_every"])
    torch.cuda.synchronize()
    m2, g2, r2, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], checkpoint_every=w["nt"])
    torch.cuda.synchronize()
    same_resident = bool(torch.equal(m1, m2) and torch.equal(g1, g2) and torch.equal(r1, r2))
    del g2, r2
    m3, g3, r3, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], binomial_slots=16)
    torch.cuda.synchronize()
    same_binomial = bool(torch.equal(m1, m3) and torch.equal(g1, g3) and torch.equal(r1, r3))
    print("full-size gradient: misfit %.6e, |g| %.6e, resident bitwise %d, binomial bitwise %d" % (
        m1.item(), g1.norm().item(), int(same_resident), int(same_binomial)), flush=True)
    assert math.isfinite(m1.item()) and m1.item() > 0 and g1.norm().item() > 0
    assert same_resident and same_binomial


def test_full_length_properties_layered3d_256():
    """All 1000 steps of layered3d_256 (too long for the oracle): source-
    receiver reciprocity and the adjoint identity hold in float32."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    w = synth.workload("layered3d_256")
    dev = torch.device("cuda:0")
    g = Grid(w["shape"], w["spacing"], torch.from_numpy(synth.velocity(w)).to(dev), space_order=8, nbl=w["nbl"])
    wav = torch.from_numpy(synth.wavelets(w)).to(dev)
    A = w["src"][0]
    B = (2012.5, 1100.0, 180.0)
    r_ab = g.forward([A], wav, [B], w["dt"])
    r_ba = g.forward([B], wav, [A], w["dt"])
    torch.cuda.synchronize()
    e_rec = rel_l2(r_ab.cpu().numpy(), r_ba.cpu().numpy())
    rec = g.forward(w["src"], wav, w["rec"], w["dt"])
    adj = g.adjoint(w["src"], w["rec"], rec, w["dt"])
    torch.cuda.synchronize()
    a1 = float((rec.double() ** 2).sum())
    a2 = float((wav.double() * adj.double()).sum())
    dot = abs(a1 - a2) / a1
    print("layered3d_256, 1000 steps: reciprocity %.3e, dot test %.3e" % (e_rec, dot))
    assert e_rec <= 1e-4
    assert dot <= 1e-6
    assert math.isfinite(a1) and a1 > 0


@pytest.mark.slow
def test_storage_error_growth_over_1500_steps():
    """The precision form at the full step count of the 512^3 GRF workload,
    on a 96^3 + 40 grid the oracle runs in under a minute: trace error
    against the FP64 oracle over the first 500, 1000 and 1500 steps for each
    storage type (float32 stays within the 1e-5 gate over the whole run)."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    shape, h, nbl, nt, so = (96, 96, 96), (10.0, 10.0, 10.0), 40, 1500, 8
    v = synth.grf_model(shape, h, seed=1)
    dt = 0.4 * 10.0 / synth.VMAX
    src = [(475.0 + 5.0, 475.0 + 5.0, 20.0)]
    rec = synth.line_receivers(96, 0.0, 950.0, (475.0, 20.0), 3)
    wav = synth.ricker(nt, dt, 15.0).astype(np.float32)[:, None]
    g0 = oracle.Grid(shape, h, (0.0, 0.0, 0.0), so, nbl)
    vp = oracle.pad_velocity(g0, v)
    sig = oracle.damping(g0, oracle.sigma_max_default(g0, float(vp.max())))
    want, *_ = oracle.forward(g0, vp, sig, dt, nt, src, wav.astype(np.float64), rec)
    dev = torch.device("cuda:0")
    rows = {}
    for st in ("f32", "f16", "bf16"):
        g = Grid(shape, h, torch.from_numpy(v).to(dev), space_order=so, nbl=nbl, storage=st)
        got = g.forward(src, torch.from_numpy(wav).to(dev), rec, dt)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        g.close()
        rows[st] = [rel_l2(got[:n], want[:n]) for n in (500, 1000, 1500)]
    print("trace error vs FP64 over 500/1000/1500 steps:",
          {k: ["%.2e" % e for e in v] for k, v in rows.items()}, flush=True)
    assert max(rows["f32"]) <= 1e-5
    assert max(rows["f16"]) <= 5e-3 and max(rows["bf16"]) <= 5e-2


@pytest.mark.parametrize("storage,tol", [("f16", 1e-2), ("bf16", 5e-2)])
def test_reduced_precision_2d_and_adjoint(storage, tol):
    """16-bit storage through the 2D step kernel (forward) and through the
    3D adjoint (residual injected at the receivers, F^T sampled at the
    sources), each against the FP64 oracle at the per-storage bound."""
    need_gpu()
    from gpu_common import case, gpu_grid, oracle_forward
    c2 = case((90, 77), 8, 6, 150, seed=21, nsrc=2, nrec=11)
    want2, *_ = oracle_forward(c2)
    dev = torch.device("cuda:0")
    g2 = gpu_grid(c2, storage=storage)
    got2 = g2.forward(c2["src"], torch.from_numpy(c2["wav"]).to(dev), c2["rec"], c2["dt"])
    torch.cuda.synchronize()
    e2 = rel_l2(got2.cpu().numpy(), want2)
    g2.close()
    c3 = case((40, 33, 26), 8, 4, 80, seed=22, nsrc=2, nrec=9)
    og = c3["og"]
    vp = oracle.pad_velocity(og, c3["v"])
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    rng = np.random.default_rng(5)
    res = rng.standard_normal((c3["nt"], len(c3["rec"])))
    want3, _ = oracle.adjoint(og, vp, sig, c3["dt"], c3["nt"], c3["src"], c3["rec"], res)
    g3 = gpu_grid(c3, storage=storage)
    got3 = g3.adjoint(c3["src"], c3["rec"], torch.from_numpy(res.astype(np.float32)).to(dev), c3["dt"])
    torch.cuda.synchronize()
    e3 = rel_l2(got3.cpu().numpy(), want3)
    g3.close()
    print("%s: 2D forward %.3e, 3D adjoint %.3e" % (storage, e2, e3), flush=True)
    assert e2 <= tol and e3 <= tol
