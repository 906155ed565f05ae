"""16-bit value-and-difference storage (f16_diff, bf16_diff) against the FP64
oracle, against the two-level 16-bit storages, across tile shapes, across
split runs and through the server.

The leapfrog update advances the difference d = u^n - u^{n-1}: with both
levels stored in 16 bits, d is the difference of two rounded numbers of
nearly equal size and keeps few significant bits where the time step is
small against the local period, so the error compounds step after step.
Stored as a field of its own, d keeps 16-bit relative precision.  A plain
2D numpy evaluation of the same recursion with the stored fields rounded to
bfloat16 (layered model, 256^2 + 80, so 8, 400 steps) gives a trace error
against float64 of 3.6e-1 for two bfloat16 levels and 1.1e-2 for the value
and difference; the bars below are stated per storage from that ratio.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import case, gpu_forward, gpu_grid, need_gpu, oracle_forward, rel_l2, torch

pytestmark = pytest.mark.gpu


def _small(name, shape=(72, 66, 60), nbl=12, nt=400):
    """A benchmark workload's medium, step and wavelet on a smaller grid:
    source at the top centre, 40 receivers along x 20 m down."""
    cx, cy = (shape[0] - 1) * 5.0, (shape[1] - 1) * 5.0
    w = synth.workload(name, shape=shape, nbl=nbl, nt=nt, src=[(cx + 5.0, cy + 5.0, 20.0)],
                       rec=synth.line_receivers(40, 0.0, 2 * cx, (cy, 20.0), 3))
    return w, synth.velocity(w)


@pytest.mark.parametrize("name", ["layered3d_256", "grf3d_512"])
def test_difference_storage_error_vs_fp64(name):
    """The layered and the GRF medium, so 8, 400 steps at Courant 0.4: the
    difference forms against the FP64 oracle, each within its bar and below
    the two-level form of the same type."""
    need_gpu()
    from paper_1906_10811_amd import Grid
    w, v = _small(name)
    g0 = oracle.Grid(w["shape"], w["spacing"], w["origin"], w["space_order"], w["nbl"])
    vp = oracle.pad_velocity(g0, v)
    sig = oracle.damping(g0, oracle.sigma_max_default(g0, float(vp.max())))
    wav = synth.wavelets(w)
    want, *_ = oracle.forward(g0, vp, sig, w["dt"], w["nt"], w["src"], wav.astype(np.float64), w["rec"])
    dev = torch.device("cuda:0")
    errs = {}
    for st in ("f16", "f16_diff", "bf16", "bf16_diff"):
        g = Grid(w["shape"], w["spacing"], torch.from_numpy(v).to(dev), space_order=w["space_order"],
                 nbl=w["nbl"], storage=st)
        rec = g.forward(w["src"], torch.from_numpy(wav).to(dev), w["rec"], w["dt"])
        torch.cuda.synchronize()
        errs[st] = rel_l2(rec.cpu().numpy(), want)
        g.close()
    print("%s storage error vs FP64 oracle:" % name, {k: "%.2e" % e for k, e in errs.items()}, flush=True)
    assert errs["bf16_diff"] <= 1e-2
    assert errs["bf16_diff"] * 2 <= errs["bf16"]
    assert errs["f16_diff"] <= 1e-3
    assert errs["f16_diff"] <= errs["f16"]


@pytest.mark.parametrize("storage", ["f16_diff", "bf16_diff"])
def test_difference_storage_split_runs_and_caller_state(storage):
    """33 + 28 steps through save_state / u0 / u_prev against 61 in one run:
    the saved previous level is u - d rounded once in float32 and the
    restarted difference u0 - u_prev recovers d exactly unless the two
    differ by more than float32's headroom over 16 bits, so the traces agree
    to far below the storage error.  A caller's initial state (white noise:
    no smooth part, so every stored level is rounded afresh) is checked
    against the oracle at three times the random walk of one rounding per
    step, sqrt(nt) eps / sqrt(12) relative with eps = 2^-10 (f16) or 2^-7
    (bf16)."""
    need_gpu()
    c = case((70, 33, 26), 8, 4, 61, seed=11, nsrc=2, nrec=6)
    dev = torch.device("cuda:0")
    g = gpu_grid(c, storage=storage)
    wav = torch.from_numpy(c["wav"]).to(dev)
    full = g.forward(c["src"], wav, c["rec"], c["dt"])
    ra, st = g.forward(c["src"], wav[:33].contiguous(), c["rec"], c["dt"], save_state=True)
    rb = g.forward(c["src"], wav[33:].contiguous(), c["rec"], c["dt"], u0=st[0], u_prev=st[1])
    torch.cuda.synchronize()
    e = rel_l2(torch.cat([ra, rb]).cpu().numpy(), full.cpu().numpy())
    print("%s split vs one run: %.3e" % (storage, e), flush=True)
    assert e <= 1e-5
    rng = np.random.default_rng(3)
    u0 = rng.standard_normal(c["og"].array_shape) * 1e-3
    um = 0.98 * u0
    c["nt"] = 25
    c["wav"] = c["wav"][:25].copy()
    want, u_nt, _, _ = oracle_forward(c, u0=u0, u_prev=um)
    rec, state = g.forward(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"], c["dt"],
                           u0=torch.from_numpy(u0).float().to(dev), u_prev=torch.from_numpy(um).float().to(dev),
                           save_state=True)
    torch.cuda.synchronize()
    eps = 2.0 ** -10 if storage == "f16_diff" else 2.0 ** -7
    bar = 3.0 * np.sqrt(c["nt"]) * eps / np.sqrt(12.0)
    er, ef = rel_l2(rec.cpu().numpy(), want), rel_l2(state[0].cpu().numpy(), u_nt)
    print("%s caller state vs oracle: traces %.3e, field %.3e (bar %.1e)" % (storage, er, ef, bar), flush=True)
    assert er <= bar and ef <= bar
    g.close()


def test_difference_storage_through_the_server_and_rejections():
    """Server requests with the difference storages are bitwise their lone
    fd_forward runs; the gradient (float32 only) refuses them."""
    need_gpu()
    from paper_1906_10811_amd import Server
    from paper_1906_10811_amd._lib import FDError
    c = case((60, 44, 30), 8, 5, 45, seed=19, nsrc=1, nrec=9)
    alone = {}
    for st in ("f16_diff", "bf16_diff"):
        g = gpu_grid(c, storage=st)
        _, rec = gpu_forward(c, grid=g)
        alone[st] = rec.cpu().numpy()
        if st == "f16_diff":
            dev = torch.device("cuda:0")
            obs = torch.zeros((c["nt"], len(c["rec"])), device=dev)
            with pytest.raises(FDError):
                g.gradient(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"], obs, c["dt"])
        g.close()
    srv = Server(1 << 30, max_slots=2, steps_per_round=7)
    kw = dict(shape=c["shape"], spacing=c["spacing"], origin=c["origin"], space_order=c["so"], nbl=c["nbl"],
              vp=c["v"], src_xyz=c["src"], wavelet=c["wav"], rec_xyz=c["rec"], dt=c["dt"])
    ids = {st: srv.submit(storage=st, **kw) for st in alone}
    for st, rid in ids.items():
        out, info = srv.wait(rid, timeout=120.0)
        assert info["status"] == 0
        assert np.array_equal(out, alone[st]), st
    srv.close()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_adjoint_on_a_difference_grid_is_the_two_level_adjoint(storage):
    """fd_adjoint keeps two 16-bit levels whatever the forward storage, so on
    a difference-storage grid it is bitwise the adjoint of the two-level grid
    of the same type."""
    need_gpu()
    c = case((50, 40, 30), 8, 5, 40, seed=23, nsrc=2, nrec=8)
    dev = torch.device("cuda:0")
    res = torch.from_numpy(np.random.default_rng(2).standard_normal((c["nt"], len(c["rec"]))).astype(np.float32)).to(dev)
    out = []
    for st in (storage, storage + "_diff"):
        g = gpu_grid(c, storage=st)
        out.append(g.adjoint(c["src"], c["rec"], res, c["dt"]))
        torch.cuda.synchronize()
        g.close()
    assert torch.equal(out[0], out[1])


def test_difference_storage_with_windowed_sinc_points():
    """Kaiser-windowed sinc sources and receivers (half-width 3, 216 nodes)
    with value-and-difference storage, against the FP64 oracle at the
    storage bars."""
    need_gpu()
    c = case((60, 50, 40), 8, 6, 60, seed=29, nsrc=2, nrec=9)
    c["sinc"] = 3
    want, *_ = oracle_forward(c)
    for st, bar in (("f16_diff", 1e-3), ("bf16_diff", 1e-2)):
        g = gpu_grid(c, storage=st)
        _, rec = gpu_forward(c, grid=g)
        e = rel_l2(rec.cpu().numpy(), want)
        print("%s sinc 3 vs FP64: %.3e" % (st, e), flush=True)
        assert e <= bar, (st, e)
        g.close()
