"""The benchmark workloads at their full size and full step count against
the FP64 oracle run over the same whole grid: layered3d_256 (336^3 padded,
so 8, 1000 steps; the headline) and the forward pass of gradient3d_200
(280^3 padded, so 8, 800 steps, on the smoothed starting model the gradient
runs on), in the launch configuration the benchmark times.

Traces over all steps are checked globally (relative L2 <= 1e-5) and per
receiver (gpu_common).  The wavefield is checked at a quarter of the run and
at the end, against a bar derived from float32 arithmetic: float32 leapfrog
accumulates rounding into a smooth, low-wavenumber error that grows faster
than the step count.  A plain float32 evaluation of the same recursion
(numpy, a 2D analogue of gradient3d_200: smoothed layered model, 200^2 + 40,
so 8) has a field error against float64 of 1.6e-6, 7.3e-6, 2.2e-5 and
9.5e-5 after 100, 200, 400 and 800 steps, 99 % of its energy below an eighth
of the Nyquist wavenumber; this GPU path measures 7.0e-6 after 200 and 9.0e-5
after 800 steps of gradient3d_200.  The bars are three times that floor:
3e-5 at a quarter of the run, 3e-4 at the end (point by point: largest
error over largest value, the same bars).  The traces, sampled 20 m below
the surface, stay within 1e-5 over the whole run.  Both sides run in two
legs through their initial-state arguments, which gives bitwise the
unsplit run.

The same oracle run of layered3d_256 gives the 16-bit storage forms' error
against FP64 at the headline size, per receiver and per offset band.

The oracle takes about a minute on 16 host cores for layered3d_256 and
half that for the gradient grid."""
import time

import numpy as np
import pytest

import oracle
import synth
from gpu_common import assert_traces, field_errors, need_gpu, rel_l2, torch

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-5


def _oracle_run(w, v):
    """Oracle traces of all nt steps, and the fields at nt // 4 and nt."""
    og = oracle.Grid(tuple(w["shape"]), tuple(w["spacing"]), tuple(w["origin"]), w["space_order"], w["nbl"])
    vp = oracle.pad_velocity(og, v)
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    wav = synth.wavelets(w).astype(np.float64)
    k, nt = w["nt"] // 4, w["nt"]
    t0 = time.perf_counter()
    rec1, a, b, _ = oracle.forward(og, vp, sig, w["dt"], k, w["src"], wav[:k], w["rec"])
    u_k = a.copy()
    rec2, u_nt, _, _ = oracle.forward(og, vp, sig, w["dt"], nt - k, w["src"], wav[k:], w["rec"], u0=a, u_prev=b)
    print("oracle %s: %d steps on %s padded in %.1f s (%d threads)" % (
        w["name"], nt, og.padded, time.perf_counter() - t0, oracle.num_threads()), flush=True)
    return np.concatenate([rec1, rec2]), u_k, u_nt


def _gpu_forward(w, v, split=True, **kw):
    from paper_1906_10811_amd import Grid
    dev = torch.device("cuda:0")
    g = Grid(w["shape"], w["spacing"], torch.from_numpy(v).to(dev), space_order=w["space_order"], nbl=w["nbl"],
             origin=w["origin"], **kw)
    wav = torch.from_numpy(synth.wavelets(w)).to(dev)
    if not split:
        rec = g.forward(w["src"], wav, w["rec"], w["dt"])
        torch.cuda.synchronize()
        g.close()
        return rec.cpu().numpy()
    k = w["nt"] // 4
    r1, (a, b) = g.forward(w["src"], wav[:k].contiguous(), w["rec"], w["dt"], save_state=True)
    u_k = a.cpu().numpy()
    r2, (u_nt, _) = g.forward(w["src"], wav[k:].contiguous(), w["rec"], w["dt"], u0=a, u_prev=b, save_state=True)
    torch.cuda.synchronize()
    out = torch.cat([r1, r2]).cpu().numpy(), u_k, u_nt.cpu().numpy()
    g.close()
    return out


FIELD_QUARTER = 3e-5   # three times the float32 floor at 200-250 steps
FIELD_END = 3e-4       # three times the float32 floor at 800 steps


def _field(got, want, bar, label):
    e, m = field_errors(got, want)
    print("%s field: rel_l2 %.3e, max-abs %.3e (bar %.0e)" % (label, e, m, bar), flush=True)
    assert e <= bar and m <= bar, (label, e, m)


def _check(w, got, want):
    rec, u_k, u_nt = got
    want_rec, want_k, want_nt = want
    label = "%s %d steps" % (w["name"], w["nt"])
    assert_traces(rec, want_rec, TOL, label)
    _field(u_k, want_k, FIELD_QUARTER, "%s, step %d" % (w["name"], w["nt"] // 4))
    _field(u_nt, want_nt, FIELD_END, "%s, step %d" % (w["name"], w["nt"]))


@pytest.fixture(scope="module")
def layered256():
    need_gpu()
    w = synth.workload("layered3d_256")
    w["name"] = "layered3d_256"
    v = synth.velocity(w)
    return w, v, _oracle_run(w, v)


def test_layered3d_256_full_length(layered256):
    """The headline workload, all 1000 steps, float32."""
    w, v, want = layered256
    _check(w, _gpu_forward(w, v), want)


def _per_offset(rec, want, w):
    """Median per-receiver trace error by source-receiver offset band."""
    xs = np.asarray(w["rec"])[:, 0]
    off = np.abs(xs - w["src"][0][0])
    per = np.linalg.norm(rec - want, axis=0) / np.linalg.norm(want, axis=0)
    out = {}
    for lo, hi in ((0, 200), (200, 600), (600, 1200), (1200, 3000)):
        m = (off >= lo) & (off < hi)
        out["%d-%d m" % (lo, hi)] = float(np.median(per[m]))
    return out


@pytest.mark.parametrize("storage,bound", [("f16", 1e-2), ("bf16", 1e-1)])
def test_layered3d_256_16bit_storage_error(layered256, storage, bound):
    """16-bit wavefield storage on the headline workload: trace error
    against the FP64 oracle (not against float32), overall and per offset
    band, printed; bounded per storage type."""
    w, v, (want_rec, _, _) = layered256
    rec = _gpu_forward(w, v, split=False, storage=storage)
    e = rel_l2(rec, want_rec)
    print("layered3d_256 %s vs FP64: %.3e; median per-receiver error by offset %s" % (
        storage, e, {k: "%.2e" % x for k, x in _per_offset(rec, want_rec, w).items()}), flush=True)
    assert e <= bound


def test_gradient3d_200_forward_full_length():
    """The forward pass of the gradient workload, all 800 steps on the
    smoothed starting model."""
    need_gpu()
    w = synth.workload("gradient3d_200")
    w["name"] = "gradient3d_200"
    v0 = synth.smooth_model(synth.velocity(w), w["spacing"], 100.0)
    want = _oracle_run(w, v0)
    _check(w, _gpu_forward(w, v0), want)
