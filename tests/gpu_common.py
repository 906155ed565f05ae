"""Helpers shared by the GPU tests: run the HIP path and the FP64 oracle on
the same seeded inputs."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def rel_l2(got, want) -> float:
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


# Element-wise bars beside the global relative L2 gate.  Per receiver the
# error is taken relative to that receiver's own norm, or to a tenth of the
# strongest receiver's norm when it is weaker (float32 rounding travels with
# the wavefield, so a receiver the wave barely reaches carries errors of the
# field's scale, not its own); K_REC times the gate.  Per field the largest
# pointwise error is taken relative to the field's largest magnitude, K_ABS
# times the gate.
K_REC = 3.0
K_ABS = 3.0


def trace_errors(got, want):
    """(global relative L2, worst per-receiver relative L2 as defined above)
    of traces [nt, nrec]."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    norms = np.linalg.norm(want, axis=0)
    per = np.linalg.norm(got - want, axis=0) / np.maximum(norms, 0.1 * norms.max())
    return rel_l2(got, want), float(per.max())


def field_errors(got, want):
    """(global relative L2, max |got - want| / max |want|) of a field."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return rel_l2(got, want), float(np.max(np.abs(got - want)) / np.max(np.abs(want)))


def assert_traces(got, want, tol=1e-5, label=""):
    e, per = trace_errors(got, want)
    print("%s traces: rel_l2 %.3e, worst receiver %.3e" % (label, e, per), flush=True)
    assert e <= tol, (label, e)
    assert per <= K_REC * tol, (label, per)
    return e, per


def assert_field(got, want, tol=1e-5, label=""):
    e, m = field_errors(got, want)
    print("%s field: rel_l2 %.3e, max-abs %.3e" % (label, e, m), flush=True)
    assert e <= tol, (label, e)
    assert m <= K_ABS * tol, (label, m)
    return e, m


def case(shape, so, nbl, nt, seed=0, nsrc=1, nrec=7, h=(10.0, 12.0, 9.0), f0=None, model="random"):
    """A heterogeneous, damped case with off-grid sources and receivers."""
    ndim = len(shape)
    spacing = tuple(h[:ndim])
    origin = tuple([3.0, -5.0, 1.0][:ndim])
    rng = np.random.default_rng(seed)
    arr_shape = tuple(reversed(shape))
    if model == "random":
        v = (1500.0 + 3000.0 * rng.uniform(size=arr_shape)).astype(np.float32)
    else:
        v = np.full(arr_shape, 2000.0, dtype=np.float32)
    ext = [(n - 1) * hh for n, hh in zip(shape, spacing)]
    src = [tuple(o + rng.uniform(0.2, 0.8) * e for o, e in zip(origin, ext)) for _ in range(nsrc)]
    rec = np.array([[o + rng.uniform(0.0, 1.0) * e for o, e in zip(origin, ext)] for _ in range(nrec)])
    vmax = float(v.max())
    g = oracle.Grid(tuple(shape), spacing, origin, so, nbl)
    dt = 0.8 * oracle.critical_dt(g, vmax)
    if f0 is None:
        f0 = 0.12 / dt / 4
    wav = np.stack([synth.ricker(nt, dt, f0, t0=1.2 / f0) * (1.0 + 0.3 * k) for k in range(nsrc)], axis=1)
    return dict(shape=tuple(shape), spacing=spacing, origin=origin, so=so, nbl=nbl, nt=nt, v=v,
                src=src, rec=rec, dt=dt, wav=wav.astype(np.float32), og=g)


def oracle_forward(c, keep_history=False, u0=None, u_prev=None):
    g = c["og"]
    vp = oracle.pad_velocity(g, c["v"])
    sig = oracle.damping(g, oracle.sigma_max_default(g, float(vp.max())))
    return oracle.forward(g, vp, sig, c["dt"], c["nt"], c["src"], c["wav"].astype(np.float64), c["rec"],
                          u0=u0, u_prev=u_prev, keep_history=keep_history, sinc_radius=c.get("sinc", 0))


def gpu_grid(c, **kw):
    from paper_1906_10811_amd import Grid
    dev = torch.device("cuda:0")
    kw.setdefault("sinc_radius", c.get("sinc", 0))
    return Grid(c["shape"], c["spacing"], torch.from_numpy(c["v"]).to(dev), space_order=c["so"],
                nbl=c["nbl"], origin=c["origin"], **kw)


def gpu_forward(c, grid=None, **kw):
    g = grid or gpu_grid(c)
    dev = torch.device("cuda:0")
    out = g.forward(c["src"], torch.from_numpy(c["wav"]).to(dev), c["rec"], c["dt"], **kw)
    torch.cuda.synchronize()
    return g, out
