"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no stepping arithmetic: it only draws velocity models,
source wavelets and acquisition geometry, in float64, and casts them to the
float32 the GPU library takes.  Every generator uses
``numpy.random.default_rng(seed)``.

Workloads (sizes in physical points per axis, axis order x, y, z):

  acoustic2d_101     2D 101 x 101, h 10 m, v 1500 m/s, so 4, no damping,
                     200 steps, 10 Hz Ricker at (500, 500) m, 101 receivers at
                     z = 20 m, x = 0..1000 m.
  layered3d_256      3D 256^3 + 40 damping points per face, h 10 m, 10
                     seeded layers 1.5-4.5 km/s, so 8, 1000 steps, 15 Hz
                     Ricker at (1275, 1275, 20) m (half a cell off-grid in x
                     and y), 256 receivers along x at y = 1275 m, z = 20 m.
  grf3d_512          3D 512^3 + 40 damping, seeded Gaussian random field
                     (Gaussian filter sigma 100 m of white noise, min-max
                     mapped to 1.5-4.5 km/s), so 8, 1500 steps, 512 receivers.
  serving            64 requests: grids from {128^3, 192^3, 256^3,
                     160x320x320} + 40 damping, so in {4, 8, 12}, 500-1000
                     steps, layered media, Poisson arrivals.
  gradient3d_200     3D 200^3 + 40 damping, so 8, 800 steps, true layered
                     model vs Gaussian-smoothed start, checkpoints every 50.
"""
from __future__ import annotations

import math

import numpy as np

VMIN = 1500.0
VMAX = 4500.0


def ricker(nt: int, dt: float, f0: float, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet w(t) = (1 - 2 pi^2 f^2 (t-t0)^2) exp(-pi^2 f^2 (t-t0)^2)
    sampled at t_n = n dt, unit peak at t0 = 1/f (float64)."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (math.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def layered_model(shape, spacing, nlayers: int = 10, vmin: float = VMIN,
                  vmax: float = VMAX, seed: int = 0) -> np.ndarray:
    """Horizontally layered velocity (float32, numpy shape reversed(shape)).
    nlayers-1 interface depths drawn U(0, depth extent) and sorted; layer k
    (top to bottom) has v = vmin + (vmax - vmin) k / (nlayers - 1)."""
    rng = np.random.default_rng(seed)
    nz = shape[-1]
    hz = spacing[-1]
    depth_extent = (nz - 1) * hz
    interfaces = np.sort(rng.uniform(0.0, depth_extent, size=nlayers - 1))
    z = np.arange(nz, dtype=np.float64) * hz
    layer = np.searchsorted(interfaces, z, side="right")
    vz = vmin + (vmax - vmin) * layer / (nlayers - 1)
    arr_shape = tuple(reversed(tuple(shape)))
    v = np.broadcast_to(vz.reshape((nz,) + (1,) * (len(shape) - 1)), arr_shape)
    return np.ascontiguousarray(v, dtype=np.float32)


def grf_model(shape, spacing, corr_sigma_m: float = 100.0, vmin: float = VMIN,
              vmax: float = VMAX, seed: int = 1) -> np.ndarray:
    """Smooth Gaussian random field: white N(0,1) noise, Gaussian filter of
    standard deviation corr_sigma_m metres (covariance exp(-r^2/l^2) with
    l = 2 sigma = 200 m), min-max mapped to [vmin, vmax]; float32."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    arr_shape = tuple(reversed(tuple(shape)))
    white = rng.standard_normal(arr_shape, dtype=np.float32)
    sig = [corr_sigma_m / h for h in reversed(tuple(spacing))]
    f = gaussian_filter(white, sigma=sig, mode="reflect").astype(np.float64)
    lo, hi = float(f.min()), float(f.max())
    v = vmin + (vmax - vmin) * (f - lo) / (hi - lo)
    return v.astype(np.float32)


def smooth_model(v, spacing, sigma_m: float = 100.0) -> np.ndarray:
    """Gaussian-smoothed copy of a model (starting model for inversion)."""
    from scipy.ndimage import gaussian_filter
    sig = [sigma_m / h for h in reversed(tuple(spacing))]
    return gaussian_filter(np.asarray(v, dtype=np.float64), sigma=sig,
                           mode="nearest").astype(np.float32)


def line_receivers(n: int, x0: float, x1: float, fixed: tuple, ndim: int) -> np.ndarray:
    """n receivers evenly spaced in x on [x0, x1]; remaining coordinates fixed
    ((y, z) in 3D or (z,) in 2D).  Returns float64 [n, ndim]."""
    xs = np.linspace(x0, x1, n) if n > 1 else np.array([x0])
    out = np.zeros((n, ndim), dtype=np.float64)
    out[:, 0] = xs
    for a, val in enumerate(fixed, start=1):
        out[:, a] = val
    return out


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded N(0, scale^2) float64 field of numpy shape ``shape``."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(shape)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------
def workload(name: str, **over) -> dict:
    """Parameters of a named workload.  Keys: ndim, shape, spacing, origin,
    space_order, nbl, nt, dt (Courant 0.4 at v_max), f0, src (list of
    coordinates), rec (array), model ('const', 'layered', 'grf'), seed."""
    if name == "acoustic2d_101":
        w = dict(ndim=2, shape=(101, 101), spacing=(10.0, 10.0), origin=(0.0, 0.0),
                 space_order=4, nbl=0, nt=200, f0=10.0, model="const", vconst=1500.0,
                 seed=0, src=[(500.0, 500.0)],
                 rec=line_receivers(101, 0.0, 1000.0, (20.0,), 2))
        w["dt"] = 0.4 * 10.0 / 1500.0
    elif name == "layered3d_256":
        w = dict(ndim=3, shape=(256, 256, 256), spacing=(10.0, 10.0, 10.0),
                 origin=(0.0, 0.0, 0.0), space_order=8, nbl=40, nt=1000, f0=15.0,
                 model="layered", seed=0, src=[(1275.0, 1275.0, 20.0)],
                 rec=line_receivers(256, 0.0, 2550.0, (1275.0, 20.0), 3))
        w["dt"] = 0.4 * 10.0 / VMAX
    elif name == "grf3d_512":
        w = dict(ndim=3, shape=(512, 512, 512), spacing=(10.0, 10.0, 10.0),
                 origin=(0.0, 0.0, 0.0), space_order=8, nbl=40, nt=1500, f0=15.0,
                 model="grf", seed=1, src=[(2555.0, 2555.0, 20.0)],
                 rec=line_receivers(512, 0.0, 5110.0, (2555.0, 20.0), 3))
        w["dt"] = 0.4 * 10.0 / VMAX
    elif name == "gradient3d_200":
        w = dict(ndim=3, shape=(200, 200, 200), spacing=(10.0, 10.0, 10.0),
                 origin=(0.0, 0.0, 0.0), space_order=8, nbl=40, nt=800, f0=15.0,
                 model="layered", seed=3, src=[(995.0, 995.0, 20.0)],
                 rec=line_receivers(200, 0.0, 1990.0, (995.0, 20.0), 3),
                 checkpoint_every=50)
        w["dt"] = 0.4 * 10.0 / VMAX
    else:
        raise KeyError(name)
    w.update(over)
    return w


def velocity(w: dict) -> np.ndarray:
    """Physical-shape float32 velocity for a workload dict."""
    if w["model"] == "const":
        return np.full(tuple(reversed(w["shape"])), w.get("vconst", VMIN), dtype=np.float32)
    if w["model"] == "layered":
        return layered_model(w["shape"], w["spacing"], seed=w["seed"])
    if w["model"] == "grf":
        return grf_model(w["shape"], w["spacing"], seed=w["seed"])
    raise KeyError(w["model"])


def wavelets(w: dict) -> np.ndarray:
    """[nt, nsrc] float32 Ricker wavelets for a workload."""
    nsrc = len(w["src"])
    r = ricker(w["nt"], w["dt"], w["f0"]).astype(np.float32)
    return np.ascontiguousarray(np.repeat(r[:, None], nsrc, axis=1))


def serving_requests(n: int = 64, seed: int = 2, rate_hz: float = 1.0):
    """The serving workload: n requests with Poisson arrival times (rate_hz),
    grids from {128^3, 192^3, 256^3, 160x320x320} (+40 damping), space order
    from {4, 8, 12}, nt from U{500..1000}, layered media with per-request
    seeds, a 15 Hz Ricker at the top centre and 128 receivers along x."""
    rng = np.random.default_rng(seed)
    shapes = [(128, 128, 128), (192, 192, 192), (256, 256, 256), (320, 320, 160)]
    reqs = []
    t = 0.0
    for i in range(n):
        t += rng.exponential(1.0 / rate_hz)
        shp = shapes[int(rng.integers(len(shapes)))]
        so = int(rng.choice([4, 8, 12]))
        nt = int(rng.integers(500, 1001))
        h = 10.0
        xc = (shp[0] - 1) * h / 2.0
        yc = (shp[1] - 1) * h / 2.0
        reqs.append(dict(ndim=3, shape=shp, spacing=(h, h, h), origin=(0.0, 0.0, 0.0),
                         space_order=so, nbl=40, nt=nt, f0=15.0, model="layered",
                         seed=1000 + i, src=[(xc, yc, 20.0)],
                         rec=line_receivers(128, 0.0, (shp[0] - 1) * h, (yc, 20.0), 3),
                         dt=0.4 * h / VMAX, arrival=t))
    return reqs
