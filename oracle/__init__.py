"""FP64 reference ("oracle") for the acoustic finite-difference stepper.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and it shares no code with the GPU library.

Plain and slow on purpose: every quantity is the closed-form definition
written out in float64, the time loop lives in ``fd_oracle.c`` (plain loops,
one pass per step, OpenMP over points only).

The thesis states the problem through Devito's objects (Section 2.1.1): a
``Grid`` with shape and extent, a ``TimeFunction`` with a time order and a
space order, a ``Function`` for the medium, ``SparseTimeFunction`` sources and
receivers, and an ``Operator`` applied for a number of steps with a time step.
The acoustic operator itself is the case left open in Section 6.2.1; the
thesis gives no formula for it, so the definitions below are readings, each
listed with its pin in the design notes:

  O1 grid        physical points N_a, spacing h_a, origin o_a; nbl damping
                 points on each face; padded index i_a in [0, N_a + 2 nbl);
                 coordinate x = o_a + (i_a - nbl) h_a.
  O2 medium      v on the padded grid, layer filled by edge replication.
  O3 weights     maximal-order central 2nd-derivative weights, r = so/2.
  O4 Laplacian   sum over axes, zero outside the padded grid.
  O5 damping     sigma = sigma_max sum_a (d_a / nbl)^2; the default
                 sigma_max is pinned by the measured round-trip reflection
                 of the layer.
  O6 update      centred leapfrog with centred damping.
  O7 time step   Courant number v_max dt / h.
  O8 sources     multilinear weights over the 2^d cell corners, / prod(h).
  O9 receivers   the same weights, sampling u^{n+1}.
  O11 adjoint    exact transpose of O6-O9.
  O12 gradient   d J / d m on the padded grid, J = 1/2 sum (rec - d_obs)^2.

Array layout: numpy arrays of shape (nz, ny, nx) in 3D or (nz, nx) in 2D
(axis 0 of the grid description, x, is the last numpy axis).  Coordinates are
given in the grid's axis order: (x, y, z) or (x, z).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction
from itertools import product

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile fd_oracle.c with gcc (FP64, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "fd_oracle.c")
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
            build(force=True)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.orc_laplacian.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P, P, P]
        lib.orc_laplacian.restype = None
        lib.orc_forward.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P, P, P,
                                    ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, P, P, P,
                                    ctypes.c_int, P, P, P, P, P, P]
        lib.orc_forward.restype = ctypes.c_int
        lib.orc_adjoint.argtypes = [ctypes.c_int, P, P, ctypes.c_int, P, P, P,
                                    ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, P, P, P,
                                    ctypes.c_int, P, P, P, P]
        lib.orc_adjoint.restype = ctypes.c_int
        lib.orc_imaging.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int,
                                    P, P, P]
        lib.orc_imaging.restype = None
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Run the oracle's loops on n threads from now on."""
    _load().orc_set_threads(int(n))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# O1: the grid
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Grid:
    """Physical shape (x, y, z) or (x, z), spacing and origin in metres,
    space order of the second derivative, nbl damping points per face."""
    shape: tuple
    spacing: tuple
    origin: tuple
    space_order: int
    nbl: int = 0

    @property
    def ndim(self) -> int:
        return len(self.shape)

    @property
    def radius(self) -> int:
        return self.space_order // 2

    @property
    def padded(self) -> tuple:
        """Padded points per axis, grid axis order (x first)."""
        return tuple(n + 2 * self.nbl for n in self.shape)

    @property
    def array_shape(self) -> tuple:
        """numpy shape of a padded field (slowest axis first)."""
        return tuple(reversed(self.padded))


def _check_grid(g: Grid) -> None:
    if g.ndim not in (2, 3):
        raise ValueError("ndim must be 2 or 3")
    if g.space_order % 2 or not 2 <= g.space_order <= 16:
        raise ValueError("space_order must be even, 2..16")


# --------------------------------------------------------------------------
# O3: second-derivative weights
# --------------------------------------------------------------------------
def fd_weights_exact(space_order: int) -> list:
    """Central second-derivative weights c_0..c_r (r = so/2) as Fractions:
    c_j = 2 (-1)^(j+1) (r!)^2 / (j^2 (r-j)! (r+j)!),  c_0 = -2 sum_j c_j.
    These are the unique weights of the symmetric (2r+1)-point stencil that
    is exact on polynomials of degree <= 2r+1 (the space order of Section
    5.1.2's u.dx2 and u.dy2; at so 2 they are the 1, -2, 1 of the printed
    diffusion kernel in Section 3.2.2)."""
    if space_order % 2 or space_order < 2:
        raise ValueError("space_order must be even and >= 2")
    r = space_order // 2
    c = [Fraction(0)] * (r + 1)
    for j in range(1, r + 1):
        c[j] = Fraction(2 * (-1) ** (j + 1) * math.factorial(r) ** 2,
                        j * j * math.factorial(r - j) * math.factorial(r + j))
    c[0] = -2 * sum(c[1:])
    return c


def fd_weights(space_order: int) -> np.ndarray:
    """fd_weights_exact rounded once to float64."""
    return np.array([float(x) for x in fd_weights_exact(space_order)], dtype=np.float64)


# --------------------------------------------------------------------------
# O2 / O5 / O7: medium, damping, time step
# --------------------------------------------------------------------------
def pad_velocity(g: Grid, v_phys) -> np.ndarray:
    """O2: widen to float64 and fill the damping layer by edge replication:
    a layer point takes the velocity of the nearest physical point (pinned by
    a brute-force nearest-point search)."""
    v = np.asarray(v_phys, dtype=np.float64)
    if v.shape != tuple(reversed(g.shape)):
        raise ValueError("velocity shape %s != %s" % (v.shape, tuple(reversed(g.shape))))
    if g.nbl == 0:
        return v.copy()
    return np.pad(v, g.nbl, mode="edge")


def sigma_max_default(g: Grid, vmax: float) -> float:
    """O5 default: 3 v_max ln(1000) / (2 nbl h), h the smallest spacing --
    the estimate that gives a perfectly matched layer of quadratic profile a
    round-trip reflection of 1e-3.  With the damping term m sigma u_t of this
    PDE, a wave of frequency w >> sigma decays as exp(-x sigma / (2 v)), half
    the PML rate, so the same sigma_max returns 1000^(-1/2) of a normally
    incident wave at v_max after a round trip through a thick layer (pinned
    by a measured reflection; the thesis describes no absorbing layer)."""
    if g.nbl == 0:
        return 0.0
    return 3.0 * vmax * math.log(1000.0) / (2.0 * g.nbl * min(g.spacing))


def damping(g: Grid, sigma_max: float) -> np.ndarray:
    """O5: sigma_i = sigma_max sum_a (d_a / nbl)^2 with
    d_a = max(0, nbl - i_a, i_a - (nbl + N_a - 1)); zero when nbl == 0.
    No passage of the thesis fixes the profile.  Pinned by hand values, and
    through the measured round-trip reflection, which depends on the sum of
    sigma over the layer (a linear or cubic profile fails it)."""
    sig = np.zeros(g.array_shape, dtype=np.float64)
    if g.nbl == 0:
        return sig
    for a in range(g.ndim):
        n_pad = g.padded[a]
        i = np.arange(n_pad)
        d = np.maximum(0, np.maximum(g.nbl - i, i - (g.nbl + g.shape[a] - 1)))
        prof = sigma_max * (d / g.nbl) ** 2
        # numpy axis of grid axis a is ndim-1-a
        shp = [1] * g.ndim
        shp[g.ndim - 1 - a] = n_pad
        sig = sig + prof.reshape(shp)
    return sig


def critical_dt(g: Grid, vmax: float) -> float:
    """Von Neumann limit of O6 without damping:
    dt_crit = 1 / (v_max sqrt(sum_{j odd} c_j * sum_a h_a^-2))."""
    c = fd_weights_exact(g.space_order)
    s_odd = float(sum(c[j] for j in range(1, len(c)) if j % 2 == 1))
    return 1.0 / (vmax * math.sqrt(s_odd * sum(1.0 / h ** 2 for h in g.spacing)))


def courant_dt(g: Grid, vmax: float, courant: float = 0.4) -> float:
    """O7 reading (i): dt = courant * h_min / v_max."""
    return courant * min(g.spacing) / vmax


# --------------------------------------------------------------------------
# O8 / O9: multilinear weights of off-grid points
# --------------------------------------------------------------------------
def kaiser_beta_default(r: int) -> float:
    """Kaiser shape used when none is given: b = pi r / 2 (a reading; Hicks
    2002 tunes b per half-width for a chosen passband, the thesis does not
    treat off-grid points at all)."""
    return math.pi * r / 2.0


def kaiser_sinc_1d(t: float, r: int, b: float = 0.0) -> tuple:
    """Kaiser-windowed sinc weights of a point at fractional grid position t
    along one axis (Hicks 2002): the 2r nodes k = floor(t) - r + 1 ..
    floor(t) + r, weight sinc(k - t) W(k - t) with the Kaiser window
    W(x) = I0(b sqrt(1 - (x/r)^2)) / I0(b) for |x| <= r, else 0.
    Returns (first node, list of the 2r weights)."""
    b = b if b > 0.0 else kaiser_beta_default(r)
    k0 = int(math.floor(t)) - r + 1
    w = []
    for i in range(2 * r):
        x = (k0 + i) - t
        if x == round(x):            # sinc is exactly 1 at 0 and 0 at the other integers
            sinc = 1.0 if x == 0.0 else 0.0
        else:
            sinc = math.sin(math.pi * x) / (math.pi * x)
        q = 1.0 - (x / r) ** 2
        win = float(np.i0(b * math.sqrt(q))) / float(np.i0(b)) if q >= 0.0 else 0.0
        w.append(sinc * win)
    return k0, w


def sparse_weights(g: Grid, coords, sinc_radius: int = 0, sinc_beta: float = 0.0) -> tuple:
    """Flat padded indices and weights of the grid points a sparse point
    touches.  sinc_radius 0 (O8): multilinear over the 2^d corners of the
    cell that contains the point: per axis t = (x - o)/h, cell k = floor(t)
    (k = N-2 when the point sits on the last grid line), p = t - k, corner
    weight the product over axes of (1 - p) or p.  sinc_radius r >= 1: the
    tensor product over axes of kaiser_sinc_1d(t, r, sinc_beta), (2r)^d
    nodes; a node outside the padded grid keeps index 0 and weight 0 (the
    field is zero there, so dropping it is the exact restriction).  Raises
    ValueError for points outside the physical extent."""
    if sinc_radius:
        return _sinc_weights(g, coords, sinc_radius, sinc_beta)
    xyz = np.asarray(coords, dtype=np.float64).reshape(-1, g.ndim)
    npts = xyz.shape[0]
    nc = 1 << g.ndim
    idx = np.zeros((npts, nc), dtype=np.int64)
    w = np.zeros((npts, nc), dtype=np.float64)
    strides = []
    s = 1
    for a in range(g.ndim):
        strides.append(s)
        s *= g.padded[a]
    for p_i in range(npts):
        ks, fr = [], []
        for a in range(g.ndim):
            t = (xyz[p_i, a] - g.origin[a]) / g.spacing[a]
            if not (0.0 <= t <= g.shape[a] - 1):
                raise ValueError("point %d outside the grid along axis %d" % (p_i, a))
            k = int(math.floor(t))
            if k >= g.shape[a] - 1:
                k = g.shape[a] - 2
            ks.append(k)
            fr.append(t - k)
        for ci, bits in enumerate(product((0, 1), repeat=g.ndim)):
            # bits[a] for axis a; corner order: last axis varies fastest
            flat = 0
            wt = 1.0
            for a in range(g.ndim):
                b = bits[a]
                flat += (ks[a] + b + g.nbl) * strides[a]
                wt *= fr[a] if b else (1.0 - fr[a])
            idx[p_i, ci] = flat
            w[p_i, ci] = wt
    return idx, w


def _sinc_weights(g: Grid, coords, r: int, b: float) -> tuple:
    xyz = np.asarray(coords, dtype=np.float64).reshape(-1, g.ndim)
    npts = xyz.shape[0]
    nc = (2 * r) ** g.ndim
    idx = np.zeros((npts, nc), dtype=np.int64)
    w = np.zeros((npts, nc), dtype=np.float64)
    strides = []
    s = 1
    for a in range(g.ndim):
        strides.append(s)
        s *= g.padded[a]
    for p_i in range(npts):
        axes = []
        for a in range(g.ndim):
            t = (xyz[p_i, a] - g.origin[a]) / g.spacing[a]
            if not (0.0 <= t <= g.shape[a] - 1):
                raise ValueError("point %d outside the grid along axis %d" % (p_i, a))
            axes.append(kaiser_sinc_1d(t, r, b))
        for ci, offs in enumerate(product(range(2 * r), repeat=g.ndim)):
            flat, wt, inside = 0, 1.0, True
            for a in range(g.ndim):
                k0, wa = axes[a]
                ip = k0 + offs[a] + g.nbl
                if not 0 <= ip < g.padded[a]:
                    inside = False
                flat += ip * strides[a]
                wt *= wa[offs[a]]
            if inside:
                idx[p_i, ci] = flat
                w[p_i, ci] = wt
    return idx, w


# --------------------------------------------------------------------------
# O4 / O6 / O9 / O11 / O12: the steppers
# --------------------------------------------------------------------------
def _dims(g: Grid):
    n = np.array(g.padded, dtype=np.int64)
    h = np.array(g.spacing, dtype=np.float64)
    return n, h


def laplacian(g: Grid, u) -> np.ndarray:
    """O4 applied to a padded field."""
    _check_grid(g)
    u = np.ascontiguousarray(u, dtype=np.float64)
    if u.shape != g.array_shape:
        raise ValueError("field shape")
    out = np.empty_like(u)
    n, h = _dims(g)
    c = fd_weights(g.space_order)
    _load().orc_laplacian(g.ndim, _ptr(n), _ptr(h), g.radius, _ptr(c), _ptr(u), _ptr(out))
    return out


def _field(g, a, name):
    if a is None:
        return np.zeros(g.array_shape, dtype=np.float64)
    a = np.array(a, dtype=np.float64, copy=True, order="C")
    if a.shape != g.array_shape:
        raise ValueError("%s shape %s != %s" % (name, a.shape, g.array_shape))
    return a


def forward(g: Grid, v_pad, sigma, dt: float, nt: int, src_coords, wavelet,
            rec_coords, u0=None, u_prev=None, keep_history: bool = False, sinc_radius: int = 0, sinc_beta: float = 0.0):
    """O6 + O8 + O9.  Returns (rec [nt, nrec], u^nt, u^{nt-1}, history or None).
    wavelet is [nt, nsrc]; history holds u^{-1}..u^{nt} when requested."""
    _check_grid(g)
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    if v_pad.shape != g.array_shape or sigma.shape != g.array_shape:
        raise ValueError("medium shape")
    sidx, sw = sparse_weights(g, src_coords, sinc_radius, sinc_beta)
    ridx, rw = sparse_weights(g, rec_coords, sinc_radius, sinc_beta)
    nsrc, nrec = sidx.shape[0], ridx.shape[0]
    nc = sidx.shape[1]
    wav = np.ascontiguousarray(wavelet, dtype=np.float64).reshape(nt, nsrc)
    rec = np.zeros((nt, nrec), dtype=np.float64)
    a = _field(g, u0, "u0")
    b = _field(g, u_prev, "u_prev")
    hist = None
    if keep_history:
        hist = np.zeros((nt + 2,) + g.array_shape, dtype=np.float64)
    n, h = _dims(g)
    c = fd_weights(g.space_order)
    rc = _load().orc_forward(g.ndim, _ptr(n), _ptr(h), g.radius, _ptr(c),
                             _ptr(v_pad), _ptr(sigma), float(dt), int(nt),
                             nc, nsrc, _ptr(sidx), _ptr(sw), _ptr(wav),
                             nrec, _ptr(ridx), _ptr(rw), _ptr(rec),
                             _ptr(a), _ptr(b),
                             _ptr(hist) if hist is not None else None)
    if rc != 0:
        raise MemoryError("oracle forward: allocation failed")
    return rec, a, b, hist


def adjoint(g: Grid, v_pad, sigma, dt: float, nt: int, src_coords, rec_coords,
            residual, keep_history: bool = False, sinc_radius: int = 0, sinc_beta: float = 0.0):
    """O11.  residual is [nt, nrec]; returns (F^T r [nt, nsrc], lam history or None)."""
    _check_grid(g)
    v_pad = np.ascontiguousarray(v_pad, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    sidx, sw = sparse_weights(g, src_coords, sinc_radius, sinc_beta)
    ridx, rw = sparse_weights(g, rec_coords, sinc_radius, sinc_beta)
    nsrc, nrec = sidx.shape[0], ridx.shape[0]
    nc = sidx.shape[1]
    res = np.ascontiguousarray(residual, dtype=np.float64).reshape(nt, nrec)
    out = np.zeros((nt, nsrc), dtype=np.float64)
    hist = np.zeros((nt,) + g.array_shape, dtype=np.float64) if keep_history else None
    n, h = _dims(g)
    c = fd_weights(g.space_order)
    rc = _load().orc_adjoint(g.ndim, _ptr(n), _ptr(h), g.radius, _ptr(c),
                             _ptr(v_pad), _ptr(sigma), float(dt), int(nt),
                             nc, nsrc, _ptr(sidx), _ptr(sw), _ptr(out),
                             nrec, _ptr(ridx), _ptr(rw), _ptr(res),
                             _ptr(hist) if hist is not None else None)
    if rc != 0:
        raise MemoryError("oracle adjoint: allocation failed")
    return out, hist


def misfit(rec, d_obs) -> tuple:
    """O12: residual r = rec - d_obs and J = 1/2 sum r^2."""
    r = np.asarray(rec, dtype=np.float64) - np.asarray(d_obs, dtype=np.float64)
    return 0.5 * float(np.sum(r * r)), r


def gradient(g: Grid, v_pad, sigma, dt: float, nt: int, src_coords, wavelet,
             rec_coords, d_obs, sinc_radius: int = 0, sinc_beta: float = 0.0):
    """O12: returns (J, g_m on the padded grid, rec).  Keeps the whole forward
    and adjoint history in memory: small problems only."""
    rec, _, _, hist = forward(g, v_pad, sigma, dt, nt, src_coords, wavelet,
                              rec_coords, keep_history=True, sinc_radius=sinc_radius, sinc_beta=sinc_beta)
    J, r = misfit(rec, d_obs)
    _, lam = adjoint(g, v_pad, sigma, dt, nt, src_coords, rec_coords, r, keep_history=True,
                     sinc_radius=sinc_radius, sinc_beta=sinc_beta)
    grad = np.zeros(g.array_shape, dtype=np.float64)
    n, _ = _dims(g)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    _load().orc_imaging(g.ndim, _ptr(n), _ptr(sigma), float(dt), int(nt),
                        _ptr(hist), _ptr(lam), _ptr(grad))
    return J, grad, rec


def energy(g: Grid, v_pad, dt: float, u_next, u_cur) -> float:
    """Discrete energy of O6 without damping or source:
    E^{n+1/2} = sum m (u^{n+1}-u^n)^2 / dt^2 + sum u^{n+1} (-Lap_h u^n)."""
    m = 1.0 / np.asarray(v_pad, dtype=np.float64) ** 2
    du = (np.asarray(u_next) - np.asarray(u_cur)) / dt
    return float(np.sum(m * du * du) - np.sum(np.asarray(u_next) * laplacian(g, u_cur)))


# --------------------------------------------------------------------------
# The thesis's benchmark problem: 2D diffusion (Section 5.1.2)
# --------------------------------------------------------------------------
def diffusion(g: Grid, u0, nu: float, dt: float, nt: int) -> np.ndarray:
    """Explicit diffusion u_t = nu (u_xx + u_yy), first order in time: the
    operator the benchmarks of Section 5.1.2 time, advanced by forward Euler,
    u^{n+1} = u^n + nu dt Lap_h u^n, with the O3 weights and the field zero
    outside the grid.  Returns u^{nt}."""
    if g.ndim != 2 or g.nbl != 0:
        raise ValueError("diffusion is defined on a 2D grid without damping layer")
    u = np.array(u0, dtype=np.float64, copy=True)
    if u.shape != g.array_shape:
        raise ValueError("field shape")
    for _ in range(int(nt)):
        u = u + nu * dt * laplacian(g, u)
    return u


def diffusion_critical_dt(g: Grid, nu: float) -> float:
    """Stability limit of the explicit diffusion step: the largest
    eigenvalue of -Lap_h is 4 sum_{j odd} c_j sum_a h_a^-2, and the forward
    Euler factor 1 - nu dt lambda must stay >= -1."""
    c = fd_weights_exact(g.space_order)
    s_odd = float(sum(c[j] for j in range(1, len(c)) if j % 2 == 1))
    return 2.0 / (nu * 4.0 * s_odd * sum(1.0 / h ** 2 for h in g.spacing))
