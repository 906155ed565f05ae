"""MI355X acoustic finite-difference stepper: Python binding of libfd.

Argument marshalling only: every step of the stepper runs in the HIP kernels
of ``libfd.so`` (see ``include/fd.h``).  PyTorch provides device memory and
streams; the library borrows them.  If the library is not built, every entry
point raises -- there is no CPU fallback.

    g = Grid(shape=(256, 256, 256), spacing=(10., 10., 10.), space_order=8,
             nbl=40, vp=vp_cuda)
    rec = g.forward(src_xyz, wavelet_cuda, rec_xyz, dt)
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import FDError  # noqa: F401

__all__ = ["Grid", "Server", "FDError", "modeling", "diffusion", "diffusion_dt_limit", "build"]

_STORAGE = {"f32": _lib.FD_STORE_F32, "f16": _lib.FD_STORE_F16, "bf16": _lib.FD_STORE_BF16,
            "f16_diff": _lib.FD_STORE_F16_DIFF, "bf16_diff": _lib.FD_STORE_BF16_DIFF}
_PARAM = {"f32": _lib.FD_PARAM_F32, "q16": _lib.FD_PARAM_Q16}


def build() -> str:
    """Compile libfd.so in-tree for gfx950."""
    from .build import build as _b
    return _b()


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _coords(xyz, ndim: int) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, ndim))
    return a


def _dev_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % name)
    return t.detach().to(torch.float32).contiguous()


class Grid:
    """A grid with its medium, owning a torch-allocated device workspace
    that libfd borrows (fd_grid_create / fd_grid_destroy).

    storage: "f32", "f16", "bf16" (two 16-bit time levels), or, in 3D,
    "f16_diff" / "bf16_diff" (the level and its difference from the
    previous one, both 16-bit).

    param: "f32" (p = dt^2 v^2 in float32) or, in 3D, "q16" (16-bit codes
    on a uniform scale from dt^2 v_min^2 to dt^2 v_max^2; forward and
    adjoint only)."""

    def __init__(self, shape, spacing, vp: torch.Tensor, space_order: int = 8, nbl: int = 0,
                 origin=None, damp_max: float = 0.0, storage: str = "f32", amp_scale: float = 0.0,
                 vp_padded: bool = False, max_src: int = 0, max_rec: int = 0, zchunk: int = 0,
                 sinc_radius: int = 0, sinc_beta: float = 0.0, tile_x: int = 0, time_block: int = 0,
                 param: str = "f32", stream=None):
        lib = _lib.load()
        ndim = len(shape)
        self.ndim = ndim
        d = _lib.GridDesc()
        d.ndim = ndim
        for a in range(ndim):
            d.shape[a] = int(shape[a])
            d.spacing[a] = float(spacing[a])
            d.origin[a] = float(origin[a]) if origin is not None else 0.0
        d.space_order = int(space_order)
        d.nbl = int(nbl)
        d.damp_max = float(damp_max)
        d.storage = _STORAGE[storage]
        d.amp_scale = float(amp_scale)
        d.vp_padded = 1 if vp_padded else 0
        d.max_src = int(max_src)
        d.max_rec = int(max_rec)
        d.zchunk = int(zchunk)
        d.sinc_radius = int(sinc_radius)
        d.sinc_beta = float(sinc_beta)
        d.tile_x = int(tile_x)
        d.time_block = int(time_block)
        d.param_storage = _PARAM[param]
        self.desc = d
        nbytes = ctypes.c_size_t()
        _lib.check(lib.fd_grid_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)))
        self.vp = _dev_f32(vp, "vp")
        self.device = self.vp.device
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(lib.fd_grid_create(ctypes.byref(d), ctypes.c_void_p(aligned), nbytes.value,
                                          ctypes.c_void_p(self.vp.data_ptr()), _stream_ptr(stream),
                                          ctypes.byref(h)))
        self._h = h
        info = _lib.GridInfo()
        _lib.check(lib.fd_grid_get_info(h, ctypes.byref(info)))
        self.padded = tuple(info.padded[a] for a in range(ndim))
        self.padded_points = int(info.padded_points)
        self.vmax = info.vmax
        self.critical_dt = info.critical_dt
        self.damp_max = info.damp_max
        self.field_bytes = int(info.field_bytes)
        self.tile = (int(info.tile[0]), int(info.tile[1]))
        self.tile_strip = int(info.tile_strip)
        self.zchunk = int(info.zchunk)
        self.time_block = int(info.time_block)

    def param_scale(self):
        """(p0, dp) of the 16-bit p codes for the latest dt, (0, 0) before
        the first step or with float32 p."""
        info = _lib.GridInfo()
        _lib.check(_lib.load().fd_grid_get_info(self._h, ctypes.byref(info)))
        return info.param_base, info.param_step

    @property
    def array_shape(self):
        """torch shape of a dense padded field (slowest axis first)."""
        return tuple(reversed(self.padded))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fd_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _shot(self, src_xyz, wavelet, rec_xyz):
        src = _coords(src_xyz, self.ndim)
        rec = _coords(rec_xyz, self.ndim)
        sh = _lib.Shot()
        sh.nsrc = src.shape[0]
        sh.src_xyz = src.ctypes.data
        sh.src_wavelet = wavelet.data_ptr() if wavelet is not None else None
        sh.nrec = rec.shape[0]
        sh.rec_xyz = rec.ctypes.data
        return sh, (src, rec)

    def forward(self, src_xyz, wavelet: torch.Tensor, rec_xyz, dt: float, nt: int | None = None,
                u0: torch.Tensor | None = None, u_prev: torch.Tensor | None = None,
                save_state: bool = False, out: torch.Tensor | None = None, stream=None):
        """fd_forward.  wavelet: CUDA float32 [nt, nsrc].  Returns traces
        [nt, nrec] (and (u^nt, u^{nt-1}) dense padded when save_state)."""
        lib = _lib.load()
        wav = _dev_f32(wavelet, "wavelet")
        if wav.dim() == 1:
            wav = wav[:, None].contiguous()
        nt = wav.shape[0] if nt is None else int(nt)
        sh, keep = self._shot(src_xyz, wav, rec_xyz)
        if wav.shape[1] != sh.nsrc or wav.shape[0] < nt:
            raise ValueError("wavelet must be [nt, nsrc]")
        rec = out if out is not None else torch.empty((nt, sh.nrec), dtype=torch.float32, device=self.device)
        opts = _lib.FwdOpts()
        keep2 = []
        if u0 is not None:
            t = _dev_f32(u0, "u0").reshape(self.array_shape)
            keep2.append(t)
            opts.u0 = t.data_ptr()
        if u_prev is not None:
            t = _dev_f32(u_prev, "u_prev").reshape(self.array_shape)
            keep2.append(t)
            opts.u_prev = t.data_ptr()
        state = None
        if save_state:
            state = (torch.empty(self.array_shape, dtype=torch.float32, device=self.device),
                     torch.empty(self.array_shape, dtype=torch.float32, device=self.device))
            opts.save_u = state[0].data_ptr()
            opts.save_u_prev = state[1].data_ptr()
        _lib.check(lib.fd_forward(self._h, ctypes.byref(sh), nt, float(dt), ctypes.c_void_p(rec.data_ptr()),
                                  ctypes.byref(opts), _stream_ptr(stream)))
        return (rec, state) if save_state else rec

    def adjoint(self, src_xyz, rec_xyz, residual: torch.Tensor, dt: float, stream=None):
        """fd_adjoint.  residual: CUDA float32 [nt, nrec]; returns F^T r [nt, nsrc]."""
        lib = _lib.load()
        res = _dev_f32(residual, "residual")
        nt = res.shape[0]
        sh, keep = self._shot(src_xyz, None, rec_xyz)
        if res.shape[1] != sh.nrec:
            raise ValueError("residual must be [nt, nrec]")
        out = torch.empty((nt, sh.nsrc), dtype=torch.float32, device=self.device)
        _lib.check(lib.fd_adjoint(self._h, ctypes.byref(sh), nt, float(dt), ctypes.c_void_p(res.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def gradient_workspace_bytes(self, nt: int, nrec: int, checkpoint_every: int = 50,
                                 binomial_slots: int | None = None) -> int:
        """fd_gradient_workspace_bytes for the schedule gradient() would use."""
        flags, K = 0, int(checkpoint_every)
        if binomial_slots is not None:
            flags, K = _lib.FD_GRAD_BINOMIAL, int(binomial_slots)
        n = ctypes.c_size_t()
        _lib.check(_lib.load().fd_gradient_workspace_bytes(self._h, int(nt), int(nrec), K, flags, ctypes.byref(n)))
        return n.value

    def gradient(self, src_xyz, wavelet: torch.Tensor, rec_xyz, d_obs: torch.Tensor, dt: float,
                 checkpoint_every: int = 50, residual_given: bool = False, want_src_adj: bool = False,
                 binomial_slots: int | None = None, wrt_velocity: bool = False, stream=None):
        """fd_gradient.  Returns (misfit [1] float64, g_m dense padded float64,
        traces [nt, nrec], F^T residual [nt, nsrc] or None).  binomial_slots
        not None selects the binomial checkpoint schedule with that many
        snapshot slots (0 allowed) instead of checkpoints every
        checkpoint_every steps.  wrt_velocity: the gradient with respect to
        the padded velocity instead of m (FD_GRAD_VELOCITY)."""
        lib = _lib.load()
        wav = _dev_f32(wavelet, "wavelet")
        if wav.dim() == 1:
            wav = wav[:, None].contiguous()
        obs = _dev_f32(d_obs, "d_obs")
        nt = obs.shape[0]
        sh, keep = self._shot(src_xyz, wav, rec_xyz)
        flags = _lib.FD_GRAD_RESIDUAL_GIVEN if residual_given else 0
        if wrt_velocity:
            flags |= _lib.FD_GRAD_VELOCITY
        K = int(checkpoint_every)
        if binomial_slots is not None:
            flags |= _lib.FD_GRAD_BINOMIAL
            K = int(binomial_slots)
        nbytes = ctypes.c_size_t()
        _lib.check(lib.fd_gradient_workspace_bytes(self._h, nt, sh.nrec, K, flags, ctypes.byref(nbytes)))
        # The workspace (up to the whole forward history) is allocated on the
        # stream the work runs on, so that torch's caching allocator hands the
        # same block to the next gradient on that stream instead of reserving
        # a second one (a block allocated on another stream is not reused).
        with torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext():
            ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        aligned = (ws.data_ptr() + 255) // 256 * 256
        misfit = torch.empty(1, dtype=torch.float64, device=self.device)
        grad = torch.empty(self.array_shape, dtype=torch.float64, device=self.device)
        rec = torch.empty((nt, sh.nrec), dtype=torch.float32, device=self.device)
        sadj = torch.empty((nt, sh.nsrc), dtype=torch.float32, device=self.device) if want_src_adj else None
        _lib.check(lib.fd_gradient(self._h, ctypes.byref(sh), nt, float(dt), ctypes.c_void_p(obs.data_ptr()),
                                   K, flags, ctypes.c_void_p(aligned), nbytes.value,
                                   ctypes.c_void_p(misfit.data_ptr()), ctypes.c_void_p(grad.data_ptr()),
                                   ctypes.c_void_p(rec.data_ptr()),
                                   ctypes.c_void_p(sadj.data_ptr()) if sadj is not None else None,
                                   _stream_ptr(stream)))
        # the workspace must outlive the enqueued work on this stream
        ws.record_stream(torch.cuda.current_stream() if stream is None else stream)
        return misfit, grad, rec, sadj


class _Modeling(torch.autograd.Function):
    """Traces as a differentiable function of the padded velocity and the
    source wavelets; the backward pass is fd_gradient driven by the incoming
    trace cotangent, which also applies the chain rule from m = 1/v^2 to v
    (FD_GRAD_VELOCITY).  The damping strength is a constant of the operator:
    the forward grid's sigma_max (given, or the library's default from that
    grid's v_max) is passed unchanged to the backward grid, so the gradient
    is the derivative of the forward map with sigma fixed."""

    @staticmethod
    def forward(ctx, vp_padded, wavelet, shape, spacing, space_order, nbl, src_xyz, rec_xyz, dt,
                checkpoint_every, sinc_radius, damp_max):
        g = Grid(shape, spacing, vp_padded, space_order=space_order, nbl=nbl, vp_padded=True,
                 sinc_radius=sinc_radius, damp_max=damp_max)
        rec = g.forward(src_xyz, wavelet, rec_xyz, dt)
        ctx.save_for_backward(vp_padded, wavelet)
        ctx.cfg = (shape, spacing, space_order, nbl, src_xyz, rec_xyz, dt, checkpoint_every, sinc_radius,
                   g.damp_max)
        g.close()
        return rec

    @staticmethod
    def backward(ctx, grad_rec):
        vp_padded, wavelet = ctx.saved_tensors
        shape, spacing, space_order, nbl, src_xyz, rec_xyz, dt, K, sinc_radius, damp_max = ctx.cfg
        g = Grid(shape, spacing, vp_padded, space_order=space_order, nbl=nbl, vp_padded=True,
                 sinc_radius=sinc_radius, damp_max=damp_max)
        _, g_v, _, g_w = g.gradient(src_xyz, wavelet, rec_xyz, grad_rec.contiguous(), dt,
                                    checkpoint_every=K, residual_given=True, want_src_adj=True,
                                    wrt_velocity=True)
        torch.cuda.current_stream().synchronize()
        g.close()
        return (g_v.to(vp_padded.dtype), g_w.to(wavelet.dtype).reshape(wavelet.shape),
                None, None, None, None, None, None, None, None, None, None)


def modeling(vp_padded: torch.Tensor, wavelet: torch.Tensor, shape, spacing, space_order: int,
             nbl: int, src_xyz, rec_xyz, dt: float, checkpoint_every: int = 50,
             sinc_radius: int = 0, damp_max: float = 0.0) -> torch.Tensor:
    """Differentiable forward modelling: traces [nt, nrec] from the velocity
    on the padded grid and the wavelets [nt, nsrc] (sparse points multilinear,
    or windowed sinc of the given half-width).  damp_max: sigma_max of the
    damping layer, 1/s; <= 0 takes the library's default from max(v) at the
    forward call.  Either way sigma is held fixed in the gradient."""
    return _Modeling.apply(vp_padded, wavelet, tuple(shape), tuple(spacing), space_order, nbl,
                           src_xyz, rec_xyz, dt, checkpoint_every, int(sinc_radius), float(damp_max))


class Server:
    """Continuous-batching shot server (fd_server_create / fd_submit / fd_wait)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 8, steps_per_round: int = 0, device: int = 0,
                 policy: str = "share"):
        """policy: "share" (every resident request advances as its previous
        chunk completes), "shortest" (preemptive shortest remaining work
        first: the device holds at most two chunks, both for the request with
        the least remaining work) or "ratio" (the same, ordered by the
        response ratio (age + remaining time) / remaining time, so that a long
        request that has waited is no longer passed)."""
        lib = _lib.load()
        d = _lib.ServerDesc()
        d.device = int(device)
        d.hbm_budget_bytes = int(hbm_budget_bytes)
        d.max_slots = int(max_slots)
        d.steps_per_round = int(steps_per_round)
        d.policy = {"share": _lib.FD_SERVE_SHARE, "shortest": _lib.FD_SERVE_SHORTEST,
                    "ratio": _lib.FD_SERVE_RATIO}[policy]
        h = ctypes.c_void_p()
        _lib.check(lib.fd_server_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @staticmethod
    def _request(shape, spacing, space_order, nbl, vp, src_xyz, wavelet, rec_xyz, dt, storage="f32",
                 origin=None, amp_scale=0.0, sinc_radius=0, sinc_beta=0.0, time_block=0, param="f32"):
        ndim = len(shape)
        r = _lib.Request()
        g = r.grid
        g.ndim = ndim
        for a in range(ndim):
            g.shape[a] = int(shape[a])
            g.spacing[a] = float(spacing[a])
            g.origin[a] = float(origin[a]) if origin is not None else 0.0
        g.space_order = int(space_order)
        g.nbl = int(nbl)
        g.storage = _STORAGE[storage]
        g.amp_scale = float(amp_scale)
        g.sinc_radius = int(sinc_radius)
        g.sinc_beta = float(sinc_beta)
        g.time_block = int(time_block)
        g.param_storage = _PARAM[param]
        vp = np.ascontiguousarray(vp, dtype=np.float32)
        src = _coords(src_xyz, ndim)
        rec = _coords(rec_xyz, ndim)
        wav = np.ascontiguousarray(np.asarray(wavelet, dtype=np.float32).reshape(-1, src.shape[0]))
        nt = wav.shape[0]
        out = np.zeros((nt, rec.shape[0]), dtype=np.float32)
        r.vp_host = vp.ctypes.data
        r.nsrc = src.shape[0]
        r.src_xyz = src.ctypes.data
        r.wavelet_host = wav.ctypes.data
        r.nrec = rec.shape[0]
        r.rec_xyz = rec.ctypes.data
        r.nt = nt
        r.dt = float(dt)
        r.rec_out_host = out.ctypes.data
        return r, (vp, src, rec, wav, out)

    @staticmethod
    def request_bytes(**kw) -> int:
        r, _ = Server._request(**kw)
        n = ctypes.c_size_t()
        _lib.check(_lib.load().fd_request_bytes(ctypes.byref(r), ctypes.byref(n)))
        return n.value

    def submit(self, **kw) -> int:
        """Queue one shot; keyword arguments as _request.  Returns the ticket."""
        r, keep = self._request(**kw)
        t = ctypes.c_uint64()
        _lib.check(_lib.load().fd_submit(self._h, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        """Block until done; returns (traces [nt, nrec] numpy, result dict)."""
        res = _lib.Result()
        rc = _lib.load().fd_wait(self._h, ctypes.c_uint64(ticket), float(timeout), ctypes.byref(res))
        if rc == _lib.FD_ERR_TIMEOUT:
            raise TimeoutError("ticket %d" % ticket)
        keep = self._keep.pop(ticket, None)
        _lib.check(rc)
        return keep[4], {"status": res.status, "t_submit": res.t_submit, "t_start": res.t_start,
                         "t_done": res.t_done, "bytes": res.bytes_reserved}

    def stats(self):
        pb = ctypes.c_size_t()
        ps = ctypes.c_int()
        _lib.check(_lib.load().fd_server_stats(self._h, ctypes.byref(pb), ctypes.byref(ps)))
        return {"peak_bytes": pb.value, "peak_slots": ps.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def diffusion_dt_limit(shape, spacing, space_order: int, nu: float) -> float:
    """fd_diffusion_dt_limit: the largest stable dt of the explicit scheme on
    an [Ny, Nx] = reversed(shape) grid (host only)."""
    d = _lib.DiffusionDesc()
    d.shape[0], d.shape[1] = int(shape[0]), int(shape[1])
    d.spacing[0], d.spacing[1] = float(spacing[0]), float(spacing[1])
    d.space_order = int(space_order)
    d.nu = float(nu)
    out = ctypes.c_double()
    _lib.check(_lib.load().fd_diffusion_dt_limit(ctypes.byref(d), ctypes.byref(out)))
    return out.value


def diffusion(u0: torch.Tensor, spacing, space_order: int, nu: float, dt: float, nt: int,
              out: torch.Tensor | None = None, time_block: int = 0, stream=None) -> torch.Tensor:
    """fd_diffusion_run: nt explicit steps of u_t = nu (u_xx + u_yy) from the
    CUDA float32 field u0 [Ny, Nx]; returns u^nt (a new tensor unless `out`).
    time_block: steps per launch (0: automatic, 1: one per launch, k: at most k)."""
    lib = _lib.load()
    u = _dev_f32(u0, "u0")
    if u.dim() != 2:
        raise ValueError("u0 must be [Ny, Nx]")
    d = _lib.DiffusionDesc()
    d.shape[0], d.shape[1] = int(u.shape[1]), int(u.shape[0])
    d.spacing[0], d.spacing[1] = float(spacing[0]), float(spacing[1])
    d.space_order = int(space_order)
    d.nu = float(nu)
    d.time_block = int(time_block)
    nbytes = ctypes.c_size_t()
    _lib.check(lib.fd_diffusion_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=u.device)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    res = out if out is not None else torch.empty_like(u)
    _lib.check(lib.fd_diffusion_run(ctypes.byref(d), ctypes.c_void_p(aligned), nbytes.value,
                                    ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(res.data_ptr()),
                                    int(nt), float(dt), _stream_ptr(stream)))
    ws.record_stream(torch.cuda.current_stream() if stream is None else stream)
    return res
