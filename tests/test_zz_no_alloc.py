"""fd_diffusion_run_noalloc, the allocation-free variant of
fd_diffusion_run (its two fields in the library's static device scratch),
called through the C ABI: two calls in a row, the second on a smaller grid,
each against fd_diffusion_run on the same input.  Both run the same kernels
on the same layout, so the bar is bitwise equality (stricter than the
float32 tolerance).  A grid beyond the static maximum is rejected on the
host, before any device work."""
import ctypes

import numpy as np
import pytest

from gpu_common import need_gpu, torch

pytestmark = pytest.mark.gpu


def _desc(_lib, u, so, nu, tb):
    d = _lib.DiffusionDesc()
    d.shape[0], d.shape[1] = int(u.shape[1]), int(u.shape[0])
    d.spacing[0], d.spacing[1] = 1.0, 1.0
    d.space_order = so
    d.nu = nu
    d.time_block = tb
    return d


def _stable_dt(so, nu):
    r = so // 2
    import math
    c = [2 * (-1) ** (j + 1) * math.factorial(r) ** 2 / (j * j * math.factorial(r - j) * math.factorial(r + j))
         for j in range(1, r + 1)]
    s_odd = sum(c[0::2])
    return 0.8 / (2.0 * s_odd * 2.0) / nu


def _both(lib, _lib, u0, so, nt, tb):
    nu = 0.5
    dt = _stable_dt(so, nu)
    d = _desc(_lib, u0, so, nu, tb)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nbytes = ctypes.c_size_t()
    _lib.check(lib.fd_diffusion_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)))
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=u0.device)
    aligned = (ws.data_ptr() + 255) // 256 * 256
    want = torch.empty_like(u0)
    _lib.check(lib.fd_diffusion_run(ctypes.byref(d), ctypes.c_void_p(aligned), nbytes.value,
                                    ctypes.c_void_p(u0.data_ptr()), ctypes.c_void_p(want.data_ptr()), nt, dt, s))
    got = torch.full_like(u0, float("nan"))
    _lib.check(lib.fd_diffusion_run_noalloc(ctypes.byref(d), ctypes.c_void_p(u0.data_ptr()),
                                            ctypes.c_void_p(got.data_ptr()), nt, dt, s))
    torch.cuda.synchronize()
    return got, want


def test_noalloc_equals_workspace_entry_point():
    need_gpu()
    from paper_1906_10811_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(11)
    # a large grid first (most of the static scratch), then a smaller ragged
    # one: the second call must not see the first call's contents
    cases = [((2400, 2304), 8, 37, 0), ((301, 257), 4, 25, 1), ((301, 257), 16, 9, 16)]
    for (ny, nx), so, nt, tb in cases:
        u0 = torch.from_numpy(rng.uniform(0.5, 2.0, size=(ny, nx)).astype(np.float32)).to(dev)
        got, want = _both(lib, _lib, u0, so, nt, tb)
        same = bool(torch.equal(got, want))
        print("noalloc %dx%d so %d nt %d time_block %d: bitwise %d, |u| %.4e" % (
            ny, nx, so, nt, tb, int(same), float(want.norm())), flush=True)
        assert torch.isfinite(got).all() and same


def test_noalloc_rejects_grids_beyond_the_static_maximum():
    need_gpu()
    from paper_1906_10811_amd import _lib
    lib = _lib.load()
    dev = torch.device("cuda:0")
    u0 = torch.ones((4000, 4000), dtype=torch.float32, device=dev)
    out = torch.empty_like(u0)
    d = _desc(_lib, u0, 4, 0.5, 0)
    rc = lib.fd_diffusion_run_noalloc(ctypes.byref(d), ctypes.c_void_p(u0.data_ptr()),
                                      ctypes.c_void_p(out.data_ptr()), 3, _stable_dt(4, 0.5),
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.FD_ERR_NOMEM
    assert b"static maximum" in lib.fd_last_error()
