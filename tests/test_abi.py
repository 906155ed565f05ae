"""The C-ABI library loads, exports every symbol include/fd.h declares, and
its host-only calls validate descriptors (no GPU needed, no compute)."""
import ctypes
import os
import re

import pytest

from paper_1906_10811_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fd_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libfd.so is not built: run `python -m paper_1906_10811_amd.build`")
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    declared = _declared()
    assert len(declared) >= 15
    assert set(declared) == set(_lib.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(**kw):
    d = _lib.GridDesc()
    d.ndim = kw.get("ndim", 3)
    shp = kw.get("shape", (64, 48, 32))
    for a in range(min(d.ndim, 3)):
        d.shape[a] = shp[a]
        d.spacing[a] = 10.0
    d.space_order = kw.get("so", 8)
    d.nbl = kw.get("nbl", 10)
    d.storage = kw.get("storage", 0)
    d.tile_x = kw.get("tile_x", 0)
    d.time_block = kw.get("time_block", 0)
    d.param_storage = kw.get("param", 0)
    return d


def _bytes(lib, d):
    n = ctypes.c_size_t()
    rc = lib.fd_grid_workspace_bytes(ctypes.byref(d), ctypes.byref(n))
    return rc, n.value


def test_workspace_bytes_grow_with_grid(lib):
    rc1, b1 = _bytes(lib, _desc(shape=(64, 48, 32)))
    rc2, b2 = _bytes(lib, _desc(shape=(128, 48, 32)))
    assert rc1 == 0 and rc2 == 0 and b2 > b1 > 0
    # 4 fields (velocity, p, two wavefields) of padded points at least
    assert b1 >= 4 * 4 * (84 * 68 * 52)
    rc3, b3 = _bytes(lib, _desc(shape=(64, 48, 32), storage=_lib.FD_STORE_BF16))
    assert rc3 == 0 and b3 < b1
    # either 3D tile shape is a valid description (their source tables differ)
    for tx in (32, 64, 96):
        rc4, b4 = _bytes(lib, _desc(shape=(64, 48, 32), tile_x=tx))
        assert rc4 == 0 and b4 > 0
    # two levels per launch (on request) keep two more wavefield buffers
    # than one step (the automatic choice)
    rc5, b5 = _bytes(lib, _desc(shape=(64, 48, 32), time_block=1))
    rc6, b6 = _bytes(lib, _desc(shape=(64, 48, 32), time_block=2))
    assert rc5 == 0 and rc6 == 0 and b5 == b1
    assert b6 - b5 >= 2 * 4 * (84 * 68 * 52)
    # value-and-difference storage keeps a third 16-bit field
    rc9, b9 = _bytes(lib, _desc(shape=(64, 48, 32), storage=_lib.FD_STORE_BF16_DIFF))
    assert rc9 == 0 and b9 - b3 >= 2 * (84 * 68 * 52) and b9 < b1
    # space order 2 in 3D float32 takes two levels per launch by default
    rc10, b10 = _bytes(lib, _desc(shape=(64, 48, 32), so=2))
    rc11, b11 = _bytes(lib, _desc(shape=(64, 48, 32), so=2, time_block=2))
    rc12, b12 = _bytes(lib, _desc(shape=(64, 48, 32), so=2, time_block=1))
    assert rc10 == rc11 == rc12 == 0 and b10 == b11 and b10 - b12 >= 2 * 4 * (84 * 68 * 52)
    rc7, b7 = _bytes(lib, _desc(shape=(64, 48, 32), so=10))
    rc8, b8 = _bytes(lib, _desc(shape=(64, 48, 32), so=10, time_block=1))
    assert rc7 == 0 and b7 == b8
    # 16-bit p codes: the parameter field takes half the bytes; at space
    # order 2 they rule out two levels per launch, so no extra buffers
    rc13, b13 = _bytes(lib, _desc(shape=(64, 48, 32), param=_lib.FD_PARAM_Q16))
    assert rc13 == 0 and b1 - b13 >= 2 * (84 * 68 * 52)
    rc14, b14 = _bytes(lib, _desc(shape=(64, 48, 32), so=2, param=_lib.FD_PARAM_Q16))
    assert rc14 == 0 and b14 < b12


@pytest.mark.parametrize("bad", [
    dict(ndim=4), dict(so=3), dict(so=18), dict(so=0), dict(nbl=-1), dict(shape=(1, 8, 8)),
    dict(storage=7), dict(tile_x=48), dict(tile_x=-32), dict(tile_x=128),
    dict(time_block=3), dict(time_block=-1), dict(time_block=2, storage=2), dict(time_block=2, so=10),
    dict(time_block=2, ndim=2), dict(storage=3, ndim=2), dict(storage=4, ndim=2), dict(storage=5),
    dict(time_block=2, storage=4),
    dict(param=2), dict(param=-1), dict(param=1, ndim=2), dict(param=1, time_block=2),
    dict(param=1, so=2, time_block=2),
])
def test_invalid_descriptors_rejected(lib, bad):
    rc, _ = _bytes(lib, _desc(**bad))
    assert rc == _lib.FD_ERR_ARG
    assert lib.fd_last_error().decode()


def test_null_arguments(lib):
    assert lib.fd_grid_workspace_bytes(None, None) == _lib.FD_ERR_ARG
    assert lib.fd_grid_destroy(None) == 0
    assert lib.fd_wait(None, 1, 0.0, None) == _lib.FD_ERR_ARG


def test_request_bytes(lib):
    r = _lib.Request()
    r.grid = _desc(shape=(32, 32, 32), nbl=8)
    r.nsrc, r.nrec, r.nt = 1, 16, 100
    n = ctypes.c_size_t()
    assert lib.fd_request_bytes(ctypes.byref(r), ctypes.byref(n)) == 0
    _, gb = _bytes(lib, _desc(shape=(32, 32, 32), nbl=8))
    assert n.value >= gb + 4 * 32 ** 3 + 4 * 100 * 17


def test_diffusion_dt_limit_is_the_von_neumann_bound(lib):
    """fd_diffusion_dt_limit against the stability bound of forward Euler:
    dt_max = 2 / (nu max_theta S), S the symbol of the 2D stencil built from
    the oracle's weights, maximised on a fine grid of wavenumbers; so 2 and
    equal spacing give the textbook h^2 / (4 nu)."""
    import numpy as np
    import oracle
    from paper_1906_10811_amd import diffusion_dt_limit
    th = np.linspace(0.0, np.pi, 20001)
    for so in (2, 4, 8, 12, 16):
        c = oracle.fd_weights(so)
        sym = -(c[0] + 2.0 * sum(c[j] * np.cos(j * th) for j in range(1, so // 2 + 1)))
        for hx, hy, nu in ((0.1, 0.1, 0.5), (2.0, 3.0, 1.7)):
            want = 2.0 / (nu * sym.max() * (1.0 / hx ** 2 + 1.0 / hy ** 2))
            got = diffusion_dt_limit((50, 40), (hx, hy), so, nu)
            assert abs(got - want) <= 1e-9 * want, (so, got, want)
    assert abs(diffusion_dt_limit((9, 9), (0.5, 0.5), 2, 2.0) - 0.5 ** 2 / 8.0) < 1e-15
    d = _lib.DiffusionDesc()
    assert lib.fd_diffusion_dt_limit(ctypes.byref(d), None) == _lib.FD_ERR_ARG
    out = ctypes.c_double()
    assert lib.fd_diffusion_dt_limit(ctypes.byref(d), ctypes.byref(out)) == _lib.FD_ERR_ARG   # zero shape
