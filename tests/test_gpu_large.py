"""A grid whose fields exceed 2^31 elements (1280 x 1280 x 1300 points,
about 2.3e9 pitched elements per field, 9 GB in float32): every offset of
the step, the sampling, the conversions and the setup kernels needs 64
bits.  An initial-value problem (a bump in the far corner, three steps, no
damping) is compared with the FP64 oracle on the corner alone: three steps
of radius 4 reach 12 points, so a 48-point corner block whose outer faces
are the grid's own faces evolves exactly as the whole grid does, and every
point outside it must stay zero.
"""
import numpy as np
import pytest

import oracle
from gpu_common import assert_field, assert_traces, need_gpu, torch

pytestmark = pytest.mark.gpu

SHAPE = (1280, 1280, 1300)   # x, y, z
H = 10.0
SO = 8
NT = 3
K = 48                       # corner block, points per axis


def _corner_case():
    g0 = oracle.Grid((K, K, K), (H, H, H), (0.0, 0.0, 0.0), SO, 0)
    dt = 0.8 * oracle.critical_dt(g0, 2000.0)
    # a bump centred 14 points from the far faces, zero beyond 6 points
    i = np.arange(K, dtype=np.float64) - (K - 14)
    w = np.where(np.abs(i) <= 6, np.exp(-i ** 2 / 12.0), 0.0)
    bump = (w[:, None, None] * w[None, :, None] * w[None, None, :]).astype(np.float32)   # [z][y][x]
    rng = np.random.default_rng(7)
    rec_local = (K - 14 + rng.uniform(-4.0, 4.0, size=(6, 3))) * H   # metres inside the block
    return g0, dt, bump, rec_local


@pytest.mark.parametrize("storage,param,tol", [("f32", "f32", 1e-5), ("bf16", "q16", 1e-2)])
def test_fields_beyond_2_31_elements(storage, param, tol):
    need_gpu()
    from paper_1906_10811_amd import Grid
    g0, dt, bump, rec_local = _corner_case()
    vp = np.full(g0.array_shape, 2000.0)
    want, u_nt, _, _ = oracle.forward(g0, vp, np.zeros(g0.array_shape), dt, NT, np.zeros((0, 3)),
                                      np.zeros((NT, 0)), rec_local, u0=bump.astype(np.float64),
                                      u_prev=bump.astype(np.float64))
    dev = torch.device("cuda:0")
    v = torch.full((SHAPE[2], SHAPE[1], SHAPE[0]), 2000.0, device=dev)
    g = Grid(SHAPE, (H, H, H), v, space_order=SO, nbl=0, storage=storage, param=param)
    del v
    elem = 4 if storage == "f32" else 2
    assert g.field_bytes // elem > 2 ** 31
    u0 = torch.zeros(g.array_shape, device=dev)
    u0[-K:, -K:, -K:] = torch.from_numpy(bump).to(dev)
    off = np.array([(n - K) * H for n in SHAPE])
    rec, (u, _) = g.forward(np.zeros((0, 3)), torch.zeros((NT, 0), device=dev), rec_local + off, dt,
                            u0=u0, u_prev=u0, save_state=True)
    del u0
    torch.cuda.synchronize()
    corner = u[-K:, -K:, -K:]
    nz_all, nz_corner = int(torch.count_nonzero(u)), int(torch.count_nonzero(corner))
    got = corner.cpu().numpy()
    print("%s/%s: %d pitched elements per field, nonzero %d (corner %d)"
          % (storage, param, g.field_bytes // elem, nz_all, nz_corner), flush=True)
    del u
    g.close()
    torch.cuda.empty_cache()
    assert nz_all == nz_corner > 0
    # the p codes of a constant medium are exact (dp = 0), so both runs
    # step the oracle's medium
    assert_traces(rec.cpu().numpy(), want, tol, "%s beyond 2^31" % storage)
    assert_field(got, u_nt, tol, "%s beyond 2^31" % storage)
