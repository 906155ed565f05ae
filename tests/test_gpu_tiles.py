"""The 3D workgroup tile shapes: 64 x 16 and 32 x 32 points in xy, and the
mixed launch (64 x 16 tiles with a last x column of 32 x 32, tile_x 96).

Each point's update is the same sequence of float32 operations whatever
tile computes it, and source terms are summed per grid point in a fixed
order, so every result must be bitwise the same under every shape: traces,
final fields, adjoint source traces and gradients, for every storage type.
The oracle parity of each shape on its own is covered by the 3D parity
tests, which run all three.
"""
import numpy as np
import pytest

from gpu_common import case, gpu_forward, gpu_grid, need_gpu, oracle_forward, rel_l2, torch

pytestmark = pytest.mark.gpu


def _shapes(c, shapes=(64, 32, 96), **kw):
    out = []
    kw.setdefault("time_block", 1)   # the one-step kernel, whose tile shape is chosen
    for tx in shapes:
        g = gpu_grid(c, tile_x=tx, **kw)
        assert g.tile == ((32, 32) if tx == 32 else (64, 16))
        assert (g.tile_strip > 0) == (tx == 96)
        _, (rec, state) = gpu_forward(c, grid=g, save_state=True)
        out.append((rec, state))
        g.close()
    return out


@pytest.mark.parametrize("param", ["f32", "q16"])
@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f16_diff", "bf16_diff"])
@pytest.mark.parametrize("so", [4, 8, 16])
def test_forward_bitwise_across_tile_shapes(storage, so, param):
    """80 x 70 x 33 + 6 (92 x 82 x 45 padded): ragged last tiles in x and y
    under every shape, the mixed one with a 28-point strip of 32 x 32
    tiles; 4 sources, 13 receivers, 50 steps; p in float32 or as 16-bit
    codes."""
    need_gpu()
    c = case((80, 70, 33), so, 6, 50, seed=40 + so, nsrc=4, nrec=13)
    shapes = (64, 32, 96) if so < 14 else (64, 32)
    res = _shapes(c, shapes, storage=storage, param=param)
    (r1, s1) = res[0]
    for tx, (r2, s2) in zip(shapes[1:], res[1:]):
        print("tiles %s p %s so=%d, %d vs 64: traces equal %d, field equal %d" % (
            storage, param, so, tx, int(torch.equal(r1, r2)), int(torch.equal(s1[0], s2[0]))), flush=True)
        assert torch.equal(r1, r2)
        assert torch.equal(s1[0], s2[0]) and torch.equal(s1[1], s2[1])


def test_narrow_tiles_against_oracle_many_sources():
    """Sources spread over several 32 x 32 tiles and planes (scatter with the
    narrow row stride), windowed-sinc nodes shared between tiles."""
    need_gpu()
    c = case((75, 69, 28), 8, 4, 40, seed=77, nsrc=12, nrec=9)
    c["sinc"] = 3
    want, u_nt, _, _ = oracle_forward(c)
    g = gpu_grid(c, tile_x=32, time_block=1)
    _, (rec, state) = gpu_forward(c, grid=g, save_state=True)
    e_rec = rel_l2(rec.cpu().numpy(), want)
    e_u = rel_l2(state[0].cpu().numpy(), u_nt)
    print("32x32 tiles, sinc 3, 12 sources: traces %.3e field %.3e" % (e_rec, e_u), flush=True)
    assert e_rec <= 1e-5 and e_u <= 1e-5


def test_adjoint_and_gradient_bitwise_across_tile_shapes():
    """fd_adjoint and fd_gradient (recomputing schedule, and every bracket
    resident) give bitwise the same outputs under either tile shape."""
    need_gpu()
    c = case((60, 45, 30), 8, 5, 70, seed=8, nsrc=2, nrec=11)
    dev = torch.device("cuda:0")
    wav = torch.from_numpy(c["wav"]).to(dev)
    rng = np.random.default_rng(4)
    obs = torch.from_numpy(rng.standard_normal((c["nt"], len(c["rec"]))).astype(np.float32) * 1e-3).to(dev)
    outs = []
    for tx in (64, 32, 96):
        g = gpu_grid(c, tile_x=tx)
        assert (g.tile_strip > 0) == (tx == 96)
        adj = g.adjoint(c["src"], c["rec"], obs, c["dt"])
        grads = [g.gradient(c["src"], wav, c["rec"], obs, c["dt"], checkpoint_every=K) for K in (9, c["nt"])]
        torch.cuda.synchronize()
        outs.append((adj, grads))
        g.close()
    (a1, g1) = outs[0]
    for (a2, g2) in outs[1:]:
        assert torch.equal(a1, a2)
        for x, y in zip(g1, g2):
            assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1]) and torch.equal(x[2], y[2])
    print("adjoint and gradients bitwise equal across tile shapes", flush=True)


@pytest.mark.parametrize("shape,so,storage,want,strip", [
    ((200, 200, 40), 8, "f32", (64, 16), 24),    # padded x 280 = 4 x 64 + a 24-point strip of 32 x 32
    ((240, 200, 40), 8, "f32", (64, 16), 0),     # padded x 320: whole 64-point columns only
    ((230, 200, 40), 8, "f32", (64, 16), 0),     # padded x 310: a 54-point last column stays 64 x 16
    ((200, 200, 40), 8, "bf16", (64, 16), 0),    # 16-bit: no strip (half-line rows)
    ((200, 200, 40), 12, "f32", (64, 16), 24),   # so 12 on 280: the strip beats 32 x 32 tiles
    ((200, 200, 40), 12, "f16", (32, 32), 0),    # 16-bit so 12 on 280: 32 x 32 uses 9 % more lanes
    ((240, 200, 40), 12, "f16", (64, 16), 0),    # padded x 320: whole 64-point rows
    ((240, 200, 40), 16, "f32", (32, 32), 0),    # so >= 14: always 32 x 32
    ((31, 20), 16, "f32", (64, 64), 0),          # 2D: 64 x-points by 64 z-rows
])
def test_automatic_tile_choice(shape, so, storage, want, strip):
    need_gpu()
    dev = torch.device("cuda:0")
    from paper_1906_10811_amd import Grid
    v = torch.full(tuple(reversed(shape)), 2000.0, device=dev)
    g = Grid(shape, (10.0,) * len(shape), v, space_order=so, nbl=40, storage=storage)
    print("padded", g.padded, "so", so, "tile", g.tile, "strip", g.tile_strip, "zchunk", g.zchunk, flush=True)
    assert g.tile == want and g.tile_strip == strip
    g.close()


@pytest.mark.parametrize("sinc", [0, 4])
def test_sources_on_the_strip_seam(sinc):
    """Mixed shape: sources on both sides of the seam between the 64 x 16
    tiles and the 32 x 32 strip (padded x 63, 64, 65 and inside the strip),
    windowed-sinc nodes that straddle it, receivers likewise; bitwise equal
    to 64 x 16 tiles alone and within the gate of the oracle."""
    need_gpu()
    c = case((76, 40, 30), 8, 3, 50, seed=31, nsrc=1, nrec=1)   # padded x 82: seam at 64, strip of 18
    h, o = c["spacing"], c["origin"]
    xs = [60.5, 63.0, 63.7, 64.0, 64.4, 70.2, 77.6]            # padded x (physical x + 3)
    c["src"] = [(o[0] + (x - 3) * h[0], o[1] + (9.3 + 3 * k) * h[1], o[2] + (11.6 + k) * h[2])
                for k, x in enumerate(xs)]
    c["rec"] = np.array([[o[0] + (x - 3 + 0.37) * h[0], o[1] + 20.5 * h[1], o[2] + 6.2 * h[2]] for x in xs])
    rng = np.random.default_rng(2)
    c["wav"] = (rng.standard_normal((c["nt"], len(xs))) * np.hanning(c["nt"])[:, None]).astype(np.float32)
    c["sinc"] = sinc
    want, u_nt, _, _ = oracle_forward(c)
    (r1, s1), (r2, s2) = _shapes(c, (64, 96))
    e_rec = rel_l2(r2.cpu().numpy(), want)
    e_u = rel_l2(s2[0].cpu().numpy(), u_nt)
    print("seam sinc=%d: traces %.3e field %.3e, bitwise %d" % (sinc, e_rec, e_u, int(torch.equal(r1, r2))),
          flush=True)
    assert torch.equal(r1, r2) and torch.equal(s1[0], s2[0])
    assert e_rec <= 1e-5 and e_u <= 1e-5
