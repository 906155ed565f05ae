"""Continuous-batching shot server: every result equals the same shot run
alone (bitwise: same kernels, same launch geometry, deterministic
injection), admission never exceeds the HBM budget or the slot count,
requests overlap on the device, every request completes, and an oversized
request is rejected."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import need_gpu, rel_l2, torch

pytestmark = pytest.mark.gpu


def _requests(n, seed=5):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        shp = [(40, 36, 30), (48, 40, 34), (33, 45, 28)][i % 3]
        so = [4, 8, 12][int(rng.integers(3))]
        nt = int(rng.integers(60, 140))
        h = (10.0, 10.0, 10.0)
        v = synth.layered_model(shp, h, seed=100 + i)
        dt = 0.4 * 10.0 / synth.VMAX
        src = [((shp[0] - 1) * 5.0 + 2.5, (shp[1] - 1) * 5.0, 20.0)]
        rec = synth.line_receivers(16, 0.0, (shp[0] - 1) * 10.0, ((shp[1] - 1) * 5.0, 20.0), 3)
        wav = synth.ricker(nt, dt, 25.0).astype(np.float32)[:, None]
        reqs.append(dict(shape=shp, spacing=h, space_order=so, nbl=6, vp=v, src_xyz=src, wavelet=wav,
                         rec_xyz=rec, dt=dt))
    return reqs


def _alone(r):
    from paper_1906_10811_amd import Grid
    dev = torch.device("cuda:0")
    g = Grid(r["shape"], r["spacing"], torch.from_numpy(r["vp"]).to(dev), space_order=r["space_order"],
             nbl=r["nbl"])
    rec = g.forward(r["src_xyz"], torch.from_numpy(r["wavelet"]).to(dev), r["rec_xyz"], r["dt"])
    torch.cuda.synchronize()
    out = rec.cpu().numpy()
    g.close()
    return out


@pytest.mark.parametrize("policy", ["share", "shortest", "ratio"])
def test_mix_equals_alone_and_budget_holds(policy):
    need_gpu()
    from paper_1906_10811_amd import Server
    reqs = _requests(9)
    alone = [_alone(r) for r in reqs]
    sizes = [Server.request_bytes(**r) for r in reqs]
    budget = int(2.2 * max(sizes))           # two of the largest, or three smaller, fit at once
    srv = Server(budget, max_slots=3, steps_per_round=16, policy=policy)
    tickets = [srv.submit(**r) for r in reqs]
    res = [srv.wait(t, timeout=120.0) for t in tickets]
    st = srv.stats()
    srv.close()
    for k, ((out, info), ref) in enumerate(zip(res, alone)):
        assert info["status"] == 0
        assert np.array_equal(out, ref), "request %d differs from its lone run" % k
        assert info["t_submit"] <= info["t_start"] <= info["t_done"]
    assert st["peak_bytes"] <= budget
    assert 2 <= st["peak_slots"] <= 3
    # requests ran concurrently: some admitted before another one finished
    ov = sum(1 for i in range(len(res)) for j in range(i + 1, len(res))
             if res[j][1]["t_start"] < res[i][1]["t_done"] and res[i][1]["t_start"] < res[j][1]["t_done"])
    assert ov >= 1
    print("serving (%s): peak %.1f MB of %.1f MB budget, peak slots %d, overlapping pairs %d"
          % (policy, st["peak_bytes"] / 1e6, budget / 1e6, st["peak_slots"], ov))


def test_shortest_policy_lets_a_short_shot_pass():
    """With the shortest-work policy a short request submitted while a long
    one runs completes first; with equal shares it completes later than
    alone would take, as both progress."""
    need_gpu()
    from paper_1906_10811_amd import Server
    reqs = _requests(2, seed=3)
    long_r, short_r = dict(reqs[0]), dict(reqs[1])
    long_r["wavelet"] = np.tile(long_r["wavelet"], (8, 1))        # 8x the steps
    short_r["wavelet"] = short_r["wavelet"][:40].copy()
    srv = Server(1 << 30, max_slots=2, steps_per_round=10, policy="shortest")
    t_long = srv.submit(**long_r)
    t_short = srv.submit(**short_r)
    _, info_s = srv.wait(t_short, timeout=120.0)
    _, info_l = srv.wait(t_long, timeout=120.0)
    srv.close()
    print("shortest policy: short done at %.4f s, long done at %.4f s" % (info_s["t_done"], info_l["t_done"]))
    assert info_s["status"] == 0 and info_l["status"] == 0
    assert info_s["t_done"] < info_l["t_done"]


def test_server_result_matches_oracle():
    need_gpu()
    from paper_1906_10811_amd import Server
    r = _requests(1, seed=9)[0]
    srv = Server(1 << 30, max_slots=2)
    out, info = srv.wait(srv.submit(**r), timeout=120.0)
    srv.close()
    g = oracle.Grid(r["shape"], r["spacing"], (0.0, 0.0, 0.0), r["space_order"], r["nbl"])
    vp = oracle.pad_velocity(g, r["vp"])
    sig = oracle.damping(g, oracle.sigma_max_default(g, float(vp.max())))
    want, *_ = oracle.forward(g, vp, sig, r["dt"], r["wavelet"].shape[0], r["src_xyz"],
                              r["wavelet"].astype(np.float64), r["rec_xyz"])
    e = rel_l2(out, want)
    print("server vs oracle rel L2 %.3e" % e)
    assert e <= 1e-5


def test_oversized_request_rejected_and_others_complete():
    need_gpu()
    from paper_1906_10811_amd import FDError, Server
    reqs = _requests(3, seed=11)
    big = dict(reqs[0])
    big["shape"] = (120, 120, 120)
    big["vp"] = synth.layered_model(big["shape"], big["spacing"], seed=1)
    small = max(Server.request_bytes(**r) for r in reqs)
    srv = Server(int(1.5 * small), max_slots=4)
    t_big = srv.submit(**big)
    ts = [srv.submit(**r) for r in reqs]
    with pytest.raises(FDError) as e:
        srv.wait(t_big, timeout=60.0)
    assert e.value.code == -3
    for t in ts:
        out, info = srv.wait(t, timeout=120.0)
        assert info["status"] == 0 and np.isfinite(out).all() and np.abs(out).max() > 0
    srv.close()


def test_ticket_is_collected_once():
    """A second wait on a collected ticket, and a wait on a ticket never
    issued, are rejected instead of blocking."""
    need_gpu()
    from paper_1906_10811_amd import FDError, Server
    r = _requests(1, seed=13)[0]
    srv = Server(1 << 30, max_slots=1)
    t = srv.submit(**r)
    srv.wait(t, timeout=120.0)
    for bad in (t, t + 1000):
        with pytest.raises(FDError) as e:
            srv.wait(bad, timeout=5.0)
        assert e.value.code == -1
    srv.close()


def test_mixed_storage_requests_equal_alone():
    """F16, BF16 and FP32 requests resident together: each result equals the
    same shot run alone with its storage type (bitwise)."""
    need_gpu()
    from paper_1906_10811_amd import Grid, Server
    reqs = _requests(6, seed=17)
    for k, r in enumerate(reqs):
        r["storage"] = ["f32", "f16", "bf16"][k % 3]
    dev = torch.device("cuda:0")
    alone = []
    for r in reqs:
        g = Grid(r["shape"], r["spacing"], torch.from_numpy(r["vp"]).to(dev), space_order=r["space_order"],
                 nbl=r["nbl"], storage=r["storage"])
        out = g.forward(r["src_xyz"], torch.from_numpy(r["wavelet"]).to(dev), r["rec_xyz"], r["dt"])
        torch.cuda.synchronize()
        alone.append(out.cpu().numpy())
        g.close()
    srv = Server(1 << 31, max_slots=4, steps_per_round=16)
    tickets = [srv.submit(**r) for r in reqs]
    res = [srv.wait(t, timeout=120.0) for t in tickets]
    srv.close()
    for k, ((out, info), ref) in enumerate(zip(res, alone)):
        assert info["status"] == 0
        assert np.array_equal(out, ref), "request %d (%s) differs from its lone run" % (k, reqs[k]["storage"])
