"""Benchmark of libfd on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--extras all|none|...]

One bench step is one fd_forward call over the whole hot path of the
layered3d_256 workload: 256^3 physical points + 40 damping points per face
(336^3 padded), space order 8, float32, 1000 time steps, a 15 Hz Ricker
source half a cell off-grid and 256 receivers -- each time step one fused
launch (stencil update, damping, source injection, receiver sampling).

Throughput: Gpts/s = padded points x time steps / wall time of the step loop
(HIP events on the stream the kernels run on, inputs resident in HBM).  The
roofline object prices the step kernel at 16 algorithmic bytes per point
(read u^n, u^{n-1}, dt^2 v^2; write u^{n+1}) against the 8 TB/s HBM peak.
Extras (same JSON line): interior-only Gpts/s, the checkpointed gradient on
gradient3d_200, 16-bit wavefield storage, and the shot server.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
B_STEP = 16.0          # algorithmic bytes per point and step, float32 wavefields
KERNEL_SRCS = [os.path.join(ROOT, "paper_1906_10811_amd", "csrc", f)
               for f in ("fd_kernels.hip", "fd_internal.h", "fd_api.cpp")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step3d_so8_layered336.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the step kernel's source and of the host code that picks its
    launch shape (z chunking changes the bytes a launch moves)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_workload(name, torch, dev, **over):
    w = synth.workload(name, **over)
    v = synth.velocity(w)
    wav = synth.wavelets(w)
    return w, torch.from_numpy(v).to(dev), torch.from_numpy(wav).to(dev)


def time_forward(torch, g, w, wav, steps, warmup, stream):
    rec = torch.empty((w["nt"], len(w["rec"])), dtype=torch.float32, device=wav.device)
    for _ in range(warmup):
        g.forward(w["src"], wav, w["rec"], w["dt"], out=rec, stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(steps):
            g.forward(w["src"], wav, w["rec"], w["dt"], out=rec, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1000.0, rec


def bench_headline(torch, dev, steps, warmup, stream):
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    g = Grid(w["shape"], w["spacing"], v, space_order=w["space_order"], nbl=w["nbl"], origin=w["origin"],
             stream=stream)
    secs, rec = time_forward(torch, g, w, wav, steps, warmup, stream)
    pts = g.padded_points
    nt = w["nt"]
    gpts = pts * nt * steps / secs / 1e9
    interior = math.prod(w["shape"]) * nt * steps / secs / 1e9
    launch_s = secs / (steps * nt)
    achieved = B_STEP * pts / launch_s / 1e9
    traffic = stored_traffic()
    out = dict(gpts=gpts, interior=interior, ms_per_step=secs / steps * 1000.0, launch_us=launch_s * 1e6,
               achieved=achieved, traffic=traffic, pts=pts, rec_norm=float(rec.norm().item()))
    g.close()
    return w, out


def copy_probe(torch, dev, stream, nbytes=1 << 30, reps=5):
    """Measured stream-copy ceiling: torch copy of a 1 GiB float32 buffer
    (reads and writes nbytes each; reported in GB/s of read + write)."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    with torch.cuda.stream(stream):
        b.copy_(a)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            b.copy_(a)
        e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1000.0 / reps
    del a, b
    return 2.0 * nbytes / secs / 1e9


def bench_cpu_baseline(w):
    """The FP64 oracle as it stands, on the host cores, over a bounded
    sample: the same grid and medium, the first `nt` time steps."""
    import oracle
    og = oracle.Grid(tuple(w["shape"]), tuple(w["spacing"]), tuple(w["origin"]), w["space_order"], w["nbl"])
    v = synth.velocity(w)
    vp = oracle.pad_velocity(og, v)
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    wav = synth.wavelets(w).astype(np.float64)
    nt = 2
    t0 = time.perf_counter()
    oracle.forward(og, vp, sig, w["dt"], nt, w["src"], wav[:nt], w["rec"])
    t1 = time.perf_counter()
    # scale to about 15 s of work (the 2-step probe overestimates a step)
    nt2 = max(2, min(1000, int(24.0 / max(1e-3, (t1 - t0) / nt))))
    t0 = time.perf_counter()
    oracle.forward(og, vp, sig, w["dt"], nt2, w["src"], wav[:nt2], w["rec"])
    t1 = time.perf_counter()
    pts = math.prod(og.padded)
    return dict(value=pts * nt2 / (t1 - t0) / 1e9, unit="Gpts/s", cores=oracle.num_threads(), kind="oracle",
                sample="layered3d_256 grid (336^3 padded, so 8, FP64), first %d of 1000 time steps, %.1f s"
                % (nt2, t1 - t0))


def bench_gradient(torch, dev, stream):
    """fd_gradient on gradient3d_200: forward with checkpoints every 50 steps,
    residual and FP64 misfit, segment recompute, adjoint with fused imaging;
    then the binomial checkpoint schedule with 16 and 4 snapshot slots."""
    from paper_1906_10811_amd import Grid
    w = synth.workload("gradient3d_200")
    v_true = synth.velocity(w)
    v0 = synth.smooth_model(v_true, w["spacing"], 100.0)
    wav = torch.from_numpy(synth.wavelets(w)).to(dev)
    gt = Grid(w["shape"], w["spacing"], torch.from_numpy(v_true).to(dev), space_order=8, nbl=w["nbl"], stream=stream)
    d_obs = gt.forward(w["src"], wav, w["rec"], w["dt"], stream=stream)
    torch.cuda.synchronize()
    gt.close()
    g = Grid(w["shape"], w["spacing"], torch.from_numpy(v0).to(dev), space_order=8, nbl=w["nbl"], stream=stream)
    g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], checkpoint_every=w["checkpoint_every"], stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 2
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(reps):
            mis, gm, _, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"],
                                       checkpoint_every=w["checkpoint_every"], stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1000.0 / reps
    # algorithmic bytes per point and time step: forward 16 (20 with the
    # bracket write in the last segment), recompute of the other segments
    # 16 + bracket write 4, adjoint 16 + bracket read 4 + float32 partial-sum
    # read-modify-write 8, the fold into the float64 gradient (read 4, RMW 16,
    # clear 4) every 32 adjoint steps, and two field copies (read + write)
    # per checkpoint (none for the last segment; a segment is recomputed in
    # its checkpoint's own fields)
    K = w["checkpoint_every"]
    nt = w["nt"]
    nseg = -(-nt // K)
    last = nt - (nseg - 1) * K
    b_alg = 16.0 + 4.0 * last / nt + 20.0 * (nt - last) / nt + 28.0 + 24.0 / 32 + 16.0 * (nseg - 1) / nt
    gpts = g.padded_points * w["nt"] / secs / 1e9
    out = dict(workload="gradient3d_200", gpts=gpts, ms=secs * 1000.0, misfit=float(mis.item()),
               checkpoint_every=K, b_alg_per_pt=b_alg, achieved_gbs=gpts * b_alg,
               frac_hbm=gpts * b_alg / HBM_PEAK_GBS,
               workspace_gb=g.gradient_workspace_bytes(w["nt"], len(w["rec"]), checkpoint_every=K) / 1e9)
    # every bracket resident (checkpoint_every >= nt: 800 FP32 fields of 280^3
    # fit in HBM): the forward pass writes the brackets, nothing is
    # recomputed; bytes per point and step 20 + 28 + 24/32
    with torch.cuda.stream(stream):
        g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], checkpoint_every=w["nt"], stream=stream)
        torch.cuda.synchronize()
        e0.record(stream)
        misa, _, _, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], checkpoint_every=w["nt"], stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    sa = e0.elapsed_time(e1) / 1000.0
    ga = g.padded_points * w["nt"] / sa / 1e9
    ba = 48.0 + 24.0 / 32
    out["all_brackets_resident"] = dict(
        ms=sa * 1000.0, gpts=ga, b_alg_per_pt=ba, frac_hbm=ga * ba / HBM_PEAK_GBS,
        misfit_equal=bool(float(misa.item()) == float(mis.item())),
        workspace_gb=g.gradient_workspace_bytes(w["nt"], len(w["rec"]), checkpoint_every=w["nt"]) / 1e9)
    # binomial (revolve-optimal) schedules: fewer stored states, more
    # recomputation.  Bytes per point: 16 per forward advance, 20 per
    # bracket step and 28 + 24/32 per adjoint step (one each per time step);
    # snapshots are kept by reference, never copied.
    from paper_1906_10811_amd._lib import checkpoint_schedule
    nt = w["nt"]
    out["binomial"] = {}
    for slots in (16, 4):
        _, fwd = checkpoint_schedule(nt, slots)
        with torch.cuda.stream(stream):
            g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], binomial_slots=slots, stream=stream)
            torch.cuda.synchronize()
            e0.record(stream)
            misb, _, _, _ = g.gradient(w["src"], wav, w["rec"], d_obs, w["dt"], binomial_slots=slots, stream=stream)
            e1.record(stream)
        torch.cuda.synchronize()
        sb = e0.elapsed_time(e1) / 1000.0
        bytes_pt = (16.0 * fwd + (48.0 + 24.0 / 32) * nt) / nt
        gb = g.padded_points * nt / sb / 1e9
        out["binomial"]["slots%d" % slots] = dict(
            ms=sb * 1000.0, gpts=gb, forward_advances=fwd, recompute_factor=fwd / nt,
            b_alg_per_pt=bytes_pt, frac_hbm=gb * bytes_pt / HBM_PEAK_GBS,
            misfit_equal=bool(float(misb.item()) == float(mis.item())),
            workspace_gb=g.gradient_workspace_bytes(nt, len(w["rec"]), binomial_slots=slots) / 1e9)
    g.close()
    return out


def bench_precision(torch, dev, stream, ref_rec):
    """16-bit wavefield storage on layered3d_256: throughput and trace error
    against the float32 run of the same workload."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    res = {}
    ref = ref_rec.double()
    for st, scale in (("bf16", 0.0), ("f16", 0.0)):   # f16: automatic power-of-two scale
        g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], storage=st, amp_scale=scale,
                 stream=stream)
        secs, rec = time_forward(torch, g, w, wav, 1, 1, stream)
        err = float((rec.double() - ref).norm() / ref.norm())
        res[st] = dict(gpts=g.padded_points * w["nt"] / secs / 1e9, rel_l2_vs_f32=err,
                       b_alg_per_pt=10, amp_scale=scale)
        g.close()
    return res


def bench_adjoint(torch, dev, stream):
    """fd_adjoint on layered3d_256: the traces of a forward run injected back
    at the 256 receivers, F^T sampled at the source (same 16 B per point and
    step as the forward)."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], stream=stream)
    rec = g.forward(w["src"], wav, w["rec"], w["dt"], stream=stream)
    g.adjoint(w["src"], w["rec"], rec, w["dt"], stream=stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        g.adjoint(w["src"], w["rec"], rec, w["dt"], stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    secs = e0.elapsed_time(e1) / 1000.0
    gp = g.padded_points * w["nt"] / secs / 1e9
    g.close()
    return dict(gpts=round(gp, 1), ms=round(secs * 1000.0, 2), b_alg_per_pt=B_STEP,
                frac_hbm=round(gp * B_STEP / HBM_PEAK_GBS, 4))


def bench_grf512(torch, dev, stream):
    """The precision workload at full size: grf3d_512 (512^3 + 40 damping =
    592^3 padded, Gaussian random field, so 8, 1500 steps), one forward each
    with FP32, F16 (automatic scale) and BF16 wavefields; 16-bit traces are
    compared with the FP32 run (their error against the FP64 oracle is
    measured at a size the oracle can run, in the tests)."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("grf3d_512", torch, dev)
    res, ref = {}, None
    for st in ("f32", "f16", "bf16"):
        g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], storage=st, stream=stream)
        secs, rec = time_forward(torch, g, w, wav, 1, 0, stream)
        gp = g.padded_points * w["nt"] / secs / 1e9
        b = B_STEP if st == "f32" else 10.0
        res[st] = dict(gpts=round(gp, 1), frac_hbm=round(gp * b / HBM_PEAK_GBS, 4), b_alg_per_pt=b)
        if st == "f32":
            ref = rec.double()
        else:
            res[st]["rel_l2_vs_f32"] = float((rec.double() - ref).norm() / ref.norm())
        g.close()
    del v
    return res


def bench_sinc(torch, dev, stream):
    """layered3d_256 forward with Kaiser-windowed sinc sources and receivers
    (half-width 4 and 8: 512 and 4096 nodes per point) instead of the
    multilinear weights."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    res = {}
    for r in (4, 8):
        g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], sinc_radius=r, stream=stream)
        secs, _ = time_forward(torch, g, w, wav, 1, 1, stream)
        gp = g.padded_points * w["nt"] / secs / 1e9
        res["r%d" % r] = dict(gpts=round(gp, 1), nodes_per_point=(2 * r) ** 3, b_alg_per_pt=B_STEP,
                              frac_hbm=round(gp * B_STEP / HBM_PEAK_GBS, 4))
        g.close()
    return res


def bench_serving(torch, n=64, budget_gib=8.0, slots=6):
    """Shot server: n requests with Poisson arrivals at 0.8x the measured
    one-at-a-time capacity; reports shots/s, p50/p99 latency and the
    throughput in Gpts/s, against plain one-at-a-time FP32 stepping."""
    from paper_1906_10811_amd import Server
    reqs = synth.serving_requests(n=n, seed=2, rate_hz=1.0)
    shots = []
    for r in reqs:
        v = synth.layered_model(r["shape"], r["spacing"], seed=r["seed"])
        wav = synth.ricker(r["nt"], r["dt"], r["f0"]).astype(np.float32)[:, None]
        shots.append(dict(shape=r["shape"], spacing=r["spacing"], space_order=r["space_order"], nbl=r["nbl"],
                          vp=v, src_xyz=r["src"], wavelet=wav, rec_xyz=r["rec"], dt=r["dt"]))
    pts = [math.prod(s + 2 * 40 for s in r["shape"]) * r["nt"] for r in reqs]
    srv = Server(int(budget_gib * 2 ** 30), max_slots=1)
    t0 = time.perf_counter()
    for s in shots:
        srv.wait(srv.submit(**s))
    serial = time.perf_counter() - t0
    srv.close()
    cap = n / serial
    rate = 0.8 * cap
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    srv = Server(int(budget_gib * 2 ** 30), max_slots=slots)
    t0 = time.perf_counter()
    tickets = []
    for a, s in zip(arrivals, shots):
        now = time.perf_counter() - t0
        if a > now:
            time.sleep(a - now)
        tickets.append((time.perf_counter() - t0, srv.submit(**s)))
    lat = []
    for ts, t in tickets:
        _, info = srv.wait(t)
        lat.append(info["t_done"] - info["t_submit"])
    total = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return dict(requests=n, budget_gib=budget_gib, slots=slots, arrival_rate_hz=rate,
                serial_shots_per_s=cap, serial_gpts=sum(pts) / serial / 1e9,
                shots_per_s=n / total, gpts=sum(pts) / total / 1e9,
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                peak_bytes=st["peak_bytes"], peak_slots=st["peak_slots"])


def bench_diffusion(torch, dev, stream):
    """The thesis's own benchmark (Section 5.1.2): 2D diffusion, nu = 0.5,
    first order in time, FP32, 1000 steps, grids 2500^2 and 10000^2, space
    orders 2..12.  Algorithmic bytes: read u^n, write u^{n+1} = 8 B/point."""
    from paper_1906_10811_amd import diffusion
    out = {}
    for n in (2500, 10000):
        h = 1.0 / (n - 1)
        u0 = torch.ones((n, n), dtype=torch.float32, device=dev)
        u0[n // 4: n // 2, n // 4: n // 2] = 2.0
        res = torch.empty_like(u0)
        for so in (2, 4, 8, 12):
            r = so // 2
            c = [0.0] * (r + 1)
            for j in range(1, r + 1):
                c[j] = 2 * (-1) ** (j + 1) * math.factorial(r) ** 2 / (j * j * math.factorial(r - j) * math.factorial(r + j))
            s_odd = sum(c[j] for j in range(1, r + 1, 2))
            dt = 0.8 / (2.0 * s_odd * 2.0 / h ** 2) / 0.5
            diffusion(u0, (h, h), so, 0.5, dt, 10, out=res, stream=stream, time_block=1)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                e0.record(stream)
                diffusion(u0, (h, h), so, 0.5, dt, 1000, out=res, stream=stream, time_block=1)
                e1.record(stream)
            torch.cuda.synchronize()
            secs = e0.elapsed_time(e1) / 1000.0
            gpts = n * n * 1000 / secs / 1e9
            # the library's automatic choice: temporally blocked (8 B per point
            # per launch of lev steps) at so 2, 4 and 8, one step per launch otherwise
            lev = {1: 8, 2: 8, 4: 4}.get(r, 1)
            diffusion(u0, (h, h), so, 0.5, dt, 10, out=res, stream=stream, time_block=0)
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                e0.record(stream)
                diffusion(u0, (h, h), so, 0.5, dt, 1000, out=res, stream=stream, time_block=0)
                e1.record(stream)
            torch.cuda.synchronize()
            secs_tb = e0.elapsed_time(e1) / 1000.0
            gpts_tb = n * n * 1000 / secs_tb / 1e9
            out["%d^2 so%d" % (n, so)] = dict(
                gpts=round(gpts, 1), frac_hbm=round(gpts * 8.0 / HBM_PEAK_GBS, 4),
                auto_gpts=round(gpts_tb, 1), auto_steps_per_launch=lev,
                auto_frac_hbm=round(gpts_tb * 8.0 / lev / HBM_PEAK_GBS, 4))
        del u0, res
    # the FP64 oracle on the host, a few steps of the 2500^2 so-8 case
    import oracle
    n, so, steps = 2500, 8, 3
    h = 1.0 / (n - 1)
    og = oracle.Grid((n, n), (h, h), (0.0, 0.0), so)
    dt = 0.8 * oracle.diffusion_critical_dt(og, 0.5)
    u = np.ones((n, n))
    t0 = time.perf_counter()
    oracle.diffusion(og, u, 0.5, dt, steps)
    secs = time.perf_counter() - t0
    out["oracle_2500^2_so8"] = dict(gpts=round(n * n * steps / secs / 1e9, 4), steps=steps, seconds=round(secs, 2),
                                    kind="oracle (numpy, FP64)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--extras", default="all",
                    help="comma list of adjoint,gradient,precision,grf512,serving,diffusion,sinc or all/none")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only (--gpus 1): the multi-GPU sharding of the stepper "
              "(shots across GPUs, z slabs for a shot too large for one GPU) is not implemented",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(dev)
    extras = set(args.extras.split(",")) if args.extras not in ("all", "none") else (
        {"adjoint", "gradient", "precision", "grf512", "serving", "diffusion", "sinc"} if args.extras == "all"
        else set())

    copy_gbs = copy_probe(torch, dev, stream)
    log("stream copy: %.0f GB/s" % copy_gbs)
    log("headline: layered3d_256 forward, steps=%d warmup=%d" % (args.steps, args.warmup))
    w, h = bench_headline(torch, dev, args.steps, args.warmup, stream)
    log("headline: %.1f Gpts/s, %.1f us per launch" % (h["gpts"], h["launch_us"]))
    line = {
        "metric": "Gpts/s (3D so-8 acoustic step) & % HBM roofline; shots/s + p99 latency",
        "value": round(h["gpts"], 3),
        "unit": "Gpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "layered3d_256", "grid": "256^3 + 2x40 damping (336^3 padded)",
                   "space_order": 8, "time_steps_per_bench_step": w["nt"], "sources": 1, "receivers": 256},
        "interior_gpts": round(h["interior"], 3),
        "pct_hbm_roofline": round(100.0 * h["achieved"] / HBM_PEAK_GBS, 2),
        "stream_copy_gbs": round(copy_gbs, 1),
        "pct_of_stream_copy": round(100.0 * h["achieved"] / copy_gbs, 2),
        "roofline": {"bound": "hbm", "achieved": round(h["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": h["traffic"], "kernel": "k_step3d<R=4,f32>",
                     "bytes_per_point": B_STEP, "points_per_launch": h["pts"],
                     "avg_launch_us": round(h["launch_us"], 2)},
    }
    if "precision" in extras:
        log("precision: 16-bit storage")
        from paper_1906_10811_amd import Grid  # noqa: F401
        w2, v2, wav2 = make_workload("layered3d_256", torch, dev)
        g = Grid(w2["shape"], w2["spacing"], v2, space_order=8, nbl=w2["nbl"], stream=stream)
        _, ref = time_forward(torch, g, w2, wav2, 1, 0, stream)
        g.close()
        line["precision"] = bench_precision(torch, dev, stream, ref)
    if "grf512" in extras:
        log("precision workload at full size: grf3d_512")
        line["grf512"] = bench_grf512(torch, dev, stream)
    if "adjoint" in extras:
        log("adjoint: layered3d_256")
        line["adjoint"] = bench_adjoint(torch, dev, stream)
    if "sinc" in extras:
        log("windowed-sinc sparse points")
        line["sinc"] = bench_sinc(torch, dev, stream)
    if "gradient" in extras:
        log("gradient: gradient3d_200")
        line["gradient"] = bench_gradient(torch, dev, stream)
    if "diffusion" in extras:
        log("diffusion (2D, the thesis's benchmark)")
        line["diffusion2d"] = bench_diffusion(torch, dev, stream)
    if "serving" in extras:
        log("serving")
        line["serving"] = bench_serving(torch)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = bench_cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
