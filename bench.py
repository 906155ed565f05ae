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
B_STEP = 16.0          # algorithmic bytes per point and step, float32 wavefields, one step per launch
B_STEP2 = 10.0         # ... two leapfrog levels per launch (20 B per point and launch)
KERNEL_SRCS = [os.path.join(ROOT, "paper_1906_10811_amd", "csrc", f)
               for f in ("fd_kernels.hip", "fd_step3d.h", "fd_step3d_f32.hip", "fd_internal.h", "fd_api.cpp")]
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


def bench_headline(torch, dev, steps, warmup, stream, time_block=0):
    """The layered3d_256 forward.  One step per launch (the automatic
    choice) moves 16 B per point; with two leapfrog levels per launch
    (time_block 2) a launch advances two time steps and moves 20 B per point
    (u^n, u^{n-1}, p in; u^{n+1}, u^{n+2} out), 10 per point-step.  The
    counted HBM traffic on record is that of the one-step kernel."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    g = Grid(w["shape"], w["spacing"], v, space_order=w["space_order"], nbl=w["nbl"], origin=w["origin"],
             time_block=time_block, stream=stream)
    secs, rec = time_forward(torch, g, w, wav, steps, warmup, stream)
    pts = g.padded_points
    nt = w["nt"]
    tb = g.time_block
    b_step = B_STEP2 if tb == 2 else B_STEP
    launches = nt // tb + nt % tb
    gpts = pts * nt * steps / secs / 1e9
    interior = math.prod(w["shape"]) * nt * steps / secs / 1e9
    launch_s = secs / (steps * launches)
    achieved = b_step * tb * pts / launch_s / 1e9
    traffic = stored_traffic() if tb == 1 else None
    out = dict(gpts=gpts, interior=interior, ms_per_step=secs / steps * 1000.0, launch_us=launch_s * 1e6,
               achieved=achieved, traffic=traffic, pts=pts, rec=rec.cpu().numpy(), time_block=tb, b_step=b_step,
               zchunk=g.zchunk)
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


def counter_references(torch, dev, stream, nbytes=1 << 30):
    """Untimed elementwise kernels of known size, so that a rocprofv3 counter
    run of this script scales FETCH_SIZE / WRITE_SIZE by kernels whose lane
    accesses match the step's: a float32 multiply (16 bytes per lane and
    access) and a float16 one (8 bytes), each reading and writing nbytes."""
    with torch.cuda.stream(stream):
        for dt in (torch.float32, torch.float16):
            n = nbytes // (4 if dt == torch.float32 else 2)
            a = torch.ones(n, dtype=dt, device=dev)
            b = torch.empty_like(a)
            torch.mul(a, 1.0, out=b)
            torch.cuda.synchronize()
            del a, b


def _oracle_setup(w, v):
    import oracle
    og = oracle.Grid(tuple(w["shape"]), tuple(w["spacing"]), tuple(w["origin"]), w["space_order"], w["nbl"])
    vp = oracle.pad_velocity(og, v)
    sig = oracle.damping(og, oracle.sigma_max_default(og, float(vp.max())))
    return og, vp, sig, synth.wavelets(w).astype(np.float64)


def bench_cpu_baseline(w, grf=None):
    """The FP64 oracle as it stands, on the host cores, over bounded samples:
    the headline grid and medium for the first time steps that take about
    15 s on all cores (its traces are also the FP64 reference the GPU traces
    of those steps are compared with), a few steps of the same on one core,
    and (grf = (workload, velocity)) the first 100 steps of grf3d_512."""
    import oracle
    og, vp, sig, wav = _oracle_setup(w, synth.velocity(w))
    pts = math.prod(og.padded)
    cores = oracle.num_threads()
    nt = 2
    t0 = time.perf_counter()
    oracle.forward(og, vp, sig, w["dt"], nt, w["src"], wav[:nt], w["rec"])
    t1 = time.perf_counter()
    # scale to about 15 s of work (the 2-step probe overestimates a step)
    nt2 = max(2, min(1000, int(24.0 / max(1e-3, (t1 - t0) / nt))))
    t0 = time.perf_counter()
    rec, *_ = oracle.forward(og, vp, sig, w["dt"], nt2, w["src"], wav[:nt2], w["rec"])
    t1 = time.perf_counter()
    out = dict(value=pts * nt2 / (t1 - t0) / 1e9, unit="Gpts/s", cores=cores, kind="oracle",
               sample="layered3d_256 grid (336^3 padded, so 8, FP64), first %d of 1000 time steps, %.1f s"
               % (nt2, t1 - t0))
    oracle.set_num_threads(1)
    one = oracle.num_threads()
    n1 = 4
    t0 = time.perf_counter()
    oracle.forward(og, vp, sig, w["dt"], n1, w["src"], wav[:n1], w["rec"])
    t1 = time.perf_counter()
    oracle.set_num_threads(cores)
    out["single_core"] = dict(value=pts * n1 / (t1 - t0) / 1e9, cores=one,
                              sample="layered3d_256 grid, first %d time steps on one core, %.1f s" % (n1, t1 - t0))
    del vp, sig
    grf_rec = None
    if grf is not None:
        wg, vg = grf
        og, vp, sig, wav = _oracle_setup(wg, vg)
        n3 = 100
        t0 = time.perf_counter()
        grf_rec, *_ = oracle.forward(og, vp, sig, wg["dt"], n3, wg["src"], wav[:n3], wg["rec"])
        t1 = time.perf_counter()
        out["grf3d_512_slice"] = dict(value=math.prod(og.padded) * n3 / (t1 - t0) / 1e9, cores=cores,
                                      sample="grf3d_512 grid (592^3 padded, so 8, FP64), first %d of 1500 time "
                                             "steps, %.1f s" % (n3, t1 - t0))
        del vp, sig
    return out, rec, grf_rec


def _vs_fp64(got, want):
    n = want.shape[0]
    g = np.asarray(got, dtype=np.float64)[:n]
    return float(np.linalg.norm(g - want) / np.linalg.norm(want))


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


def b_alg(storage, param="f32"):
    """Algorithmic bytes per point-step of the one-step forward: u^n and
    u^{n-1} (or the difference) read, u^{n+1} written, p read."""
    field = 4 if storage == "f32" else 2
    return 3 * field + (field if storage.endswith("_diff") else 0) + (2 if param == "q16" else 4)


def _forms(storages):
    """(key, storage, param) for each storage with float32 p, then each with
    16-bit p codes."""
    return [(st, st, "f32") for st in storages] + [(st + "_q16", st, "q16") for st in storages]


def bench_precision(torch, dev, stream, ref_rec):
    """16-bit wavefield storage and 16-bit p codes on layered3d_256:
    throughput and trace error against the float32 run of the same workload
    over all 1000 steps (their error against the FP64 oracle on the
    unquantised medium is added from the CPU-baseline sample).  Returns
    (results, traces per form)."""
    from paper_1906_10811_amd import Grid
    w, v, wav = make_workload("layered3d_256", torch, dev)
    res, recs = {}, {}
    ref = np.asarray(ref_rec, dtype=np.float64)
    forms = [f for f in _forms(("f32", "bf16", "f16", "bf16_diff", "f16_diff")) if f[0] != "f32"]
    for key, st, param in forms:
        # f16: automatic power-of-two scale; *_diff: the level and its difference
        g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], storage=st, param=param,
                 stream=stream)
        secs, rec = time_forward(torch, g, w, wav, 1, 1, stream)
        recs[key] = rec.cpu().numpy()
        err = float(np.linalg.norm(recs[key] - ref) / np.linalg.norm(ref))
        gp = g.padded_points * w["nt"] / secs / 1e9
        b = b_alg(st, param)
        res[key] = dict(gpts=gp, rel_l2_vs_f32=err, b_alg_per_pt=b, frac_hbm=round(gp * b / HBM_PEAK_GBS, 4))
        g.close()
    return res, recs


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
    with FP32, F16 (automatic scale), BF16 and the two difference storages,
    and FP32, F16 and BF16 with 16-bit p codes; the other traces are
    compared with the FP32 run over all 1500 steps, and every form with the
    FP64 oracle over the first 100 steps (the CPU-baseline slice).
    Returns (results, traces per storage type, (workload, velocity))."""
    from paper_1906_10811_amd import Grid
    w = synth.workload("grf3d_512")
    v_host = synth.velocity(w)
    v = torch.from_numpy(v_host).to(dev)
    wav = torch.from_numpy(synth.wavelets(w)).to(dev)
    res, recs, ref = {}, {}, None
    forms = _forms(("f32", "f16", "bf16", "f16_diff", "bf16_diff"))
    forms = forms[:5] + [f for f in forms[5:] if f[1] in ("f32", "f16", "bf16")]
    for key, st, param in forms:
        g = Grid(w["shape"], w["spacing"], v, space_order=8, nbl=w["nbl"], storage=st, param=param,
                 stream=stream)
        secs, rec = time_forward(torch, g, w, wav, 1, 0, stream)
        recs[key] = rec.cpu().numpy()
        gp = g.padded_points * w["nt"] / secs / 1e9
        b = b_alg(st, param)
        res[key] = dict(gpts=round(gp, 1), frac_hbm=round(gp * b / HBM_PEAK_GBS, 4), b_alg_per_pt=b)
        if key == "f32":
            ref = recs[key].astype(np.float64)
        else:
            res[key]["rel_l2_vs_f32"] = float(np.linalg.norm(recs[key] - ref) / np.linalg.norm(ref))
        g.close()
    del v
    return res, recs, (w, v_host)


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


def bench_serving(torch, n=64, slots=6, budget_gib=2.0, roomy_gib=32.0):
    """Shot server on the serving workload (64 requests, grids of 9-38 M
    padded points, so 4/8/12, 500-1000 steps, FP32).  Poisson arrivals at
    0.8x the measured one-at-a-time capacity.  Runs, each with shots/s,
    Gpts/s, p50/p99 latency (submission to completion, numpy linear
    percentiles) and the peak arena bytes and resident requests:
      fifo_one_at_a_time  plain FP32 stepping one shot at a time (one slot),
                          same arrivals: the baseline;
      batched             continuous batching, `slots` slots, a roomy arena
                          (the budget does not bind);
      batched_budget      the same with a budget that binds (2 GiB: about
                          three of the largest shots at once);
      *_shortest_first    the same two with the shortest-remaining-work
                          policy (at most two chunks on the device, for the
                          requests with the least remaining point-steps);
      *_response_ratio    the same two ordered by the response ratio
                          (age + remaining time) / remaining time;
      saturated_*         all requests at t = 0, one slot and `slots` slots
                          (throughput without arrival gaps)."""
    from paper_1906_10811_amd import Server
    reqs = synth.serving_requests(n=n, seed=2, rate_hz=1.0)
    shots = []
    for r in reqs:
        v = synth.layered_model(r["shape"], r["spacing"], seed=r["seed"])
        wav = synth.ricker(r["nt"], r["dt"], r["f0"]).astype(np.float32)[:, None]
        shots.append(dict(shape=r["shape"], spacing=r["spacing"], space_order=r["space_order"], nbl=r["nbl"],
                          vp=v, src_xyz=r["src"], wavelet=wav, rec_xyz=r["rec"], dt=r["dt"]))
    pts = sum(math.prod(s + 2 * 40 for s in r["shape"]) * r["nt"] for r in reqs)

    def run(budget_gib, nslots, arrivals, policy="share"):
        srv = Server(int(budget_gib * 2 ** 30), max_slots=nslots, policy=policy)
        t0 = time.perf_counter()
        tickets = []
        for a, s in zip(arrivals, shots):
            now = time.perf_counter() - t0
            if a > now:
                time.sleep(a - now)
            tickets.append(srv.submit(**s))
        lat = []
        for t in tickets:
            _, info = srv.wait(t)
            lat.append(info["t_done"] - info["t_submit"])
        total = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return dict(budget_gib=budget_gib, slots=nslots, policy=policy, shots_per_s=round(n / total, 3),
                    gpts=round(pts / total / 1e9, 1), p50_s=round(float(np.percentile(lat, 50)), 4),
                    p99_s=round(float(np.percentile(lat, 99)), 4), makespan_s=round(total, 3),
                    peak_gb=round(st["peak_bytes"] / 1e9, 3), peak_slots=st["peak_slots"])

    zeros = np.zeros(n)
    sat1 = run(roomy_gib, 1, zeros)
    cap = sat1["shots_per_s"]
    rng = np.random.default_rng(7)
    arrivals = np.cumsum(rng.exponential(1.0 / (0.8 * cap), size=n))
    out = dict(requests=n, arrival_rate_hz=round(0.8 * cap, 3), capacity_one_at_a_time_shots_per_s=cap,
               request_gb=[round(min(Server.request_bytes(**s) for s in shots) / 1e9, 3),
                           round(max(Server.request_bytes(**s) for s in shots) / 1e9, 3)])
    out["fifo_one_at_a_time"] = run(roomy_gib, 1, arrivals)
    out["batched"] = run(roomy_gib, slots, arrivals)
    out["batched_budget"] = run(budget_gib, slots, arrivals)
    out["batched_shortest_first"] = run(roomy_gib, slots, arrivals, policy="shortest")
    out["batched_budget_shortest_first"] = run(budget_gib, slots, arrivals, policy="shortest")
    out["batched_response_ratio"] = run(roomy_gib, slots, arrivals, policy="ratio")
    out["batched_budget_response_ratio"] = run(budget_gib, slots, arrivals, policy="ratio")
    out["saturated_one_slot"] = sat1
    out["saturated_batched"] = run(roomy_gib, slots, zeros)
    return out


def bench_diffusion(torch, dev, stream):
    """The thesis's own benchmark (Section 5.1.2): 2D diffusion, nu = 0.5,
    first order in time, FP32, 1000 steps, grids 2500^2 and 10000^2, space
    orders 2..12.  Algorithmic bytes: read u^n, write u^{n+1} = 8 B/point."""
    from paper_1906_10811_amd import diffusion, diffusion_dt_limit
    out = {}
    for n in (2500, 10000):
        h = 1.0 / (n - 1)
        u0 = torch.ones((n, n), dtype=torch.float32, device=dev)
        u0[n // 4: n // 2, n // 4: n // 2] = 2.0
        res = torch.empty_like(u0)
        for so in (2, 4, 8, 12):
            r = so // 2
            dt = 0.8 * diffusion_dt_limit((n, n), (h, h), so, 0.5)
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
    counter_references(torch, dev, stream)
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
        "blit_copy_gbs": round(copy_gbs, 1),
        "roofline": {"bound": "hbm", "achieved": round(h["achieved"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(h["achieved"] / HBM_PEAK_GBS, 4),
                     "traffic": h["traffic"],
                     "kernel": "k_step3d_t2<R=4>" if h["time_block"] == 2 else "k_step3d<R=4,f32>",
                     "steps_per_launch": h["time_block"], "bytes_per_point_step": h["b_step"],
                     "bytes_per_launch": h["b_step"] * h["time_block"] * h["pts"],
                     "points_per_launch": h["pts"], "avg_launch_us": round(h["launch_us"], 2)},
    }
    # the other launch form on the same workload: two leapfrog levels per
    # launch (3D temporal blocking, 10 B per point-step) when the headline
    # runs one step per launch, and the reverse
    other = 2 if h["time_block"] == 1 else 1
    _, h2 = bench_headline(torch, dev, max(1, args.steps // 2), 1, stream, time_block=other)
    line["two_levels_per_launch" if other == 2 else "one_step_per_launch"] = dict(
        gpts=round(h2["gpts"], 3), ms_per_step=round(h2["ms_per_step"], 3),
        kernel="k_step3d_t2<R=4>" if other == 2 else "k_step3d<R=4,f32>", zchunk=h2["zchunk"],
        avg_launch_us=round(h2["launch_us"], 2), bytes_per_point_step=h2["b_step"],
        frac=round(h2["achieved"] / HBM_PEAK_GBS, 4), traces_equal_bitwise=bool(np.array_equal(h2["rec"], h["rec"])))
    recs16, grf = {}, None
    if "precision" in extras:
        log("precision: 16-bit storage")
        line["precision"], recs16 = bench_precision(torch, dev, stream, h["rec"])
    if "grf512" in extras:
        log("precision workload at full size: grf3d_512")
        line["grf512"], grf_recs, grf = bench_grf512(torch, dev, stream)
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
        cpu, ref64, grf64 = bench_cpu_baseline(w, grf)
        line["cpu_baseline"] = cpu
        # the GPU traces of the sampled steps against the FP64 oracle's
        n = ref64.shape[0]
        line["vs_fp64_first_%d_steps" % n] = dict(
            f32=_vs_fp64(h["rec"], ref64), **{st: _vs_fp64(r, ref64) for st, r in recs16.items()})
        if grf64 is not None:
            line["grf512"]["vs_fp64_first_%d_steps" % grf64.shape[0]] = {
                st: _vs_fp64(r, grf64) for st, r in grf_recs.items()}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
