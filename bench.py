#!/usr/bin/env python3
"""Throughput of the SRT3D hot path on one MI355X.

One step = the photon sketch of a 256x256 frame (T = 4096 bins, ~1000 photons per pixel,
SBR = 1, m = 16 harmonics; ~6.6e7 int32 stamps resident in HBM) followed by the SRT3D
reconstruction of that sketch (initialisation, 50 iterations of data step + depth denoiser +
intensity denoiser, background and output).  Prints one JSON line.  The sketch runs on the
binned path by default (per-pixel histogram on the FP16 matrix cores); --sketch photon times
the photon-parallel FP32 pass instead.  Both meet the same tolerance against the oracle, and
the line reports the other one's time beside the timed steps.

    python bench.py [--steps K] [--warmup W] [--workload throughput] [--sketch binned|photon]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photons sketched/s + SRT3D frames/s (fraction of HBM roofline); p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# per sketch method: (kernel name, its source file, the committed HBM-counter summary)
SKETCH_KERNELS = {
    "binned": ("sketch_binned_kernel", "binned.hip", "traffic_{w}.md"),
    "photon": ("sketch_photons_kernel", "sketch.hip", "traffic_{w}.md"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="throughput")
    ap.add_argument("--sketch", default="binned", choices=sorted(SKETCH_KERNELS),
                    help="sketch path timed in the step (both meet the same oracle tolerance)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=96, help="serving workload: number of requests")
    ap.add_argument("--graph", action="store_true",
                    help="replay the reconstruction's kernels from a HIP graph captured during the warm-up "
                         "(the line then also carries the host-launched figure as `eager`)")
    ap.add_argument("--frames-in-flight", type=int, default=4,
                    help="streams of the frames-in-flight leg in the default line (0 = skip; profile runs skip "
                         "it so that the traced kernel times are those of lone frames)")
    ap.add_argument("--serving-requests", type=int, default=96,
                    help="requests of the short serving leg in the default line (0 = skip)")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serving workload: HBM budget")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (scale reference for HBM counters)")
    return ap.parse_args()


def profile_figure(summary: str, src: str, key: str):
    """A figure from a committed rocprofv3 summary under profiles/ (the line `key: value`), if the
    summary records the sha256 of the current kernel source `src` (else None: the counters were
    taken on other code)."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2203_00952_amd", "csrc", src), "rb").read()).hexdigest()
    m_sha = re.search(re.escape(src) + r" sha256:\s*([0-9a-f]{64})", text)
    m_v = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    if not m_sha or not m_v or m_sha.group(1) != sha:
        return None
    return float(m_v.group(1))


def sketch_traffic(method: str, workload: str):
    """HBM bytes per sketch launch from the committed counter summary (None if stale)."""
    kernel, src, summary = SKETCH_KERNELS[method]
    return profile_figure(summary.format(w=workload), src, f"{kernel} traffic_bytes_per_launch")


VALU_PEAK = 256 * 2.4e9        # wave64 VALU instructions per second: one per clock per CU


def valu_per_launch(kernel: str, src: str, workload: str):
    """VALU wave instructions per launch of `kernel` from the committed counter summary of the
    workload (None if stale or absent)."""
    return profile_figure(f"valu_counters_{workload}.md", src, f"{kernel} VALU wave instructions per launch")


def iteration_bytes_per_pixel(m: int, K: int) -> float:
    """Algorithmic HBM bytes per pixel of one fused iteration: the sketch (8 m) and the photon count
    (4) in, the point state (t and alpha, 4 B each per point, and the activity word) in and out."""
    return 8.0 * m + 4.0 + 2.0 * (8.0 * K + 4.0)


def _oracle_sketch_chunk(args):
    """Worker of the all-cores CPU baseline: the oracle's sketch of one contiguous block of
    pixels (a spawned process: it imports numpy and the oracle only)."""
    stamps, offsets, T, m = args
    from threadpoolctl import threadpool_limits

    from oracle import sketch as OS
    with threadpool_limits(limits=1):
        return OS.sketch(stamps, offsets, T, m)


def cpu_cores() -> int:
    """Host cores the baseline may use: the process's CPU set, at most 16 (one GPU's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_all_cores(frame, w, params):
    """The oracle on the whole frame with every host core: the FP64 sketch of all pixels split
    into contiguous blocks over a process pool, then the FP64 SRT3D oracle (init, all iterations,
    background, output) in this process on the pool-computed sketch, numpy's thread pools
    limited to the same core count.  Wall time of both, no extrapolation."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import srt3d as O

    spec = frame.spec
    cores = cpu_cores()
    st_np, off_np = frame.stamps.cpu().numpy(), frame.offsets.cpu().numpy()
    bounds = np.linspace(0, spec.P, 4 * cores + 1).astype(np.int64)
    chunks = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        lo, hi = off_np[a], off_np[b]
        chunks.append((st_np[lo:hi], off_np[a:b + 1] - lo, spec.T, w.m))
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_sketch_chunk, chunks[:cores])          # start-up and imports, untimed
        t0 = time.perf_counter()
        parts = pool.map(_oracle_sketch_chunk, chunks)
        t_sketch = time.perf_counter() - t0
    zc = np.concatenate([p[0] for p in parts])
    nn = np.concatenate([p[1] for p in parts]).astype(np.int64)
    op = O.Params(spec.T, w.m, w.K_max, iters=params.iters, r_min=params.r_min)
    with threadpool_limits(limits=cores):
        t0 = time.perf_counter()
        O.reconstruct(zc, nn, frame.irf, frame.irf_origin, spec.rows, spec.cols, op)
        t_srt3d = time.perf_counter() - t0
    per_frame = t_sketch + t_srt3d
    return {
        "value": 1.0 / per_frame, "unit": "frames/s", "cores": cores, "kind": "oracle",
        "sample": (f"FP64 numpy oracle on the whole frame: sketch of all {spec.P} pixels over a pool of "
                   f"{cores} processes ({t_sketch:.2f} s), then init + {params.iters} iterations + background "
                   f"+ output in one process with numpy's thread pools limited to {cores} ({t_srt3d:.2f} s)"),
        "photons_per_s": float(frame.stamps.numel()) / t_sketch,
    }


def cpu_baseline(frame, z_gpu, n_gpu, w, params):
    """Time the FP64 oracle on this host, single-threaded, on a bounded sample of the step."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import sketch as OS
    from oracle import srt3d as O

    spec = frame.spec
    st_np, off_np = frame.stamps.cpu().numpy(), frame.offsets.cpu().numpy()
    zc = z_gpu.cpu().numpy().astype(np.float64)
    zc = zc[..., 0] + 1j * zc[..., 1]
    nn = n_gpu.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(0)
    S = min(2048, spec.P)
    sel = np.sort(rng.choice(spec.P, S, replace=False))
    it_sample = 5
    op = O.Params(spec.T, w.m, w.K_max, iters=params.iters, r_min=params.r_min)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        OS.sketch(st_np, off_np, spec.T, w.m, pixels=sel)
        t_sketch = (time.perf_counter() - t0) * spec.P / S
        hhat = O.irf_spectrum(frame.irf, frame.irf_origin, spec.T, w.m)
        tau_z = O.default_tau_z(frame.irf, frame.irf_origin, op)
        t0 = time.perf_counter()
        st = O.init_points(zc, nn, hhat, op)
        t_init = time.perf_counter() - t0
        t0 = time.perf_counter()
        st = O.iterate(st, zc, nn, hhat, spec.rows, spec.cols, op, tau_z, it_sample)
        t_iter = (time.perf_counter() - t0) / it_sample
        t0 = time.perf_counter()
        O.output(st, nn)
        O.background(st, nn, spec.rows, spec.cols, op)
        t_fin = time.perf_counter() - t0
    per_frame = t_sketch + t_init + params.iters * t_iter + t_fin
    return {
        "value": 1.0 / per_frame, "unit": "frames/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 numpy oracle, 1 thread: sketch of {S} random pixels of the frame scaled to "
                   f"{spec.P} pixels ({t_sketch:.1f} s/frame), full-frame init ({t_init:.2f} s) and "
                   f"{it_sample} full-frame iterations scaled to {params.iters} ({t_iter:.2f} s each)"),
        "photons_per_s": float(frame.stamps.numel()) / t_sketch,
    }


def precision_report(args):
    """Histogram sketch (256x256 x T=1024 uint16, ~4000 photons/pixel, m=16) in the three
    arithmetic forms next to the photon sketch of the same frame; errors against the FP64
    oracle per harmonic on sampled pixels, times by HIP events."""
    import numpy as np
    import torch

    import paper_2203_00952_amd as srt
    import synth
    from oracle import sketch as OS

    dev = torch.device("cuda:0")
    w = synth.preset("precision")
    spec = w.frame
    frame = synth.make_frame(spec, device=dev)
    H = synth.histogram(frame.stamps, frame.offsets, spec.T)
    P, T, m = spec.P, spec.T, w.m
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(P, 2048, replace=False))
    zr, nr = OS.sketch_hist(synth.frames.hist_as_uint(H[torch.from_numpy(sel).to(dev)]), m)
    floor = 1.0 / np.sqrt(np.maximum(nr, 1))[:, None]
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
        for i in range(args.steps):
            ev[2 * i].record(stream)
            out = fn()
            ev[2 * i + 1].record(stream)
        torch.cuda.synchronize()
        return out, float(np.mean([ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)]))

    forms = {}
    table = srt.phase_table(T, dev)
    (zp, _), t_ph = timed(lambda: srt.sketch(frame.stamps, frame.offsets, T, m, table=table))
    zpc = zp.cpu().numpy().astype(np.float64)
    zpc = zpc[..., 0] + 1j * zpc[..., 1]
    for prec in ("fp32", "fp16x2", "bf16x3"):
        ws = srt.hist_workspace(T, m, prec, dev)
        (z, _), t_ms = timed(lambda: srt.sketch_from_hist(H, m, prec, workspace=ws))
        zc = z.cpu().numpy().astype(np.float64)
        zc = zc[..., 0] + 1j * zc[..., 1]
        rel = np.abs(zc[sel] - zr) / np.maximum(np.abs(zr), floor)
        hbytes = 2.0 * P * T + 8.0 * m * P + 4.0 * P
        forms[prec] = {"ms": t_ms, "GB_per_s": hbytes / (t_ms * 1e-3) / 1e9,
                       "hbm_frac": hbytes / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "max_rel_err_vs_oracle_per_harmonic": [float(v) for v in rel.max(0)],
                       "p99_rel_err_vs_oracle": float(np.percentile(rel, 99)),
                       "max_rel_diff_vs_photon_path": float(np.max(np.abs(zc - zpc) / np.maximum(
                           np.abs(zpc), 1.0 / np.sqrt(np.maximum(frame.n.cpu().numpy(), 1))[:, None])))}
    rel = np.abs(zpc[sel] - zr) / np.maximum(np.abs(zr), floor)
    forms["photon_fp32"] = {"ms": t_ph, "max_rel_err_vs_oracle_per_harmonic": [float(v) for v in rel.max(0)]}
    print(json.dumps({"workload": w.name, "pixels": P, "T": T, "m": m, "photons": int(frame.stamps.numel()),
                      "error_rule": "|dz| / max(|z_ref|, n^-1/2), 2048 sampled pixels", "forms": forms}),
          flush=True)


def frames_in_flight(frame, w, params, irf, table, method: str, streams: int, rounds: int, ref_out):
    """`streams` frames at a time, each step (sketch + reconstruct) of a frame on its own HIP
    stream (default priority) with its own outputs and Reconstructor; `rounds` frames per stream.
    Returns frames/s over the streams * rounds frames, timed with events on the current stream
    that every stream waits for and that waits for every stream, and whether every stream's
    output equals `ref_out` (the single-stream step's) bit for bit."""
    import torch

    import paper_2203_00952_amd as srt

    dev = frame.stamps.device
    spec = w.frame
    P, T, m = spec.P, spec.T, w.m
    cur = torch.cuda.current_stream(dev)
    lanes = []
    for _ in range(streams):
        lanes.append(dict(s=torch.cuda.Stream(dev), rec=srt.Reconstructor(params, dev),
                          z=torch.empty((P, m, 2), dtype=torch.float32, device=dev),
                          n=torch.empty(P, dtype=torch.int32, device=dev),
                          out=dict(depth=torch.empty((P, w.K_max), dtype=torch.float32, device=dev),
                                   intensity=torch.empty((P, w.K_max), dtype=torch.float32, device=dev),
                                   active=torch.empty((P, w.K_max), dtype=torch.uint8, device=dev),
                                   bg=torch.empty(P, dtype=torch.float32, device=dev))))
    torch.cuda.synchronize()

    def run(k):
        start = torch.cuda.Event()
        start.record(cur)
        for ln in lanes:
            ln["s"].wait_event(start)
        for _ in range(k):
            for ln in lanes:
                with torch.cuda.stream(ln["s"]):
                    srt.sketch(frame.stamps, frame.offsets, T, m, z=ln["z"], n=ln["n"], table=table, method=method)
                    ln["rec"].reconstruct(ln["z"], ln["n"], irf, frame.irf_origin, out=ln["out"])
        for ln in lanes:
            done = torch.cuda.Event()
            done.record(ln["s"])
            cur.wait_event(done)

    run(1)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record(cur)
    run(rounds)
    e[1].record(cur)
    torch.cuda.synchronize()
    ms = e[0].elapsed_time(e[1])
    same = all(torch.equal(ln["out"][k], ref_out[k]) for ln in lanes for k in ref_out)
    del lanes
    return {"streams": streams, "frames": streams * rounds, "ms": ms,
            "frames_per_s": streams * rounds / (ms * 1e-3), "same_as_step": same}


def serving_measure(count: int, budget_bytes: int, seed: int = 4):
    """Continuous batching of a Poisson stream of `count` frames (32^2..512^2, 10..2000
    photons/px, T = 2048, m = 8..32, sketch + 20 iterations each).  The single-slot sequential
    capacity is measured first; the stream is then replayed at 0.5x and 0.9x that rate on 4
    slots under an HBM budget.  Latency = completion - arrival (host clock)."""
    import numpy as np
    import torch

    import paper_2203_00952_amd as srt
    import synth
    from paper_2203_00952_amd.serve import Request, percentile, serve

    dev = torch.device("cuda:0")
    stream = synth.request_stream(seed=seed, count=count, rate_hz=1.0, iters=20)
    reqs, photons = [], 0
    for q in stream:
        f = synth.make_frame(q.frame, device=dev)
        params = srt.Params.default(q.frame.rows, q.frame.cols, q.frame.T, q.m, 1, iters=q.iters)
        reqs.append(Request(q.rid, f.stamps, f.offsets, torch.from_numpy(f.irf).to(dev), f.irf_origin, params))
        photons += int(f.stamps.numel())
    torch.cuda.synchronize()
    serve(reqs[:4], slots=1, budget_bytes=budget_bytes)                 # warm-up
    for r in reqs:
        r.arrival = 0.0
    recs, _, _ = serve(reqs, slots=1, budget_bytes=budget_bytes)
    capacity = len(reqs) / max(r.finished for r in recs)
    res = {"workload": "serving", "requests": len(reqs), "photons": photons, "slots": 4,
           "sizes": sorted({q.frame.rows for q in stream}), "hbm_budget_bytes": budget_bytes,
           "single_slot_capacity_frames_per_s": capacity}
    for load in (0.5, 0.9):
        rate = load * capacity
        for r, q in zip(reqs, stream):
            r.arrival = q.arrival_s / rate
        recs, _, peak = serve(reqs, slots=4, budget_bytes=budget_bytes)
        lat = [1e3 * r.latency for r in recs]
        makespan = max(r.finished for r in recs)
        res[f"load_{load}"] = {"arrival_rate_per_s": rate, "p50_ms": percentile(lat, 50),
                               "p99_ms": percentile(lat, 99), "mean_ms": float(np.mean(lat)),
                               "frames_per_s": len(reqs) / makespan, "peak_admitted_bytes": peak}
    del reqs
    torch.cuda.empty_cache()
    return res


def serving_report(args):
    """The serving workload alone (`--requests` frames), one JSON line."""
    print(json.dumps(serving_measure(args.requests, int(args.budget_gib * (1 << 30)))), flush=True)


def table1_report(args):
    """SRT3D reconstruction time per frame on synthetic frames of the shapes the paper's Table 1
    times (141^2 .. 705^2 px, T = 4613, m = 5 and 10, one surface), 50 iterations (the paper does
    not state its count; photons/px does not change the reconstruction's work).  Context only:
    the paper's numbers come from another GPU, an unstated precision and the head dataset."""
    import numpy as np
    import torch

    import paper_2203_00952_amd as srt
    import synth

    dev = torch.device("cuda:0")
    paper_ms = {5: [6, 12, 28, 55, 68], 10: [7, 18, 35, 60, 88]}
    out = {"workload": "table1", "T": 4613, "iters": 50, "photons_per_pixel": 100, "rows": []}
    for si, side in enumerate((141, 282, 423, 564, 705)):
        spec = synth.FrameSpec(side, side, 4613, 8.0, 100.0, 1.0, 1, seed=30 + si)
        f = synth.make_frame(spec, device=dev)
        irf = torch.from_numpy(f.irf).to(dev)
        for m in (5, 10):
            z, n = srt.sketch(f.stamps, f.offsets, spec.T, m)
            params = srt.Params.default(side, side, spec.T, m, 1, iters=50)
            rec = srt.Reconstructor(params, dev)
            outb = None
            for _ in range(2):
                outb = rec.reconstruct(z, n, irf, f.irf_origin, out=outb)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            reps = 10
            ev[0].record()
            for _ in range(reps):
                rec.reconstruct(z, n, irf, f.irf_origin, out=outb)
            ev[1].record()
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / reps
            out["rows"].append({"pixels": side * side, "side": side, "m": m, "srt3d_ms": ms,
                                "frames_per_s": 1e3 / ms, "paper_ms_rtx3070_laptop": paper_ms[m][si]})
            del rec, z, n
        del f
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def nsweep_report(args):
    """Sketch and SRT3D times against photons per pixel on 256x256 frames (T = 4096, m = 16,
    50 iterations): the sketch grows with the photon count, the reconstruction from the sketch
    does not (the claim of Section 1 / Fig. 1 for SRT3D)."""
    import torch

    import paper_2203_00952_amd as srt
    import synth

    dev = torch.device("cuda:0")
    out = {"workload": "nsweep", "pixels": 65536, "T": 4096, "m": 16, "iters": 50, "rows": []}
    for lam in (10.0, 100.0, 1000.0, 4000.0):
        spec = synth.FrameSpec(256, 256, 4096, 8.0, lam, 1.0, 1, seed=40)
        f = synth.make_frame(spec, device=dev)
        irf = torch.from_numpy(f.irf).to(dev)
        params = srt.Params.default(256, 256, 4096, 16, 1, iters=50)
        rec = srt.Reconstructor(params, dev)
        z, n = srt.sketch(f.stamps, f.offsets, spec.T, 16, method="binned")
        o = rec.reconstruct(z, n, irf, f.irf_origin)
        torch.cuda.synchronize()
        z2, n2 = srt.sketch(f.stamps, f.offsets, spec.T, 16, method="photon")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        reps = 10
        ev[0].record()
        for _ in range(reps):
            srt.sketch(f.stamps, f.offsets, spec.T, 16, z=z, n=n, method="binned")
        ev[1].record()
        for _ in range(reps):
            srt.sketch(f.stamps, f.offsets, spec.T, 16, z=z2, n=n2, method="photon")
        ev[2].record()
        for _ in range(reps):
            rec.reconstruct(z, n, irf, f.irf_origin, out=o)
        ev[3].record()
        torch.cuda.synchronize()
        out["rows"].append({"photons_per_pixel": lam, "photons": int(f.stamps.numel()),
                            "sketch_binned_ms": ev[0].elapsed_time(ev[1]) / reps,
                            "sketch_photon_ms": ev[1].elapsed_time(ev[2]) / reps,
                            "srt3d_ms": ev[2].elapsed_time(ev[3]) / reps})
        del z2, n2
        del f, z, n, rec
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the library has no "
                                   "multi-GPU path (pixels would shard with no communication)"}))
        sys.exit(2)
    if args.workload == "precision":
        precision_report(args)
        return
    if args.workload == "serving":
        serving_report(args)
        return
    if args.workload == "table1":
        table1_report(args)
        return
    if args.workload == "nsweep":
        nsweep_report(args)
        return

    import numpy as np
    import torch

    import paper_2203_00952_amd as srt
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = synth.preset(args.workload)
    spec = w.frame
    frame = synth.make_frame(spec, device=dev)
    N = frame.stamps.numel()
    P, T, m = spec.P, spec.T, w.m
    params = srt.Params.default(spec.rows, spec.cols, T, m, w.K_max, iters=w.iters, r_min=w.r_min)
    irf = torch.from_numpy(frame.irf).to(dev)
    table = srt.phase_table(T, dev)
    z = torch.empty((P, m, 2), dtype=torch.float32, device=dev)
    n = torch.empty(P, dtype=torch.int32, device=dev)
    rec = srt.Reconstructor(params, dev)
    out = dict(depth=torch.empty((P, w.K_max), dtype=torch.float32, device=dev),
               intensity=torch.empty((P, w.K_max), dtype=torch.float32, device=dev),
               active=torch.empty((P, w.K_max), dtype=torch.uint8, device=dev),
               bg=torch.empty(P, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()

    if args.calibrate_copy:
        a = torch.ones(1 << 26, dtype=torch.float32, device=dev)    # 256 MiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    stream = torch.cuda.current_stream(dev)

    # --graph: the reconstruction's ~55 dependent launches (setup, init, data step, 50
    # iterations, finalize) are captured once into a HIP graph, through torch's CUDAGraph wrapper
    # of stream capture, and replayed each step; the sketch (one launch) stays a host launch.
    # srt3d_reconstruct is capturable (no allocation, memset or host synchronisation, and init
    # resets the state's ping-pong index, so every replay runs the same launches on the same
    # buffers).  Measured on this workload, replay and host launches take the same time.
    graph = None

    def reconstruct():
        if graph is not None:
            graph.replay()
        else:
            rec.reconstruct(z, n, irf, frame.irf_origin, out=out)

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        srt.sketch(frame.stamps, frame.offsets, T, m, z=z, n=n, table=table, method=args.sketch)
        if ev:
            ev[1].record(stream)
        reconstruct()
        if ev:
            ev[2].record(stream)

    def timed_steps(k):
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(k)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(k):
            step(evs[i])
        torch.cuda.synchronize()
        return evs, time.perf_counter() - t0

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    eager_evs, eager_wall = None, None
    if args.graph:
        # the same number of host-launched steps first, for the line's `eager` entry
        eager_evs, eager_wall = timed_steps(args.steps)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, capture_error_mode="relaxed"):
            rec.reconstruct(z, n, irf, frame.irf_origin, out=out)
        torch.cuda.synchronize()
        graph = g
        step()                                        # the graph's first replay, untimed
        torch.cuda.synchronize()
    evs, wall = timed_steps(args.steps)

    sk_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    rc_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    st_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps

    # algorithmic bytes of one sketch launch: stamps + offsets in, sketch + counts out
    alg_bytes = 4.0 * N + 8.0 * (P + 1) + 8.0 * m * P + 4.0 * P
    achieved = alg_bytes / (sk_ms.mean() * 1e-3) / 1e9
    traffic = sketch_traffic(args.sketch, w.name)
    valu = valu_per_launch(SKETCH_KERNELS[args.sketch][0], SKETCH_KERNELS[args.sketch][1], w.name)
    kernel = SKETCH_KERNELS[args.sketch][0]

    # the fused iteration alone (outside the timed steps, on the stream it is launched on): the
    # average launch of `iters` back-to-back iterations from the last step's state
    e_i = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    rec.iterate(z, n, params.iters)
    e_i[0].record(stream)
    rec.iterate(z, n, params.iters)
    e_i[1].record(stream)
    torch.cuda.synchronize()
    it_ms = e_i[0].elapsed_time(e_i[1]) / params.iters
    # with several points per pixel on frames of 2^17 pixels or more an iteration is two launches:
    # the stand-alone depth denoiser, then the fused kernel without its depth phase
    it_kernel = ("depth_denoise_kernel + iteration_kernel" if w.K_max >= 2 and P >= (1 << 17)
                 else "iteration_kernel")
    it_bytes = iteration_bytes_per_pixel(m, w.K_max) * P
    it_achieved = it_bytes / (it_ms * 1e-3) / 1e9
    it_traffic = profile_figure(f"traffic_{w.name}.md", "srt3d.hip", "iteration_kernel traffic_bytes_per_launch")
    it_valu = valu_per_launch("iteration_kernel", "srt3d.hip", w.name)

    # achievable HBM bandwidth on this device: a plain 1 GiB device-to-device copy (reads and
    # writes 1 GiB each), outside the timed steps
    src_b = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    dst_b = torch.empty_like(src_b)
    dst_b.copy_(src_b)
    e_c = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_c[0].record(stream)
    for _ in range(5):
        dst_b.copy_(src_b)
    e_c[1].record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2.0 * src_b.numel() * 4 * 5 / (e_c[0].elapsed_time(e_c[1]) * 1e-3) / 1e9
    del src_b, dst_b

    # several frames of the workload in flight (outside the timed steps): frames are
    # independent, so a stream of them can run one per HIP stream; each stream does the whole
    # step (sketch + reconstruction) on its own buffers, and the stream's frames/s shows how much
    # of a lone frame's step is launch and latency rather than work
    fif = (frames_in_flight(frame, w, params, irf, table, args.sketch, streams=args.frames_in_flight, rounds=8,
                            ref_out=out) if args.frames_in_flight > 0 else None)

    # the other sketch path on the same frame, for reference (outside the timed steps)
    other = "photon" if args.sketch == "binned" else "binned"
    z2 = torch.empty_like(z)
    n2 = torch.empty_like(n)
    srt.sketch(frame.stamps, frame.offsets, T, m, z=z2, n=n2, table=table, method=other)
    e_o = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_o[0].record(stream)
    for _ in range(3):
        srt.sketch(frame.stamps, frame.offsets, T, m, z=z2, n=n2, table=table, method=other)
    e_o[1].record(stream)
    torch.cuda.synchronize()
    other_ms = e_o[0].elapsed_time(e_o[1]) / 3

    # the same photons as an arrival-order event stream (pixel, stamp) in random order, sketched
    # by srt3d_sketch_events (grouped on the device, then sketched); outside the timed steps
    counts = frame.offsets[1:] - frame.offsets[:-1]
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed)
    order = torch.randperm(N, device=dev, generator=gen)
    ev_pix = torch.repeat_interleave(torch.arange(P, device=dev, dtype=torch.int32), counts)[order].contiguous()
    ev_st = frame.stamps[order].contiguous()
    del order
    ev_ws = srt.events_workspace(N, P, dev)
    srt.sketch_events(ev_pix, ev_st, P, T, m, z=z2, n=n2, table=table, workspace=ev_ws)
    e_v = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e_v[0].record(stream)
    for _ in range(3):
        srt.sketch_events(ev_pix, ev_st, P, T, m, z=z2, n=n2, table=table, workspace=ev_ws)
    e_v[1].record(stream)
    torch.cuda.synchronize()
    ev_ms = e_v[0].elapsed_time(e_v[1]) / 3
    ev_same = bool(torch.equal(n2, n)) and (args.sketch != "binned" or bool(torch.equal(z2, z)))
    ev_alg = 8.0 * N + 8.0 * m * P + 4.0 * P          # events in, sketch + counts out
    del z2, n2, ev_pix, ev_st, ev_ws

    # the pixelwise comparison estimators on the same sketch (outside the timed steps): W = I from
    # four starts, then 20 steps of the precision-weighted fit (eq. 6 with W = Sigma^-1)
    pw = srt.Reconstructor(params, dev)
    starts, wsteps = 4, 20
    weighted = m <= 32 and 2 * m < T
    pw.smle(z, n, irf, frame.irf_origin, starts)
    if weighted:
        pw.weighted_fit(z, n, irf, frame.irf_origin, wsteps)
    e_p = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e_p[0].record(stream)
    pw.smle(z, n, irf, frame.irf_origin, starts)
    e_p[1].record(stream)
    if weighted:
        pw.weighted_fit(z, n, irf, frame.irf_origin, wsteps)
    e_p[2].record(stream)
    torch.cuda.synchronize()
    pixelwise = {"smle_starts": starts, "smle_steps_per_start": w.iters, "smle_ms": e_p[0].elapsed_time(e_p[1]),
                 "weighted_fit_steps": wsteps if weighted else 0,
                 "weighted_fit_ms": e_p[1].elapsed_time(e_p[2]) if weighted else None}
    del pw
    # SRT3D with W_p = Sigma(theta_0)^-1 inside the data step (eq. 8 with a per-pixel W): init,
    # the weights, the iterations and finalize, on the step's sketch (outside the timed steps)
    weighted_srt3d = None
    if weighted:
        wr = srt.Reconstructor(params, dev)

        def wrun(ev=None):
            if ev:
                ev[0].record(stream)
            wr.init(z, n, irf, frame.irf_origin)
            wr.weighted_prepare(n, irf, frame.irf_origin)
            if ev:
                ev[1].record(stream)
            wr.weighted_iterate(z, n, params.iters)
            if ev:
                ev[2].record(stream)
            wr.finalize(n)
            if ev:
                ev[3].record(stream)

        wrun()
        e_w = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        wrun(e_w)
        torch.cuda.synchronize()
        weighted_srt3d = {"iters": params.iters, "weights_bytes": int(wr.wws.numel()),
                          "init_and_weights_ms": e_w[0].elapsed_time(e_w[1]),
                          "iterations_ms": e_w[1].elapsed_time(e_w[2]),
                          "total_ms": e_w[0].elapsed_time(e_w[3])}
        del wr
    res = {
        "metric": METRIC,
        "value": args.steps / wall,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x2-split products, f32 accumulation" if args.sketch == "binned" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "pixels": P, "rows": spec.rows, "cols": spec.cols, "T": T, "m": m,
                   "K_max": w.K_max, "iters": w.iters, "photons": N, "photons_per_pixel": spec.lam,
                   "sbr": spec.sbr, "irf_sigma_bins": spec.sigma},
        "photons_per_s": N * args.steps / wall,
        "sketch_photons_per_s": N / (sk_ms.mean() * 1e-3),
        "sketch_method": args.sketch,
        "other_sketch": {"method": other, "ms": other_ms, "photons_per_s": N / (other_ms * 1e-3)},
        "event_stream_sketch": {"ms": ev_ms, "events_per_s": N / (ev_ms * 1e-3),
                                "hbm_frac": ev_alg / (ev_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "algorithmic_bytes": ev_alg, "same_as_step_sketch": ev_same},
        "pixelwise_estimators": pixelwise,
        "weighted_srt3d": weighted_srt3d,
        "frames_in_flight": fif,
        "launch": ("host launches" if graph is None else
                   "reconstruction replayed from a HIP graph captured in the warm-up; sketch launched from the host"),
        "eager": None if eager_wall is None else {
            "frames_per_s": args.steps / eager_wall, "ms_per_step": eager_wall * 1e3 / args.steps,
            "srt3d_ms_mean": float(np.mean([e[1].elapsed_time(e[2]) for e in eager_evs]))},
        "sketch_ms": {"mean": float(sk_ms.mean()), "p50": float(np.percentile(sk_ms, 50)),
                      "p99": float(np.percentile(sk_ms, 99))},
        "srt3d_ms": {"mean": float(rc_ms.mean()), "p50": float(np.percentile(rc_ms, 50)),
                     "p99": float(np.percentile(rc_ms, 99))},
        "latency_ms": {"p50": float(np.percentile(st_ms, 50)), "p99": float(np.percentile(st_ms, 99))},
        "roofline_sketch": {"bound": "hbm", "kernel": kernel, "achieved": achieved,
                            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                            "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes,
                            "launch_ms": float(sk_ms.mean()), "launches_per_step": 1,
                            "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                            # against its binding limit, VALU issue (counts from the committed
                            # rocprofv3 summary, the time live)
                            "valu_issue_frac": None if valu is None else valu / (sk_ms.mean() * 1e-3) / VALU_PEAK,
                            "valu_wave_insts_per_launch": valu},
        "roofline_iteration": {"bound": "hbm", "kernel": it_kernel, "achieved": it_achieved,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": it_achieved / HBM_PEAK_GBS,
                               "traffic": it_traffic, "algorithmic_bytes_per_launch": it_bytes,
                               "launch_ms": it_ms, "launches_per_step": params.iters,
                               "launch_note": "launch_ms is per iteration (both launches when split)",
                               "copy_gbs": copy_gbs, "frac_of_copy": it_achieved / copy_gbs,
                               "valu_issue_frac": None if it_valu is None else it_valu / (it_ms * 1e-3) / VALU_PEAK,
                               "valu_wave_insts_per_launch": it_valu},
    }
    # the dominant kernel of the step (launch time x launches per step) is the line's roofline
    share = {k: res[k]["launch_ms"] * res[k]["launches_per_step"] for k in ("roofline_sketch", "roofline_iteration")}
    res["roofline"] = dict(res[max(share, key=share.get)])
    res["roofline"]["step_share"] = max(share.values()) / ms_per_step
    # the serving workload's request stream, short (outside the timed steps): p50/p99 latency
    # under Poisson arrivals at 0.5x and 0.9x of the measured single-slot capacity
    if args.serving_requests > 0:
        res["serving"] = serving_measure(args.serving_requests, int(args.budget_gib * (1 << 30)))
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_all_cores(frame, w, params)
        res["cpu_baseline"]["single_core"] = cpu_baseline(frame, z, n, w, params)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
