#!/usr/bin/env python3
"""Throughput of the SRT3D hot path on one MI355X.

One step = the photon sketch of a 256x256 frame (T = 4096 bins, ~1000 photons per pixel,
SBR = 1, m = 16 harmonics; ~6.6e7 int32 stamps resident in HBM) followed by the SRT3D
reconstruction of that sketch (initialisation, 50 iterations of data step + depth denoiser +
intensity denoiser, background and output).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload throughput] [--no-cpu-baseline]
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
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "sketch_photons_throughput_traffic.md")
SKETCH_SRC = os.path.join(ROOT, "paper_2203_00952_amd", "csrc", "sketch.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="throughput")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (scale reference for HBM counters)")
    return ap.parse_args()


def sketch_traffic(launch_bytes: float):
    """HBM bytes per sketch launch from the committed counter summary, if it describes the
    current kernel source (else None)."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    text = open(TRAFFIC_SUMMARY).read()
    sha = hashlib.sha256(open(SKETCH_SRC, "rb").read()).hexdigest()
    m_sha = re.search(r"sketch\.hip sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


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
    S = 2048
    sel = np.sort(rng.choice(spec.P, S, replace=False))
    it_sample = 5
    op = O.Params(spec.T, w.m, w.K_max, iters=params.iters)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not "
                                   "part of this build (pixels shard with no communication)"}))
        sys.exit(2)

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
    params = srt.Params.default(spec.rows, spec.cols, T, m, w.K_max, iters=w.iters)
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

    def step(ev=None):
        if ev:
            ev[0].record(stream)
        srt.sketch(frame.stamps, frame.offsets, T, m, z=z, n=n, table=table)
        if ev:
            ev[1].record(stream)
        rec.reconstruct(z, n, irf, frame.irf_origin, out=out)
        if ev:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    sk_ms = np.array([e[0].elapsed_time(e[1]) for e in evs])
    rc_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    st_ms = np.array([e[0].elapsed_time(e[2]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps

    # algorithmic bytes of one sketch launch: stamps + offsets in, sketch + counts out
    alg_bytes = 4.0 * N + 8.0 * (P + 1) + 8.0 * m * P + 4.0 * P
    achieved = alg_bytes / (sk_ms.mean() * 1e-3) / 1e9
    traffic = sketch_traffic(alg_bytes)
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "pixels": P, "rows": spec.rows, "cols": spec.cols, "T": T, "m": m,
                   "K_max": w.K_max, "iters": w.iters, "photons": N, "photons_per_pixel": spec.lam,
                   "sbr": spec.sbr, "irf_sigma_bins": spec.sigma},
        "photons_per_s": N * args.steps / wall,
        "sketch_photons_per_s": N / (sk_ms.mean() * 1e-3),
        "sketch_ms": {"mean": float(sk_ms.mean()), "p50": float(np.percentile(sk_ms, 50)),
                      "p99": float(np.percentile(sk_ms, 99))},
        "srt3d_ms": {"mean": float(rc_ms.mean()), "p50": float(np.percentile(rc_ms, 50)),
                     "p99": float(np.percentile(rc_ms, 99))},
        "latency_ms": {"p50": float(np.percentile(st_ms, 50)), "p99": float(np.percentile(st_ms, 99))},
        "roofline": {"bound": "hbm", "kernel": "sketch_photons_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": alg_bytes},
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(frame, z, n, w, params)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
