"""Serving on the GPU: each request's result is the same alone and in a mix of overlapping
requests of different sizes, and the same as a direct library call."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from paper_2203_00952_amd.serve import Request, serve
from tests.gpu_common import device

pytestmark = pytest.mark.gpu

# (side, photons/px, m): the serving workload's sizes 32^2..512^2 among smaller and odd ones
MIX = [(32, 500.0, 8), (256, 400.0, 16), (48, 200.0, 12), (128, 300.0, 20), (512, 60.0, 32), (96, 800.0, 10),
       (16, 50.0, 4), (80, 1000.0, 24), (256, 1500.0, 8)]


def _requests(dev, arrivals):
    reqs = []
    for i, ((side, lam, m), t) in enumerate(zip(MIX, arrivals)):
        spec = synth.FrameSpec(side, side, 2048, 8.0, lam, 1.0, 1, seed=100 + i)
        f = synth.make_frame(spec, device=dev)
        params = srt.Params.default(side, side, 2048, m, 1, iters=20)
        reqs.append(Request(i, f.stamps, f.offsets, torch.from_numpy(f.irf).to(dev), f.irf_origin, params, t))
    return reqs


def test_results_identical_alone_and_in_the_mix():
    dev = device()
    print("case serve_alone_vs_mix", flush=True)
    reqs = _requests(dev, [0.0] * len(MIX))
    alone = {}
    for r in reqs:
        _, res, _ = serve([r], slots=1)
        alone[r.rid] = res[r.rid]
    recs, mixed, peak = serve(reqs, slots=4)
    assert len(recs) == len(MIX) and peak > 0
    for rid, out in alone.items():
        for key in ("depth", "intensity", "active", "bg"):
            assert torch.equal(out[key], mixed[rid][key]), (rid, key)
    # staggered arrivals and a tight budget (admission waits for memory) give the same results
    budget = max(r.working_bytes() for r in reqs) * 2
    reqs2 = _requests(dev, list(np.arange(len(MIX)) * 2e-4))
    recs2, mixed2, peak2 = serve(reqs2, slots=3, budget_bytes=budget)
    assert peak2 <= budget
    for rid, out in alone.items():
        for key in ("depth", "intensity", "active", "bg"):
            assert torch.equal(out[key], mixed2[rid][key]), (rid, key)
    assert all(r.latency >= 0 for r in recs2)


def test_served_result_equals_direct_call():
    dev = device()
    print("case serve_vs_direct", flush=True)
    r = _requests(dev, [0.0])[0]
    _, res, _ = serve([r], slots=2)
    z, n = srt.sketch(r.stamps, r.offsets, r.params.T, r.params.m, method=r.sketch)
    out = srt.Reconstructor(r.params, dev).reconstruct(z, n, r.irf, r.irf_origin)
    torch.cuda.synchronize()
    for key in ("depth", "intensity", "active", "bg"):
        assert torch.equal(out[key], res[0][key]), key
