"""srt3d_reconstruct_noalloc (scratch in the library's static device array) against
srt3d_reconstruct (scratch in a caller workspace), through the C ABI: two calls in a row on one
device, the second on a smaller frame, so the second finds the first one's scratch contents."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from tests.gpu_common import device

pytestmark = pytest.mark.gpu


def _frame(spec, m, K, dev, **pk):
    f = synth.make_frame(spec, device=dev)
    z, n = srt.sketch(f.stamps, f.offsets, spec.T, m)
    params = srt.Params.default(spec.rows, spec.cols, spec.T, m, K, **pk)
    return z, n, torch.from_numpy(f.irf).to(dev), f.irf_origin, params


def test_noalloc_equals_workspace_entry_point_on_two_calls():
    dev = device()
    cases = [
        # 48x40 px, T = 8192, three surfaces, m = 32: the largest scratch of the two
        ("layered", _frame(synth.FrameSpec(48, 40, 8192, 8.0, 4000.0, 0.5, 3, seed=5), 32, 3, dev, r_min=100.0)),
        # 32x32 px, T = 1024, m = 4: smaller frame and scratch, after the first call
        ("tiny", _frame(synth.preset("tiny").frame, 4, 1, dev)),
    ]
    for name, (z, n, irf, origin, params) in cases:
        print("case", name, "P", params.P, "T", params.T, "m", params.m, "K", params.K_max, flush=True)
        a = srt.Reconstructor(params, dev).reconstruct(z, n, irf, origin, no_alloc=True)
        b = srt.Reconstructor(params, dev).reconstruct(z, n, irf, origin)
        torch.cuda.synchronize()
        for k in a:
            assert torch.equal(a[k], b[k]), (name, k)
        act = a["active"].cpu().numpy().astype(bool)
        assert act.any(1).mean() > 0.9, name              # a real reconstruction, not an empty one
        assert np.isfinite(a["depth"].cpu().numpy()).all()
