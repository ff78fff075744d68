"""Degenerate and ragged frame shapes, end to end through the C ABI against the FP64 oracle (its
own sketch of the same stamps, then its reconstruction, 50 iterations): a single pixel, a
single row, a single column, tiles ragged in both directions with three points per pixel, one
harmonic, and a frame with no photons at all."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import sketch as OS
from oracle import srt3d as O
from synth.frames import FrameSpec
from tests.gpu_common import device
from tests.test_gpu_srt3d import pixel_pass

pytestmark = pytest.mark.gpu

CASES = {
    # name: (frame, m, K_max)
    "1x1": (FrameSpec(1, 1, 1024, 5.0, 200.0, 2.0, 1, seed=41), 4, 1),
    "1x37": (FrameSpec(1, 37, 1024, 5.0, 200.0, 2.0, 1, seed=42), 6, 1),
    "37x1_K2": (FrameSpec(37, 1, 2048, 6.0, 200.0, 2.0, 2, seed=43), 8, 2),
    "9x17_K3": (FrameSpec(9, 17, 512, 4.0, 150.0, 1.0, 3, seed=44), 5, 3),
    "m1": (FrameSpec(16, 24, 1024, 5.0, 300.0, 5.0, 1, seed=45), 1, 1),
}


def _check(out, r, T):
    ok = pixel_pass(out["depth"].cpu().numpy(), out["active"].cpu().numpy(), r["depth"], r["active"], T)
    bg_g = out["bg"].cpu().numpy()
    bg_ok = np.abs(bg_g - r["bg"]) <= 1e-3 * np.abs(r["bg"]) + 1e-6
    return ok, bg_ok


@pytest.mark.parametrize("name", list(CASES))
def test_shape_end_to_end(name):
    dev = device()
    spec, m, K = CASES[name]
    f = synth.make_frame(spec, device=dev)
    print("case", name, spec.rows, spec.cols, "m", m, "K", K, "photons", f.stamps.numel(), flush=True)
    z, n = srt.sketch(f.stamps, f.offsets, spec.T, m, method="auto")
    p = srt.Params.default(spec.rows, spec.cols, spec.T, m, K, iters=50, r_min=1.0)
    out = srt.Reconstructor(p, dev).reconstruct(z, n, torch.from_numpy(f.irf).to(dev), f.irf_origin)
    torch.cuda.synchronize()
    z_ref, n_ref = OS.sketch(f.stamps.cpu().numpy(), f.offsets.cpu().numpy(), spec.T, m)
    np.testing.assert_array_equal(n.cpu().numpy(), n_ref)
    op = O.Params(spec.T, m, K, iters=50, r_min=1.0)
    r = O.reconstruct(z_ref, n_ref, f.irf, f.irf_origin, spec.rows, spec.cols, op)
    ok, bg_ok = _check(out, r, spec.T)
    print(name, "pixels within 1 bin", ok.mean(), "active points", int(r["active"].sum()),
          "background within 1e-3", bg_ok.mean())
    assert r["active"].any()
    assert ok.mean() >= 0.999 and bg_ok.mean() >= 0.999


def test_frame_without_photons():
    """No stamps at all: no point survives, the background is zero and n is zero everywhere."""
    dev = device()
    spec = FrameSpec(5, 7, 1024, 5.0, 200.0, 2.0, 1, seed=46)
    f = synth.make_frame(spec)                        # for the IRF only
    P, m = spec.P, 4
    stamps = torch.zeros(0, dtype=torch.int32, device=dev)
    offsets = torch.zeros(P + 1, dtype=torch.int64, device=dev)
    print("case empty frame", spec.rows, spec.cols, flush=True)
    z, n = srt.sketch(stamps, offsets, spec.T, m)
    p = srt.Params.default(spec.rows, spec.cols, spec.T, m, 1, iters=50, r_min=1.0)
    out = srt.Reconstructor(p, dev).reconstruct(z, n, torch.from_numpy(f.irf).to(dev), f.irf_origin)
    torch.cuda.synchronize()
    assert int(n.abs().sum()) == 0 and float(z.abs().sum()) == 0.0
    assert int(out["active"].sum()) == 0
    assert float(out["bg"].abs().sum()) == 0.0
    z_ref, n_ref = OS.sketch(np.zeros(0, np.int32), np.zeros(P + 1, np.int64), spec.T, m)
    r = O.reconstruct(z_ref, n_ref, f.irf, f.irf_origin, spec.rows, spec.cols, O.Params(spec.T, m, 1, iters=50))
    assert not r["active"].any() and not np.abs(r["bg"]).any()
