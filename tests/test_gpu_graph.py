"""srt3d_reconstruct captured into a HIP graph (through torch's CUDAGraph wrapper of stream
capture) and replayed: every replay must give the eager call's outputs and final state bit for
bit, with other eager GPU work and host synchronisations between the replays.  Covers the
one-point path, merge/birth stages (their fill kernels) and the split depth-denoiser launches
of larger frames with several points per pixel."""
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from synth.frames import FrameSpec
from tests.gpu_common import device

pytestmark = pytest.mark.gpu

CASES = {
    # name: (frame, m, K_max, extra parameters)
    "one_point": (FrameSpec(64, 96, 4096, 8.0, 300.0, 1.0, 1, seed=31), 16, 1, {}),
    "births": (FrameSpec(32, 32, 153, 2.0, 200.0, 2.0, 2, seed=11), 10, 2, {"birth_every": 10, "r_min": 5.0}),
    "split_depth": (FrameSpec(512, 256, 2048, 6.0, 60.0, 1.0, 3, seed=7), 8, 3, {"r_min": 5.0}),
}


def _outputs(P, K, dev):
    return dict(depth=torch.empty((P, K), dtype=torch.float32, device=dev),
                intensity=torch.empty((P, K), dtype=torch.float32, device=dev),
                active=torch.empty((P, K), dtype=torch.uint8, device=dev),
                bg=torch.empty(P, dtype=torch.float32, device=dev))


@pytest.mark.parametrize("name", list(CASES))
def test_reconstruct_graph_replays_equal_eager(name):
    dev = device()
    spec, m, K, extra = CASES[name]
    print("case", name, spec.rows, spec.cols, "m", m, "K", K, flush=True)
    f = synth.make_frame(spec, device=dev)
    z, n = srt.sketch(f.stamps, f.offsets, spec.T, m, method="auto")
    irf = torch.from_numpy(f.irf).to(dev)
    p = srt.Params.default(spec.rows, spec.cols, spec.T, m, K, iters=50, **extra)
    rec = srt.Reconstructor(p, dev)
    ref = rec.reconstruct(z, n, irf, f.irf_origin)
    ref_state = [t.clone() for t in rec.state()]
    torch.cuda.synchronize()

    out = _outputs(p.P, K, dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        rec.reconstruct(z, n, irf, f.irf_origin, out=out)
    torch.cuda.synchronize()

    # other eager work between the replays: a second reconstruction of another frame
    spec2 = FrameSpec(48, 40, 1024, 4.0, 100.0, 2.0, 1, seed=32)
    f2 = synth.make_frame(spec2, device=dev)
    z2, n2 = srt.sketch(f2.stamps, f2.offsets, spec2.T, 8)
    rec2 = srt.Reconstructor(srt.Params.default(spec2.rows, spec2.cols, spec2.T, 8, 1, iters=20), dev)
    irf2 = torch.from_numpy(f2.irf).to(dev)
    for r in range(3):
        rec2.reconstruct(z2, n2, irf2, f2.irf_origin)
        for t in out.values():
            t.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (name, r, k)
        for a, b in zip(rec.state(), ref_state):
            assert torch.equal(a, b), (name, r)
    assert int(out["active"].sum()) > 0
