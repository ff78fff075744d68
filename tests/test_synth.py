"""The seeded input generator: structure and statistics of the frames it draws."""
import numpy as np
import pytest
import torch

import synth
from synth.frames import FrameSpec, binned_gaussian_irf, hist_as_uint


def test_frame_structure_and_statistics():
    spec = FrameSpec(48, 40, 2048, 6.0, 200.0, 1.0, 1, seed=11)
    f = synth.make_frame(spec)
    P = spec.P
    assert f.stamps.dtype == torch.int32 and f.offsets.dtype == torch.int64
    assert f.offsets.numel() == P + 1 and int(f.offsets[-1]) == f.stamps.numel()
    assert int(f.stamps.min()) >= 0 and int(f.stamps.max()) < spec.T
    n = f.n.numpy()
    assert abs(n.mean() - 200.0) < 3.0
    sig = f.counts[:, :-1].sum().item()
    bg = f.counts[:, -1].sum().item()
    assert abs(sig / bg - 1.0) < 0.03
    # signal stamps cluster around the depth of their pixel, interleaved with the background
    p = int(np.argmax(n))
    x = f.stamps[f.offsets[p]:f.offsets[p + 1]].numpy()
    d = (x - f.scene.depth[p, 0] + spec.T / 2) % spec.T - spec.T / 2
    near = np.abs(d) <= 6 * spec.sigma
    nsig, nbg = int(f.counts[p, 0]), int(f.counts[p, 1])
    assert nsig <= near.sum() <= nsig + nbg * (12 * spec.sigma + 1) / spec.T + 5 * np.sqrt(nbg) + 1
    assert abs(np.median(d[near])) < 3 and np.std(d[near]) < 12
    first = near[:nsig].mean()
    assert 0.2 < first < 0.9          # grouped by source would give 1.0


def test_reproducible_and_seeded():
    spec = FrameSpec(16, 16, 1024, 5.0, 30.0, 1.0, 1, seed=5)
    a, b = synth.make_frame(spec), synth.make_frame(spec)
    assert torch.equal(a.stamps, b.stamps) and torch.equal(a.offsets, b.offsets)
    c = synth.make_frame(FrameSpec(16, 16, 1024, 5.0, 30.0, 1.0, 1, seed=6))
    assert not torch.equal(a.offsets, c.offsets)


def test_layered_scene():
    spec = FrameSpec(64, 64, 8192, 8.0, 100.0, 0.5, 3, seed=5)
    sc = synth.make_scene(spec)
    k = (sc.weight > 0).sum(1)
    assert k.max() == 3 and k.min() >= 1
    np.testing.assert_allclose(sc.weight.sum(1), 1.0)
    both = (sc.weight[:, 0] > 0) & (sc.weight[:, 2] > 0)
    assert np.min(sc.depth[both, 2] - sc.depth[both, 0]) > 8192 / 32


def test_camouflage_scene():
    """Two surfaces on most pixels: a netting in front, the nearest object or the wall behind."""
    w = synth.preset("camouflage")
    sc = synth.make_scene(w.frame)
    k = (sc.weight > 0).sum(1)
    assert set(np.unique(k)) == {1, 2} and np.mean(k == 2) > 0.9
    np.testing.assert_allclose(sc.weight.sum(1), 1.0)
    both = k == 2
    assert np.all(sc.depth[both, 1] > sc.depth[both, 0])
    assert w.frame.T == 153 and w.m == 10 and w.K_max == 2


def test_irf_and_histogram():
    h, o = binned_gaussian_irf(8.0)
    assert o == 48 and h.size == 97
    assert h.sum() == pytest.approx(1.0, abs=1e-8)
    np.testing.assert_allclose(h, h[::-1], atol=1e-15)
    spec = FrameSpec(8, 8, 512, 4.0, 50.0, 1.0, 1, seed=2)
    f = synth.make_frame(spec)
    H = hist_as_uint(synth.histogram(f.stamps, f.offsets, spec.T))
    assert H.shape == (64, 512)
    np.testing.assert_array_equal(H.sum(1), f.n.numpy())


def test_request_stream():
    reqs = synth.request_stream(4, 50, rate_hz=100.0)
    assert len(reqs) == 50
    assert all(b.arrival_s > a.arrival_s for a, b in zip(reqs, reqs[1:]))
    assert {r.frame.rows for r in reqs} <= {32, 128, 256, 512}
    assert all(8 <= r.m <= 32 and 10 <= r.frame.lam <= 2000 for r in reqs)
