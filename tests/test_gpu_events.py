"""GPU parity of the event-stream sketch (srt3d_sketch_events: arrival-order (pixel, stamp)
events grouped on the device, then sketched) against the FP64 oracle's per-event online sums,
through the C ABI: shuffled ragged streams over several tiles, events outside the frame,
folded stamps, empty streams, long-exposure chunks, m above 32 (photon pass), and the full
throughput frame as a shuffled stream in the benchmark's configuration."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import sketch as OS
from tests.gpu_common import device, sketch_violations, to_complex

pytestmark = pytest.mark.gpu


def _print_case(**kw):
    print("case events", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _stream(rng, P, T, counts):
    pix = np.repeat(np.arange(P), counts)
    st = rng.integers(0, T, pix.size)
    order = rng.permutation(pix.size)
    return pix[order], st[order]


def _to_dev(a, dev):
    return torch.from_numpy(np.asarray(a, dtype=np.int32)).to(dev)


def _check(pix, st, P, T, m, z, n, label):
    zr, nr = OS.sketch_events(pix, st, P, T, m)
    np.testing.assert_array_equal(n.cpu().numpy(), nr)
    bad, err, tol = sketch_violations(to_complex(z), zr, nr)
    worst = float(np.max(err / np.maximum(tol, 1e-300))) if err.size else 0.0
    print(label, "max |dz|/tol", worst)
    assert not bad.any(), f"{label}: {bad.sum()} entries off, worst err/tol {worst:.3g}"


@pytest.mark.parametrize("T,m", [(4096, 16), (8192, 32), (1024, 4), (4613, 5), (3000, 20), (100, 1)])
def test_shuffled_stream_matches_oracle(T, m):
    dev = device()
    rng = np.random.default_rng(T + 7 * m)
    P = 2000
    counts = rng.integers(0, 400, P)
    counts[::17] = 0
    counts[5] = 3000
    pix, st = _stream(rng, P, T, counts)
    _print_case(test="shuffled", T=T, m=m, N=pix.size)
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m)
    torch.cuda.synchronize()
    _check(pix, st, P, T, m, z, n, f"T={T} m={m}")


def test_same_bits_as_the_csr_binned_pass():
    """With no bin above 255 the grouped stream gives exactly the CSR pass's numbers, whatever
    the order of the events."""
    dev = device()
    rng = np.random.default_rng(3)
    P, T, m = 3000, 4096, 16
    counts = rng.integers(0, 250, P)
    pix, st = _stream(rng, P, T, counts)
    _print_case(test="bits_vs_csr", N=pix.size)
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m)
    order = np.argsort(pix, kind="stable")
    offsets = np.zeros(P + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    zc, nc = srt.sketch(_to_dev(st[order], dev), torch.from_numpy(offsets).to(dev), T, m, method="binned")
    torch.cuda.synchronize()
    assert torch.equal(n, nc)
    assert torch.equal(z, zc)


def test_events_outside_the_frame_and_folded_stamps():
    dev = device()
    T, m, P = 1000, 6, 5
    pix = np.array([0, 7, 2, -1, 2, 4, 4, 5, 0, 2], dtype=np.int64)
    st = np.array([3, 1, 999, 5, -2001, 1000, 7, 9, 2500, 4], dtype=np.int64)
    err = torch.zeros(2, dtype=torch.int32, device=dev)
    _print_case(test="bad_events")
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m, err=err)
    torch.cuda.synchronize()
    _, _, dropped, folded = OS.sketch_event_sums(pix, st, P, T, m)
    assert err.cpu().tolist() == [folded, dropped] == [3, 3]
    _check(pix, st, P, T, m, z, n, "bad events")


def test_events_outside_the_frame_in_a_long_stream():
    """A stream of several chunks (13 counting workgroups), with a share of events whose pixel
    is outside the frame and stamps outside [0, T)."""
    dev = device()
    rng = np.random.default_rng(12)
    P, T, m = 1000, 2048, 8
    pix, st = _stream(rng, P, T, rng.integers(0, 200, P))
    k = pix.size // 20
    pix[:k] = np.where(rng.random(k) < 0.5, -1 - rng.integers(0, 50, k), P + rng.integers(0, 50, k))
    st[k:2 * k] = rng.integers(-3 * T, 4 * T, k)
    err = torch.zeros(2, dtype=torch.int32, device=dev)
    _print_case(test="bad_events_long", N=pix.size)
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m, err=err)
    torch.cuda.synchronize()
    _, _, dropped, folded = OS.sketch_event_sums(pix, st, P, T, m)
    assert dropped == k
    assert err.cpu().tolist() == [folded, dropped]
    _check(pix, st, P, T, m, z, n, "bad events, long stream")


def test_large_frame_with_wide_bucket_tables():
    """2^21 + 1 pixels: 1025 buckets of 2048 pixels, past the small LDS tables of both grouping
    levels; the result is the CSR pass's, bit for bit, and the oracle's."""
    dev = device()
    rng = np.random.default_rng(13)
    P, T, m = 2**21 + 1, 1024, 4
    counts = rng.integers(0, 2, P)
    counts[-1] = 5                      # the one-pixel last bucket
    pix, st = _stream(rng, P, T, counts)
    _print_case(test="large_frame", P=P, N=pix.size)
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m)
    order = np.argsort(pix, kind="stable")
    offsets = np.zeros(P + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    zc, nc = srt.sketch(_to_dev(st[order], dev), torch.from_numpy(offsets).to(dev), T, m, method="binned")
    torch.cuda.synchronize()
    assert torch.equal(n, nc)
    assert torch.equal(z, zc)
    _check(pix, st, P, T, m, z, n, "large frame")


def test_empty_stream_and_single_events():
    dev = device()
    for pix, st, P in (([], [], 7), ([3], [17], 5), ([0, 0, 0], [1, 2, 3], 1)):
        _print_case(test="small", N=len(pix), P=P)
        z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, 128, 4)
        torch.cuda.synchronize()
        _check(np.asarray(pix, np.int64), np.asarray(st, np.int64), P, 128, 4, z, n, "small")


def test_long_exposure_chunks_of_the_stream():
    dev = device()
    rng = np.random.default_rng(21)
    P, T, m = 500, 4096, 32
    pix, st = _stream(rng, P, T, rng.integers(0, 1500, P))
    acc = torch.zeros((P, m, 2), dtype=torch.float64, device=dev)
    nacc = torch.zeros(P, dtype=torch.int64, device=dev)
    cut = pix.size // 3
    _print_case(test="long_exposure", N=pix.size)
    for a, b in ((0, cut), (cut, pix.size)):
        z, n = srt.sketch_events(_to_dev(pix[a:b], dev), _to_dev(st[a:b], dev), P, T, m, acc=acc, nacc=nacc)
    torch.cuda.synchronize()
    _check(pix, st, P, T, m, z, n, "chunked")
    S, nr, _, _ = OS.sketch_event_sums(pix, st, P, T, m)
    np.testing.assert_array_equal(nacc.cpu().numpy(), nr)
    accc = acc.cpu().numpy()
    ratio = np.abs(accc[..., 0] + 1j * accc[..., 1] - S) / (1e-5 * np.sqrt(np.maximum(nr, 1))[:, None])
    assert np.max(ratio) <= 1.0, np.max(ratio)


def test_more_than_32_harmonics_use_the_photon_pass():
    dev = device()
    rng = np.random.default_rng(8)
    P, T, m = 300, 2048, 48
    pix, st = _stream(rng, P, T, rng.integers(0, 600, P))
    _print_case(test="m48", N=pix.size)
    z, n = srt.sketch_events(_to_dev(pix, dev), _to_dev(st, dev), P, T, m)
    torch.cuda.synchronize()
    _check(pix, st, P, T, m, z, n, "m=48")


def test_full_frame_as_a_shuffled_stream():
    """The 256x256, T = 4096, m = 16 frame's photons in random arrival order: 2000 sampled pixels
    against the oracle one by one, every pixel bitwise against the CSR binned pass."""
    dev = device()
    w = synth.preset("throughput")
    f = synth.make_frame(w.frame, device=dev)
    P, T, m = w.frame.P, w.frame.T, w.m
    counts = f.offsets[1:] - f.offsets[:-1]
    pix = torch.repeat_interleave(torch.arange(P, device=dev, dtype=torch.int32), counts)
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    order = torch.randperm(pix.numel(), device=dev, generator=g)
    pix_s, st_s = pix[order].contiguous(), f.stamps[order].contiguous()
    _print_case(test="full_frame", N=pix.numel())
    z, n = srt.sketch_events(pix_s, st_s, P, T, m)
    zc, nc = srt.sketch(f.stamps, f.offsets, T, m, method="binned")
    torch.cuda.synchronize()
    assert torch.equal(n, nc)
    assert torch.equal(z, zc)
    rng = np.random.default_rng(2)
    sel = np.sort(rng.choice(P, 2000, replace=False))
    st_np, off_np = f.stamps.cpu().numpy(), f.offsets.cpu().numpy()
    zr, nr = OS.sketch(st_np, off_np, T, m, pixels=sel)
    np.testing.assert_array_equal(n.cpu().numpy()[sel], nr)
    bad, err, tol = sketch_violations(to_complex(z)[sel], zr, nr)
    assert not bad.any()
