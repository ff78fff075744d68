"""GPU parity of the binned photon sketch (per-pixel histogram on the FP16 matrix cores,
srt3d_sketch_binned) against the FP64 oracle, through the C ABI: ragged pixels over several
tiles and a ragged tail of histogram rows, 8-bit bin overflow, folding and error counts, the
long-exposure accumulators, and the full-size frame in the benchmark's launch configuration."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import sketch as OS
from tests.gpu_common import csr, device, sketch_violations, to_complex

pytestmark = pytest.mark.gpu


def _print_case(**kw):
    print("case binned", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _check(stamps_np, offsets_np, T, m, z, n, label):
    zr, nr = OS.sketch(stamps_np, offsets_np, T, m)
    np.testing.assert_array_equal(n.cpu().numpy(), nr)
    bad, err, tol = sketch_violations(to_complex(z), zr, nr)
    worst = float(np.max(err / np.maximum(tol, 1e-300))) if err.size else 0.0
    print(label, "max |dz|/tol", worst)
    assert not bad.any(), f"{label}: {bad.sum()} entries off, worst err/tol {worst:.3g}"


@pytest.mark.parametrize("T,m", [(4096, 16), (8192, 32), (1024, 4), (2048, 8), (4613, 5), (3000, 20),
                                 (8192, 17), (64, 32), (100, 1), (7000, 32)])
def test_ragged_pixels_match_oracle(T, m):
    dev = device()
    rng = np.random.default_rng(T * 31 + m)
    counts = rng.integers(0, 600, 700)
    counts[::13] = 0
    counts[3] = 5000
    pixels = [rng.integers(0, T, c) for c in counts]
    st, off, st_np, off_np = csr(pixels, dev)
    _print_case(test="ragged", T=T, m=m)
    z, n = srt.sketch(st, off, T, m, method="binned")
    torch.cuda.synchronize()
    _check(st_np, off_np, T, m, z, n, f"T={T} m={m}")


def test_peaked_pixels_like_the_frames():
    """Narrow returns (sigma = 1 bin) at high counts put many photons in few bins."""
    dev = device()
    rng = np.random.default_rng(4)
    T, m = 4096, 16
    pixels = []
    for c in rng.integers(100, 3000, 300):
        t0 = rng.integers(0, T)
        pixels.append(np.mod(np.rint(t0 + rng.normal(0, 1.0, c)).astype(np.int64), T))
    st, off, st_np, off_np = csr(pixels, dev)
    _print_case(test="peaked")
    z, n = srt.sketch(st, off, T, m, method="binned")
    torch.cuda.synchronize()
    _check(st_np, off_np, T, m, z, n, "peaked")


def test_bin_overflow_is_recomputed():
    """Bins with 255, 256 and thousands of photons, in each byte of a 32-bit word (the carry out
    of the top byte is lost, out of the others it lands in the neighbour).  The photon pass runs
    the same pixels: 70000 equal stamps and 3e5 random ones test its two-level FP32 sums."""
    dev = device()
    T, m = 4096, 16
    pixels = [np.full(255, 17), np.full(256, 17), np.full(256, 19), np.full(300, 16), np.full(1000, 18),
              np.concatenate([np.full(700, 4095), np.arange(T)]), np.full(70000, 3),
              np.concatenate([np.full(254, 5), np.full(254, 6), np.full(254, 7)]), np.zeros(0, np.int64),
              np.full(511, 0), np.random.default_rng(0).integers(0, T, 300000)]
    st, off, st_np, off_np = csr(pixels, dev)
    for method in ("binned", "photon"):
        _print_case(test="overflow", method=method)
        z, n = srt.sketch(st, off, T, m, method=method)
        torch.cuda.synchronize()
        _check(st_np, off_np, T, m, z, n, f"overflow {method}")


def test_single_pixel_and_empty_frame():
    dev = device()
    for pixels in ([[5]], [[]], [[], [], []], [list(range(100))]):
        st, off, st_np, off_np = csr(pixels, dev)
        _print_case(test="single", P=len(pixels))
        z, n = srt.sketch(st, off, 128, 4, method="binned")
        torch.cuda.synchronize()
        _check(st_np, off_np, 128, 4, z, n, "single")


def test_out_of_range_stamps_and_bad_offsets_are_counted():
    dev = device()
    T, m = 1000, 6
    stamps = np.array([3, -1, 1000, 2500, 7, 999, -2001], dtype=np.int64)
    offsets = np.array([0, 4, 7, 5, 7], dtype=np.int64)          # pixel 2 decreases -> empty
    err = torch.zeros(2, dtype=torch.int32, device=dev)
    _print_case(test="errors")
    z, n = srt.sketch(torch.from_numpy(stamps.astype(np.int32)).to(dev), torch.from_numpy(offsets).to(dev), T, m,
                      err=err, method="binned")
    torch.cuda.synchronize()
    assert err.cpu().tolist() == [5, 1]     # -2001 is read by pixels 1 and 3
    assert n.cpu().tolist() == [4, 3, 0, 2]
    zc = to_complex(z)
    for p, sl in enumerate([slice(0, 4), slice(4, 7), slice(0, 0), slice(5, 7)]):
        zr, _ = OS.sketch(stamps[sl], np.array([0, sl.stop - sl.start]), T, m)
        bad, _, _ = sketch_violations(zc[p:p + 1], zr, np.array([sl.stop - sl.start]))
        assert not bad.any()
    err.zero_()
    offsets = torch.tensor([0, 2, 50], dtype=torch.int64, device=dev)
    z, n = srt.sketch(torch.tensor([1, 2, 3], dtype=torch.int32, device=dev), offsets, T, m, err=err,
                      method="binned")
    torch.cuda.synchronize()
    assert n.cpu().tolist() == [2, 1] and err.cpu().tolist() == [0, 1]


def test_long_exposure_chunks_equal_whole():
    dev = device()
    rng = np.random.default_rng(19)
    T, m = 4096, 32
    counts = rng.integers(0, 2000, 300)
    pixels = [rng.integers(0, T, c) for c in counts]
    cut = [rng.integers(0, c + 1) for c in counts]
    acc = torch.zeros((300, m, 2), dtype=torch.float64, device=dev)
    nacc = torch.zeros(300, dtype=torch.int64, device=dev)
    _print_case(test="long_exposure")
    for part in ([p[:c] for p, c in zip(pixels, cut)], [p[c:] for p, c in zip(pixels, cut)]):
        st, off, _, _ = csr(part, dev)
        z, n = srt.sketch(st, off, T, m, acc=acc, nacc=nacc, method="binned")
    torch.cuda.synchronize()
    _, _, st_np, off_np = csr(pixels, dev)
    _check(st_np, off_np, T, m, z, n, "chunked")
    S, nr = OS.sketch_sums(st_np, off_np, T, m)
    np.testing.assert_array_equal(nacc.cpu().numpy(), nr)
    accc = acc.cpu().numpy()
    ratio = np.abs(accc[..., 0] + 1j * accc[..., 1] - S) / (1e-5 * np.sqrt(np.maximum(nr, 1))[:, None])
    assert np.max(ratio) <= 1.0, np.max(ratio)


def test_rejects_more_than_32_harmonics():
    dev = device()
    st, off, _, _ = csr([[1, 2]], dev)
    with pytest.raises(ValueError):
        srt.sketch(st, off, 4096, 33, method="binned")


@pytest.mark.parametrize("preset", ["throughput", "throughput_sbr10"])
def test_full_frame_sampled_pixels(preset):
    """Full 256x256, T=4096, m=16 frame in the benchmark's launch configuration; 2000 sampled
    pixels checked against the oracle one by one, and every pixel against the photon pass."""
    dev = device()
    w = synth.preset(preset)
    f = synth.make_frame(w.frame, device=dev)
    _print_case(test=preset, N=f.stamps.numel())
    z, n = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m, method="binned")
    zp, np_ = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m, method="photon")
    torch.cuda.synchronize()
    assert torch.equal(n, np_)
    rng = np.random.default_rng(2)
    sel = np.sort(rng.choice(w.frame.P, 2000, replace=False))
    st_np, off_np = f.stamps.cpu().numpy(), f.offsets.cpu().numpy()
    zr, nr = OS.sketch(st_np, off_np, w.frame.T, w.m, pixels=sel)
    np.testing.assert_array_equal(n.cpu().numpy()[sel], nr)
    bad, err, tol = sketch_violations(to_complex(z)[sel], zr, nr)
    print("max |dz| / tol =", float(np.max(err / tol)))
    assert not bad.any()
    # every pixel: the two GPU paths agree to twice the oracle rule
    nn = n.cpu().numpy()
    floor = 1.0 / np.sqrt(np.maximum(nn, 1))[:, None]
    zb, zpp = to_complex(z), to_complex(zp)
    d = np.abs(zb - zpp) / (2e-5 * np.maximum(np.abs(zpp), floor))
    print("binned vs photon, max |dz| / (2 tol) =", float(d.max()))
    assert d.max() <= 1.0


def test_auto_route_takes_the_faster_pass_bit_for_bit():
    """method "auto": the photon pass's bits below 0.04 T photons per pixel, the binned pass's
    bits above."""
    dev = device()
    rng = np.random.default_rng(17)
    T, m, P = 4096, 16, 700
    for lam, expect in ((20, "photon"), (400, "binned")):
        counts = rng.poisson(lam, P)
        stamps, offsets, _, _ = csr([rng.integers(0, T, c) for c in counts], dev)
        _print_case(test="auto_route", lam=lam)
        assert srt.sketch_route(stamps.numel(), P, T, m) == expect
        za, na = srt.sketch(stamps, offsets, T, m, method="auto")
        ze, ne = srt.sketch(stamps, offsets, T, m, method=expect)
        torch.cuda.synchronize()
        assert torch.equal(za, ze) and torch.equal(na, ne)
