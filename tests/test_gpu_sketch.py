"""GPU parity of the photon sketch (eq. 3) and the histogram sketch (eq. 2-3) against the
FP64 oracle, through the C ABI."""
import os

import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import sketch as OS
from tests.gpu_common import csr, device, sketch_violations, to_complex

pytestmark = pytest.mark.gpu


def _print_case(**kw):
    print("case", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def test_phase_table_is_rounded_fp64():
    dev = device()
    for T in (1024, 4613, 8192, 3):
        _print_case(test="phase_table", T=T)
        tab = srt.phase_table(T, dev).cpu().numpy()
        k = np.arange(T)
        ref = np.stack([np.cos(2 * np.pi * k / T), np.sin(2 * np.pi * k / T)], 1)
        quarter = (4 * k) % T == 0           # exact values at multiples of pi/2 (FP64 cos/sin of a
        ref[quarter] = np.rint(ref[quarter])  # rounded 2 pi k / T leave ~1e-16 there)
        ref = ref.astype(np.float32)
        differ = tab != ref                                   # +0 and -0 compare equal
        ulps = np.abs(tab.view(np.int32).astype(np.int64) - ref.view(np.int32).astype(np.int64))
        assert np.all(ulps[differ] <= 1)                      # never more than 1 ulp
        assert np.count_nonzero(differ) <= max(1, T // 10000)  # and essentially always exact


def test_phase_indices_bit_exact():
    dev = device()
    rng = np.random.default_rng(0)
    for T, m in ((1024, 4), (4096, 16), (4613, 10), (8192, 32), (7, 3)):
        _print_case(test="phase_indices", T=T, m=m)
        x = rng.integers(-2 * T, 3 * T, 20000)
        k = srt.phase_indices(torch.from_numpy(x.astype(np.int32)).to(dev), T, m).cpu().numpy()
        np.testing.assert_array_equal(k, OS.phase_indices(x, T, m))


@pytest.mark.parametrize("T,m", [(4096, 16), (4613, 5), (1024, 33), (8192, 64), (2048, 1), (7, 3), (3000, 31)])
def test_photon_pass_phases_bit_exact(T, m):
    """The phases the photon pass itself reads from its table (eq. 3's exact integer part):
    every odd harmonic's index equals (l x) mod T after folding; even harmonics are formed as
    the product of the l-1 and l = 1 entries and read nothing.  The pass that writes them is
    the 4-lane production kernel, so its z and n must equal srt3d_sketch_lanes' bit for bit."""
    dev = device()
    rng = np.random.default_rng(T * 17 + m)
    counts = rng.integers(0, 120, 301)
    counts[::13] = 0
    counts[7] = 2000
    skip = 37                                      # leading photons that belong to no pixel
    N = skip + int(counts.sum()) + 11              # and a trailing run
    x = rng.integers(0, T, N)
    wild = rng.random(N) < 0.05                    # out-of-range stamps, folded into [0, T)
    x[wild] = rng.integers(-3 * T, 4 * T, int(wild.sum()))
    offsets = np.concatenate([[0], np.cumsum(counts)]) + skip
    covered = np.zeros(N, bool)
    covered[skip:skip + int(counts.sum())] = True
    st = torch.from_numpy(x.astype(np.int32)).to(dev)
    off = torch.from_numpy(offsets.astype(np.int64)).to(dev)
    _print_case(test="pass_phases", T=T, m=m, N=N)
    z, n, k = srt.sketch_phases(st, off, T, m)
    z4, n4 = srt.sketch(st, off, T, m, lanes=4)
    torch.cuda.synchronize()
    k = k.cpu().numpy()
    ref = OS.phase_indices(x, T, m)
    odd = np.arange(m) % 2 == 0                    # rows l-1 of odd l
    np.testing.assert_array_equal(k[np.ix_(odd, covered)], ref[np.ix_(odd, covered)])
    assert np.all(k[~odd] == -1) and np.all(k[:, ~covered] == -1)
    for l in range(2, m + 1, 2):                   # phase of the product = sum of the phases
        np.testing.assert_array_equal((k[l - 2, covered] + k[0, covered]) % T, ref[l - 1, covered])
    assert torch.equal(z, z4) and torch.equal(n, n4)
    assert np.count_nonzero(wild & covered) > 0


def _check_sketch(stamps_np, offsets_np, T, m, z, n, label):
    zr, nr = OS.sketch(stamps_np, offsets_np, T, m)
    np.testing.assert_array_equal(n.cpu().numpy(), nr)
    bad, err, tol = sketch_violations(to_complex(z), zr, nr)
    assert not bad.any(), f"{label}: {bad.sum()} entries off, worst err/tol {np.max(err / np.maximum(tol, 1e-300)):.3g}"
    return err


def test_tiny_frame_all_pixels():
    dev = device()
    w = synth.preset("tiny")
    f = synth.make_frame(w.frame, device=dev)
    _print_case(test="tiny", P=w.frame.P, N=f.stamps.numel())
    z, n = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m)
    torch.cuda.synchronize()
    _check_sketch(f.stamps.cpu().numpy(), f.offsets.cpu().numpy(), w.frame.T, w.m, z, n, "tiny")


@pytest.mark.parametrize("lanes", [4, 8, 16, 32, 64])
@pytest.mark.parametrize("T,m", [(4096, 16), (4613, 5), (1024, 33), (8192, 64), (2048, 1), (64, 32)])
def test_ragged_pixels_every_lane_count(lanes, T, m):
    dev = device()
    rng = np.random.default_rng(T * 131 + m * 7 + lanes)
    counts = rng.integers(0, 300, 777)
    counts[::11] = 0
    counts[5] = 3000
    pixels = [rng.integers(0, T, c) for c in counts]
    st, off, st_np, off_np = csr(pixels, dev)
    _print_case(test="ragged", T=T, m=m, lanes=lanes)
    z, n = srt.sketch(st, off, T, m, lanes=lanes)
    torch.cuda.synchronize()
    _check_sketch(st_np, off_np, T, m, z, n, f"T={T} m={m} G={lanes}")


def test_single_pixel_and_empty_frame():
    dev = device()
    for pixels in ([[5]], [[]], [[], [], []], [list(range(100))]):
        st, off, st_np, off_np = csr(pixels, dev)
        _print_case(test="single", P=len(pixels))
        z, n = srt.sketch(st, off, 128, 4)
        torch.cuda.synchronize()
        _check_sketch(st_np, off_np, 128, 4, z, n, "single")


def test_out_of_range_stamps_and_bad_offsets_are_counted():
    dev = device()
    T, m = 1000, 6
    stamps = np.array([3, -1, 1000, 2500, 7, 999, -2001], dtype=np.int64)
    offsets = np.array([0, 4, 7, 5, 7], dtype=np.int64)          # pixel 2 decreases -> empty
    err = torch.zeros(2, dtype=torch.int32, device=dev)
    _print_case(test="errors")
    z, n = srt.sketch(torch.from_numpy(stamps.astype(np.int32)).to(dev), torch.from_numpy(offsets).to(dev), T, m,
                      err=err)
    torch.cuda.synchronize()
    assert err.cpu().tolist() == [5, 1]     # -2001 is read by pixels 1 and 3
    assert n.cpu().tolist() == [4, 3, 0, 2]
    zc = to_complex(z)
    for p, sl in enumerate([slice(0, 4), slice(4, 7), slice(0, 0), slice(5, 7)]):
        zr, _ = OS.sketch(stamps[sl], np.array([0, sl.stop - sl.start]), T, m)
        bad, _, _ = sketch_violations(zc[p:p + 1], zr, np.array([sl.stop - sl.start]))
        assert not bad.any()
    # offsets beyond the stamp array are clamped, never read out of bounds
    err.zero_()
    offsets = torch.tensor([0, 2, 50], dtype=torch.int64, device=dev)
    z, n = srt.sketch(torch.tensor([1, 2, 3], dtype=torch.int32, device=dev), offsets, T, m, err=err)
    torch.cuda.synchronize()
    assert n.cpu().tolist() == [2, 1] and err.cpu().tolist() == [0, 1]


def test_long_exposure_chunks_equal_whole():
    """Two batches through the FP64 accumulators give the sketch of the whole exposure."""
    dev = device()
    rng = np.random.default_rng(9)
    T, m = 4096, 16
    counts = rng.integers(0, 2000, 300)
    pixels = [rng.integers(0, T, c) for c in counts]
    cut = [rng.integers(0, c + 1) for c in counts]
    a = [p[:c] for p, c in zip(pixels, cut)]
    b = [p[c:] for p, c in zip(pixels, cut)]
    acc = torch.zeros((300, m, 2), dtype=torch.float64, device=dev)
    nacc = torch.zeros(300, dtype=torch.int64, device=dev)
    _print_case(test="long_exposure")
    for part in (a, b):
        st, off, _, _ = csr(part, dev)
        z, n = srt.sketch(st, off, T, m, acc=acc, nacc=nacc)
    torch.cuda.synchronize()
    _, _, st_np, off_np = csr(pixels, dev)
    _check_sketch(st_np, off_np, T, m, z, n, "chunked")
    S, nr = OS.sketch_sums(st_np, off_np, T, m)
    np.testing.assert_array_equal(nacc.cpu().numpy(), nr)
    accc = acc.cpu().numpy()
    ratio = np.abs(accc[..., 0] + 1j * accc[..., 1] - S) / (1e-5 * np.sqrt(np.maximum(nr, 1))[:, None])
    assert np.max(ratio) <= 1.0, np.max(ratio)


def test_throughput_frame_sampled_pixels():
    """Full 256x256, T=4096, m=16 frame in the launch configuration the benchmark times;
    2000 sampled pixels are checked against the oracle one by one."""
    dev = device()
    w = synth.preset("throughput")
    f = synth.make_frame(w.frame, device=dev)
    _print_case(test="throughput", N=f.stamps.numel())
    z, n = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    sel = np.sort(rng.choice(w.frame.P, 2000, replace=False))
    st_np, off_np = f.stamps.cpu().numpy(), f.offsets.cpu().numpy()
    zr, nr = OS.sketch(st_np, off_np, w.frame.T, w.m, pixels=sel)
    np.testing.assert_array_equal(n.cpu().numpy()[sel], nr)
    bad, err, tol = sketch_violations(to_complex(z)[sel], zr, nr)
    print("max |dz| / tol =", float(np.max(err / tol)))
    assert not bad.any()


# --------------------------------------------------------------------------- histogram path
def _hist_frame(dev, rows=64, cols=64, lam=4000.0, seed=3, T=1024):
    spec = synth.FrameSpec(rows, cols, T, 5.0, lam, 1.0, 1, seed=seed)
    f = synth.make_frame(spec, device=dev)
    return spec, f, synth.histogram(f.stamps, f.offsets, T)


@pytest.mark.parametrize("precision", ["fp32", "fp16x2", "bf16x3"])
@pytest.mark.parametrize("m", [16, 1, 7, 32])
def test_hist_sketch_matches_oracle(precision, m):
    dev = device()
    spec, f, H = _hist_frame(dev, rows=40, cols=50)        # P = 2000: not a multiple of the row tile
    _print_case(test="hist", precision=precision, m=m)
    z, n = srt.sketch_from_hist(H, m, precision)
    torch.cuda.synchronize()
    Hn = synth.frames.hist_as_uint(H)
    zr, nr = OS.sketch_hist(Hn, m)
    np.testing.assert_array_equal(n.cpu().numpy(), nr)
    bad, err, tol = sketch_violations(to_complex(z), zr, nr)
    per_l = np.max(err / tol, axis=0)
    print(precision, "max err/tol per harmonic:", np.array2string(per_l, precision=3))
    assert not bad.any()


@pytest.mark.parametrize("T,m", [(8192, 32), (8192, 24), (32, 5), (96, 3), (2080, 9)])
def test_hist_sketch_shapes(T, m):
    """Every precision at the longest histogram (T = 8192: the largest staged F chunks and level
    table in LDS, 3 and 4 column tiles), a single 32-bin chunk, chunk counts that are not a
    multiple of the FP64 product's K (96 and 2080 bins), and a pixel count that leaves the last
    workgroup with idle waves."""
    dev = device()
    spec, f, H = _hist_frame(dev, rows=23, cols=29, lam=1500.0, seed=T + m, T=T)
    Hn = synth.frames.hist_as_uint(H)
    zr, nr = OS.sketch_hist(Hn, m)
    for precision in ("fp32", "fp16x2", "bf16x3"):
        _print_case(test="hist_shapes", T=T, m=m, precision=precision)
        z, n = srt.sketch_from_hist(H, m, precision)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(n.cpu().numpy(), nr)
        bad, err, tol = sketch_violations(to_complex(z), zr, nr)
        print(precision, "max err/tol", float((err / tol).max()))
        assert not bad.any()


@pytest.mark.parametrize("precision", ["fp32", "fp16x2", "bf16x3"])
def test_hist_hi_counts_path(precision):
    """Counts at and above 2^8 / 2^11 exercise the exact hi/lo split of the 16-bit forms, and
    rows with high levels exercise the per-chunk level removed before the product and added
    back in FP64 (a constant row sketches to exactly zero; a row whose first 32 bins hold 30000
    or 65535 counts and the rest near zero has a harmonic at which the block cancels, with n
    near 2e6, where the rule asks for 7e-9 in z).  Held to the sketch rule with no absolute
    floor."""
    dev = device()
    rng = np.random.default_rng(4)
    P, T, m = 100, 256, 8
    H = rng.integers(0, 5, (P, T)).astype(np.int64)
    H[::3, 17] = rng.integers(250, 65535, len(H[::3]))
    H[1, :] = 65535 // T                                         # constant: z = 0 exactly
    H[2, :] = rng.poisson(240, T)                                # high level, Poisson spread
    H[4, :32] = 30000                                            # level 30000, then near zero
    H[5, :32] = 65535                                            # level capped at 2^15
    H[7, :] = rng.integers(0, 65535, T)                          # uniform over the whole range
    H[8, 100:] = 1000 + rng.integers(0, 3, T - 100)              # the level set by a low start
    Ht = torch.from_numpy(np.where(H > 0x7FFF, H - 0x10000, H).astype(np.int16)).to(dev)
    _print_case(test="hist_hi", precision=precision)
    z, n = srt.sketch_from_hist(Ht, m, precision)
    torch.cuda.synchronize()
    zr, nr = OS.sketch_hist(H, m)
    np.testing.assert_array_equal(n.cpu().numpy(), nr)
    bad, err, tol = sketch_violations(to_complex(z), zr, nr)
    print(precision, "max err/tol", float((err / tol).max()), "constant row max |z|", float(np.abs(to_complex(z)[1]).max()))
    assert not bad.any()


def test_hist_constant_rows_are_zero_and_match_photon_path():
    dev = device()
    T, m = 512, 8
    H = np.full((3, T), 7, dtype=np.int64)
    H[1] = 0
    Ht = torch.from_numpy(H.astype(np.int16)).to(dev)
    for precision in ("fp32", "fp16x2", "bf16x3"):
        z, n = srt.sketch_from_hist(Ht, m, precision)
        torch.cuda.synchronize()
        zc = to_complex(z)
        assert np.max(np.abs(zc)) < 1e-6 and n.cpu().tolist() == [7 * T, 0, 7 * T]
    # the histogram of a photon list sketches like the list itself
    rng = np.random.default_rng(5)
    pixels = [rng.integers(0, T, c) for c in rng.integers(0, 500, 64)]
    st, off, st_np, off_np = csr(pixels, dev)
    zp, npp = srt.sketch(st, off, T, m)
    Hh = synth.histogram(st, off, T)
    zh, nh = srt.sketch_from_hist(Hh, m, "fp32")
    torch.cuda.synchronize()
    assert torch.equal(npp, nh)
    bad, _, _ = sketch_violations(to_complex(zh), to_complex(zp), npp.cpu().numpy())
    assert not bad.any()


def test_hist_precision_frame_sampled_rows():
    """Full 256x256 x T=1024 histograms at ~4000 photons/pixel, every precision, sampled rows."""
    dev = device()
    w = synth.preset("precision")
    f = synth.make_frame(w.frame, device=dev)
    H = synth.histogram(f.stamps, f.offsets, w.frame.T)
    rng = np.random.default_rng(2)
    sel = np.sort(rng.choice(w.frame.P, 1500, replace=False))
    Hn = synth.frames.hist_as_uint(H[torch.from_numpy(sel).to(dev)])
    zr, nr = OS.sketch_hist(Hn, w.m)
    for precision in ("fp32", "fp16x2", "bf16x3"):
        _print_case(test="hist_full", precision=precision)
        z, n = srt.sketch_from_hist(H, w.m, precision)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(n.cpu().numpy()[sel], nr)
        bad, err, tol = sketch_violations(to_complex(z)[sel], zr, nr)
        print(precision, "max err/tol per harmonic:", np.array2string(np.max(err / tol, 0), precision=3))
        assert not bad.any()


def test_binding_checks_output_shapes():
    """The C ABI takes no output sizes: the binding refuses mis-shaped outputs, accumulators and
    a histogram workspace prepared for another shape or precision before any launch."""
    dev = device()
    st, off, _, _ = csr([[1, 2, 3], [4], []], dev)
    P, T, m = 3, 64, 4
    with pytest.raises(ValueError):
        srt.sketch(st, off, T, m, z=torch.empty((P, m + 1, 2), device=dev))
    with pytest.raises(ValueError):
        srt.sketch(st, off, T, m, n=torch.empty(P - 1, dtype=torch.int32, device=dev))
    with pytest.raises(ValueError):
        srt.sketch(st, off, T, m, acc=torch.zeros((P, m, 2), dtype=torch.float64, device=dev),
                   nacc=torch.zeros(P + 1, dtype=torch.int64, device=dev))
    with pytest.raises(ValueError):
        srt.sketch(st, off, T, m, acc=torch.zeros((P, m, 2), dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        srt.sketch(st, off, T, m, method="binned", lanes=8)
    H = torch.zeros((P, 128), dtype=torch.int16, device=dev)
    ws = srt.hist_workspace(128, 8, "fp32", dev)
    with pytest.raises(ValueError):
        srt.sketch_from_hist(H, 4, "fp32", workspace=ws)
    with pytest.raises(ValueError):
        srt.sketch_from_hist(H, 8, "fp16x2", workspace=ws)
    z, n = srt.sketch_from_hist(H, 8, "fp32", workspace=ws)
    torch.cuda.synchronize()
    assert n.tolist() == [0, 0, 0] and not z.any()
