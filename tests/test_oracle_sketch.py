"""Pins of the sketch oracle (eq. 2, eq. 3) against hand-derived values and identities."""
import math

import numpy as np
import pytest

from oracle import sketch as OS

pytestmark = pytest.mark.filterwarnings("ignore")


def _csr(pixels):
    stamps = np.concatenate([np.asarray(p, dtype=np.int64) for p in pixels]) if pixels else np.zeros(0)
    offsets = np.zeros(len(pixels) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in pixels])
    return stamps, offsets


def test_golden_hand_derived(golden):
    for (T, m), stamps, expect in golden("sketch_small.txt"):
        x = np.asarray(stamps, dtype=np.int64)
        z, n = OS.sketch(*_csr([x]), T, m)
        assert n[0] == len(x)
        np.testing.assert_allclose(z[0], expect, atol=1e-15)
        zl, nl = OS.sketch_loop(x, T, m)
        np.testing.assert_allclose(zl, expect, atol=1e-15)


def test_single_photon_unit_modulus():
    rng = np.random.default_rng(0)
    for _ in range(50):
        T = int(rng.integers(2, 10000))
        m = int(rng.integers(1, T // 2 + 1)) if T >= 2 else 1
        x = int(rng.integers(0, T))
        z, n = OS.sketch(*_csr([[x]]), T, min(m, 64))
        assert n[0] == 1
        np.testing.assert_allclose(np.abs(z[0]), 1.0, atol=1e-14)


def test_shift_identity():
    """z_l(x + D mod T) = exp(i w_l D) z_l(x) for an integer shift D."""
    rng = np.random.default_rng(1)
    for T in (1024, 4613, 4096):
        m = 16
        x = rng.integers(0, T, 500)
        for D in (1, 7, T // 3, T - 1):
            z0, _ = OS.sketch(*_csr([x]), T, m)
            z1, _ = OS.sketch(*_csr([(x + D) % T]), T, m)
            ph = np.exp(1j * 2 * np.pi * np.arange(1, m + 1) * D / T)
            np.testing.assert_allclose(z1[0], ph * z0[0], atol=1e-12)


@pytest.mark.parametrize("T", [2, 3, 8, 1024, 4613])
def test_uniform_background_is_invisible(T):
    """Every bin once: sum_x exp(i w_l x) = 0 for 1 <= l <= T-1 (Section 2, background-blind sampling)."""
    m = T - 1 if T < 64 else 64
    z, n = OS.sketch(*_csr([np.arange(T)]), T, m)
    assert n[0] == T
    np.testing.assert_allclose(z[0], 0.0, atol=1e-12)


def test_random_uniform_ecf_variance():
    """Uniform stamps: E z_l = 0 and E |z_l|^2 = 1/n (eq. 5 with Psi = 0)."""
    rng = np.random.default_rng(2)
    T, m, n, P = 1024, 8, 50, 4000
    x = rng.integers(0, T, (P, n))
    z, _ = OS.sketch(*_csr(list(x)), T, m)
    mean_sq = (np.abs(z) ** 2).mean(0) * n
    assert np.all(np.abs(mean_sq - 1.0) < 5 * math.sqrt(1.0 / P) * 1.5)
    assert np.all(np.abs(z.mean(0)) < 5 / math.sqrt(n * P))


@pytest.mark.parametrize("T", [8, 16, 30, 64])
def test_inverse_dft_recovers_histogram(T):
    """With m = T/2 the sketch and n determine the histogram exactly:
    y_t = (1/T) [n + 2 sum_{l<T/2} Re(n z_l e^{-i w_l t}) + Re(n z_{T/2}) (-1)^t]."""
    rng = np.random.default_rng(T)
    x = rng.integers(0, T, 200)
    m = T // 2
    z, n = OS.sketch(*_csr([x]), T, m)
    nz = n[0] * z[0]
    t = np.arange(T)
    y = np.full(T, float(n[0]))
    for ell in range(1, m):
        y += 2 * (nz[ell - 1] * np.exp(-1j * 2 * np.pi * ell * t / T)).real
    y += nz[m - 1].real * (-1.0) ** t
    y /= T
    np.testing.assert_allclose(y, np.bincount(x, minlength=T), atol=1e-9)
    assert np.array_equal(np.rint(y).astype(int), np.bincount(x, minlength=T))


def test_histogram_sketch_equals_photon_sketch():
    rng = np.random.default_rng(3)
    T, m = 4613, 12
    pixels = [rng.integers(0, T, int(k)) for k in rng.integers(0, 300, 40)]
    z, n = OS.sketch(*_csr(pixels), T, m)
    H = np.stack([np.bincount(p, minlength=T) for p in pixels])
    zh, nh = OS.sketch_hist(H, m)
    assert np.array_equal(n, nh)
    np.testing.assert_allclose(zh, z, atol=1e-12)


def test_empty_pixel_and_folding():
    T, m = 64, 5
    stamps, offsets = _csr([[], [3, 70, -5], [], [1]])
    z, n = OS.sketch(stamps, offsets, T, m)
    assert list(n) == [0, 3, 0, 1]
    assert np.all(z[0] == 0) and np.all(z[2] == 0)
    zf, _ = OS.sketch(*_csr([[3, 70 % 64, (-5) % 64]]), T, m)
    np.testing.assert_allclose(z[1], zf[0], atol=1e-15)


def test_phase_indices_brute_force():
    rng = np.random.default_rng(4)
    for T in (7, 1024, 4613, 8192):
        m = min(32, T // 2)
        x = rng.integers(-3 * T, 3 * T, 300)
        k = OS.phase_indices(x, T, m)
        for ell in range(1, m + 1):
            assert [int(v) for v in k[ell - 1]] == [(ell * int(xx)) % T for xx in x]


def test_loop_matches_vectorised():
    rng = np.random.default_rng(5)
    T, m = 1000, 9
    pixels = [rng.integers(0, T, int(k)) for k in rng.integers(0, 60, 10)]
    z, n = OS.sketch(*_csr(pixels), T, m)
    for p, x in enumerate(pixels):
        zl, nl = OS.sketch_loop(x, T, m)
        assert nl == n[p]
        np.testing.assert_allclose(zl, z[p], atol=1e-14)


def test_pixel_subset():
    rng = np.random.default_rng(6)
    T, m = 512, 6
    pixels = [rng.integers(0, T, int(k)) for k in rng.integers(0, 40, 30)]
    z, n = OS.sketch(*_csr(pixels), T, m)
    sel = np.array([29, 0, 5, 5, 17])
    zs, ns = OS.sketch(*_csr(pixels), T, m, pixels=sel)
    np.testing.assert_array_equal(ns, n[sel])
    np.testing.assert_allclose(zs, z[sel], atol=0)


# ----------------------------------------------------------------------------- event streams
def _stream(rng, P, T, counts):
    """A shuffled arrival-order stream holding `counts[p]` uniform stamps for pixel p."""
    pix = np.repeat(np.arange(P), counts)
    st = rng.integers(0, T, pix.size)
    order = rng.permutation(pix.size)
    return pix[order], st[order]


def test_event_stream_matches_per_pixel_loop():
    """Each pixel's sum is the correctly rounded per-photon loop over its events."""
    rng = np.random.default_rng(11)
    P, T, m = 12, 997, 7
    pix, st = _stream(rng, P, T, rng.integers(0, 40, P))
    z, n = OS.sketch_events(pix, st, P, T, m)
    for p in range(P):
        zl, nl = OS.sketch_loop(st[pix == p], T, m)
        assert nl == n[p]
        np.testing.assert_allclose(zl, z[p], atol=1e-14)


def test_event_stream_order_does_not_matter():
    rng = np.random.default_rng(12)
    P, T, m = 40, 4096, 16
    pix, st = _stream(rng, P, T, rng.integers(0, 300, P))
    z, n = OS.sketch_events(pix, st, P, T, m)
    for _ in range(3):
        o = rng.permutation(pix.size)
        z2, n2 = OS.sketch_events(pix[o], st[o], P, T, m)
        np.testing.assert_array_equal(n2, n)
        np.testing.assert_allclose(z2, z, atol=1e-12)


def test_event_stream_chunks_add_up():
    """The sums are linear in the stream: any split into consecutive chunks adds up to the whole."""
    rng = np.random.default_rng(13)
    P, T, m = 25, 2048, 8
    pix, st = _stream(rng, P, T, rng.integers(0, 200, P))
    S, n, _, _ = OS.sketch_event_sums(pix, st, P, T, m)
    cut = pix.size // 3
    S1, n1, _, _ = OS.sketch_event_sums(pix[:cut], st[:cut], P, T, m)
    S2, n2, _, _ = OS.sketch_event_sums(pix[cut:], st[cut:], P, T, m)
    np.testing.assert_array_equal(n1 + n2, n)
    np.testing.assert_allclose(S1 + S2, S, atol=1e-10)


def test_event_stream_closed_forms_and_bad_events():
    T, m, P = 64, 5, 4
    # pixel 0: one photon (|z| = 1); pixel 1: every stamp once (z = 0, eq. 4 with a uniform
    # background); pixel 2: nothing; pixel 3: a folded stamp.  Events for pixels -1 and 4 are
    # outside the frame.
    pix = [0, 4] + [1] * T + [-1, 3, 3]
    st = [9, 1] + list(range(T)) + [5, 70, 6]
    S, n, dropped, folded = OS.sketch_event_sums(pix, st, P, T, m)
    z, _ = OS.sketch_events(pix, st, P, T, m)
    assert list(n) == [1, T, 0, 2] and dropped == 2 and folded == 1
    np.testing.assert_allclose(np.abs(z[0]), 1.0, atol=1e-15)
    np.testing.assert_allclose(z[1], 0.0, atol=1e-13)
    assert np.all(z[2] == 0)
    z3, _ = OS.sketch(*_csr([[70 % T, 6]]), T, m)
    np.testing.assert_allclose(z[3], z3[0], atol=1e-15)
