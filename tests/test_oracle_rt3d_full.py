"""Pins of the full-data RT3D oracle (oracle/rt3d_full.py) and the quality cross-check it exists
for: SRT3D (sketched data term, eq. 8) and RT3D (every photon, eq. 1) reconstruct high-SBR frames
equally well against the synthetic truth (Section 4)."""
import math

import numpy as np
import pytest
from scipy.stats import poisson

import synth
from oracle import rt3d_full as RF
from oracle import sketch as OS
from oracle import srt3d as O


def _irf(sigma=3.0):
    h, o = synth.binned_gaussian_irf(sigma)
    return h, o


def _state(rng, P, K, T, active_frac=1.0):
    t = rng.uniform(0, T, (P, K))
    t = np.floor(t) + rng.uniform(0.2, 0.8, (P, K))           # away from the interpolation kinks
    a = rng.uniform(0.05, 0.3, (P, K))
    act = rng.uniform(size=(P, K)) < active_frac
    act[:, 0] = True
    return t, np.where(act, a, 0.0), act


def test_irf_interpolation_is_the_normalised_response():
    h, o = _irf(2.5)
    hn = h / h.sum()
    lags = np.arange(h.size) - o
    v, d = RF.irf_at(h, o, lags.astype(np.float64))
    np.testing.assert_allclose(v, hn, rtol=0, atol=1e-15)
    mid, _ = RF.irf_at(h, o, lags[:-1] + 0.25)
    np.testing.assert_allclose(mid, 0.75 * hn[:-1] + 0.25 * hn[1:], atol=1e-15)
    out, dout = RF.irf_at(h, o, np.array([-o - 1.5, o + 1.0, o + 7.3]))
    assert np.all(out == 0) and np.all(dout == 0)
    # for any real shift the circular shape sums to one over the T bins (so sum_x pi_x = 1)
    T = 97
    for t in (0.0, 3.4, 50.5, 96.9):
        H, _ = RF.irf_at(h, o, O.circ_diff(np.arange(T) - t, T))
        assert H.sum() == pytest.approx(1.0, abs=1e-14)


def test_dense_nll_is_the_poisson_likelihood_of_the_histogram():
    """nll = -sum_x log Poisson(y_x; mu_x) - sum_x log y_x! with mu = n pi (scipy's pmf), and it
    equals n - n log n - sum_x y_x log pi_x because sum_x pi_x = 1."""
    rng = np.random.default_rng(0)
    T, P, K = 64, 12, 2
    h, o = _irf(2.0)
    t, a, act = _state(rng, P, K, T, 0.6)
    y = rng.poisson(0.4, (P, T)).astype(np.float64)
    n = y.sum(1)
    L = RF.nll(y, n, t, a, act, h, o, T)
    pi, _, _ = RF.pmf(t, a, act, h, o, T)
    np.testing.assert_allclose(pi.sum(1), 1.0, atol=1e-14)
    mu = n[:, None] * pi
    ref = -poisson.logpmf(y, mu).sum(1) - np.vectorize(math.lgamma)(y + 1).sum(1)
    np.testing.assert_allclose(L, ref, rtol=1e-12)
    closed = n - n * np.log(n) - (y * np.log(pi)).sum(1)
    np.testing.assert_allclose(L, closed, rtol=1e-12)


def test_sparse_form_equals_the_dense_form():
    rng = np.random.default_rng(1)
    T, P, K = 128, 20, 3
    h, o = _irf(3.0)
    t, a, act = _state(rng, P, K, T, 0.7)
    y = rng.poisson(0.2, (P, T)).astype(np.float64)
    y[3] = 0                                                   # an empty pixel
    n = y.sum(1)
    ph = RF.Photons(y)
    np.testing.assert_allclose(ph.nll(t, a, act, h, o, T), RF.nll(y, n, t, a, act, h, o, T), rtol=1e-12, atol=1e-12)
    gs = ph.gradients(t, a, act, h, o, T)
    gd = RF.nll_gradients(y, n, t, a, act, h, o, T)
    for s_, d_ in zip(gs, gd):
        np.testing.assert_allclose(s_, d_, rtol=1e-11, atol=1e-11)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(2)
    T, P, K = 64, 6, 2
    h, o = _irf(2.0)
    t, a, act = _state(rng, P, K, T)
    y = rng.poisson(0.5, (P, T)).astype(np.float64)
    n = y.sum(1)
    gt, ga = RF.nll_gradients(y, n, t, a, act, h, o, T)
    eps = 1e-6
    for k in range(K):
        dt = np.zeros_like(t)
        dt[:, k] = eps
        fd = (RF.nll(y, n, t + dt, a, act, h, o, T) - RF.nll(y, n, t - dt, a, act, h, o, T)) / (2 * eps)
        np.testing.assert_allclose(gt[:, k], fd, rtol=1e-6, atol=1e-6)
        fa = (RF.nll(y, n, t, a + dt, act, h, o, T) - RF.nll(y, n, t, a - dt, act, h, o, T)) / (2 * eps)
        np.testing.assert_allclose(ga[:, k], fa, rtol=1e-6, atol=1e-6)


def test_noiseless_histogram_is_a_stationary_point_and_the_minimum():
    """y = n pi(theta*) (the expected histogram): the gradient vanishes at theta* (sum_x y_x d log
    pi_x = n d(sum_x pi_x) = 0), and theta* beats every perturbation (the KL divergence)."""
    rng = np.random.default_rng(3)
    T, P, K = 96, 8, 2
    h, o = _irf(2.0)
    t = np.stack([rng.uniform(10, 40, P), rng.uniform(55, 85, P)], 1) + 0.37
    a = np.stack([rng.uniform(0.2, 0.4, P), rng.uniform(0.2, 0.4, P)], 1)
    act = np.ones((P, K), dtype=bool)
    n = np.full(P, 500.0)
    pi, _, _ = RF.pmf(t, a, act, h, o, T)
    y = n[:, None] * pi
    gt, ga = RF.nll_gradients(y, n, t, a, act, h, o, T)
    assert np.abs(gt).max() < 1e-9 and np.abs(ga).max() < 1e-9
    L0 = RF.nll(y, n, t, a, act, h, o, T)
    for _ in range(5):
        dt = rng.normal(0, 0.3, t.shape)
        da = rng.normal(0, 0.02, a.shape)
        assert np.all(RF.nll(y, n, t + dt, a + da, act, h, o, T) > L0)


def test_data_step_never_raises_the_likelihood_and_converges_on_noiseless_data():
    rng = np.random.default_rng(4)
    T, P, K = 128, 30, 1
    h, o = _irf(3.0)
    t_true = rng.uniform(20, 100, (P, 1)) + 0.25
    a_true = np.full((P, 1), 0.6)
    act = np.ones((P, 1), dtype=bool)
    n = np.full(P, 1000.0)
    pi, _, _ = RF.pmf(t_true, a_true, act, h, o, T)
    y = np.round(n[:, None] * pi * 8) / 8                       # near-noiseless, non-integer counts
    ph = RF.Photons(y)
    p = O.Params(T, 4, K)
    st = O.State(t_true + rng.uniform(-3, 3, (P, 1)), np.full((P, 1), 0.3), act)
    gt, ga = np.full(P, RF.START_STEP_T), np.full(P, RF.START_STEP_A)
    L = ph.nll(st.t, st.alpha, st.active, h, o, T)
    for _ in range(200):
        st, gt, ga = RF.data_step(st, ph, h, o, p, gt * 2, ga * 2)
        L1 = ph.nll(st.t, st.alpha, st.active, h, o, T)
        assert np.all(L1 <= L + 1e-9)
        L = L1
    assert np.abs(O.circ_diff(st.t - t_true, T)).max() < 0.05
    assert np.abs(st.alpha - a_true).max() < 5e-3


def _detection(out, scene, T, tol):
    """Fraction of the true surfaces (weight > 0) with an active reconstructed point within `tol`
    bins (circular), and the fraction of active points within `tol` of some true surface."""
    hit = tot = 0
    good = np.zeros_like(out["active"])
    for k in range(scene.depth.shape[1]):
        present = scene.weight[:, k] > 0
        close = np.abs(O.circ_diff(out["depth"] - scene.depth[:, k:k + 1], T)) <= tol
        hit += ((out["active"] & close).any(1) & present).sum()
        tot += present.sum()
        good |= close & present[:, None]
    return hit / tot, (good & out["active"]).sum() / max(1, out["active"].sum())


FRAMES = [
    # the tiny frame's shape (32x32, T = 1024, sigma = 5, ~10 photons/px, m = 4) at SBR 10
    ("tiny_sbr10_a", synth.FrameSpec(32, 32, 1024, 5.0, 10.0, 10.0, 1, seed=101), 4, 1, 1.0),
    ("tiny_sbr10_b", synth.FrameSpec(32, 32, 1024, 5.0, 10.0, 10.0, 1, seed=102), 4, 1, 1.0),
    ("tiny_sbr10_c", synth.FrameSpec(32, 32, 1024, 5.0, 10.0, 10.0, 1, seed=104), 4, 1, 1.0),
    # the camouflage-like two-surface frame (32x32, T = 153, m = 10, K = 2)
    ("camouflage", synth.FrameSpec(32, 32, 153, 2.0, 200.0, 2.0, 2, seed=11), 10, 2, 5.0),
]


@pytest.mark.parametrize("name,spec,m,K,r_min", FRAMES, ids=[f[0] for f in FRAMES])
def test_srt3d_and_full_data_rt3d_reconstruct_equally_well(name, spec, m, K, r_min):
    """Both find the synthetic surfaces within 3 sigma on the same fraction of them (within 1%),
    and at least 99%, from the same initialisation, denoisers and 50 iterations."""
    f = synth.make_frame(spec)
    z, n = OS.sketch(f.stamps.numpy(), f.offsets.numpy(), spec.T, m)
    y = synth.frames.hist_as_uint(synth.histogram(f.stamps, f.offsets, spec.T)).astype(np.float64)
    p = O.Params(spec.T, m, K, iters=50, r_min=r_min)
    rs = O.reconstruct(z, n, f.irf, f.irf_origin, spec.rows, spec.cols, p)
    rf = RF.reconstruct(y, z, n, f.irf, f.irf_origin, spec.rows, spec.cols, p)
    tol = 3.0 * spec.sigma
    ds, ps = _detection(rs, f.scene, spec.T, tol)
    df, pf = _detection(rf, f.scene, spec.T, tol)
    print(f"{name}: detected SRT3D {ds:.4f} RT3D {df:.4f}; points on a surface SRT3D {ps:.4f} RT3D {pf:.4f}")
    assert ds >= 0.99 and df >= 0.99
    assert abs(ds - df) <= 0.01
    assert ps >= 0.99 and pf >= 0.99
