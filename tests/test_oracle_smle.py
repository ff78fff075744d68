"""Pins of the pixelwise sketched estimator (SMLE) oracle: exact recovery from noiseless sketches,
the global minimum against brute force over a fine depth grid, start construction, descent and
the selection rule."""
import numpy as np

from oracle import model as OM
from oracle import smle as OS
from oracle import srt3d as O


def _gauss_irf(sigma):
    o = int(np.ceil(6 * sigma))
    return np.exp(-0.5 * (np.arange(-o, o + 1) / sigma) ** 2), o


def _circ(d, T):
    d = np.mod(d, T)
    return np.minimum(d, T - d)


def test_noiseless_sketch_recovers_the_surface():
    """z = Phi(theta*) exactly: the loss is zero at theta* and the estimator returns theta*."""
    T, m, P = 1024, 8, 24
    rng = np.random.default_rng(1)
    h, o = _gauss_irf(3.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    t = rng.uniform(0, T, (P, 1))
    alpha = rng.uniform(0.3, 0.9, (P, 1))
    z = OM.model_sketch(t, alpha, np.ones((P, 1), bool), hhat, T)
    n = np.full(P, 500)
    r = OS.smle(z, n, h, o, O.Params(T, m, 1), starts=4, iters=400)
    st = r["state"]
    assert st.active.all()
    assert np.max(_circ(st.t - t, T)) < 1e-3
    np.testing.assert_allclose(st.alpha, alpha, atol=1e-5)
    assert np.max(r["loss"]) < 1e-8


def _profile_minimum(z, n, hhat, T, step):
    """Brute force for K = 1: the loss at every depth of a grid of spacing `step`, the amplitude
    at each depth its least-squares value clipped to [0, 1] (the exact minimiser over alpha of a
    convex quadratic on an interval).  Returns (min loss, argmin depth) per pixel."""
    grid = np.arange(0.0, T, step)
    g = hhat * OM.unit_phasors(grid, T, hhat.size)                     # [G, m]
    e2 = np.sum(np.abs(hhat) ** 2)
    c = (np.conj(g)[None, :, :] * z[:, None, :]).sum(-1).real          # [P, G]
    a = np.clip(c / e2, 0.0, 1.0)
    res = z[:, None, :] - a[..., None] * g[None]
    L = n[:, None] * (np.abs(res) ** 2).sum(-1)
    j = np.argmin(L, axis=1)
    return L[np.arange(z.shape[0]), j], grid[j]


def test_global_minimum_against_brute_force():
    """Noisy single-surface sketches: the multi-start result is the global minimum of the
    pixel's loss found by exhaustive search over depth (grid spacing 0.02 bins)."""
    T, m, P = 512, 6, 40
    rng = np.random.default_rng(2)
    h, o = _gauss_irf(2.5)
    hhat = OM.irf_spectrum(h, o, T, m)
    t = rng.uniform(0, T, (P, 1))
    alpha = rng.uniform(0.3, 0.8, (P, 1))
    n = rng.integers(50, 400, P)
    z = OM.model_sketch(t, alpha, np.ones((P, 1), bool), hhat, T)
    z = z + (rng.normal(0, 1, z.shape) + 1j * rng.normal(0, 1, z.shape)) * 0.5 / np.sqrt(n)[:, None]
    r = OS.smle(z, n, h, o, O.Params(T, m, 1), starts=8, iters=600)
    Lb, tb = _profile_minimum(z, n, hhat, T, 0.02)
    # the grid minimum is within (grid spacing)^2 curvature of the true minimum: the estimate
    # may only be lower, and by a small amount
    assert np.all(r["loss"] <= Lb * (1 + 1e-9) + 1e-12)
    assert np.all(r["loss"] >= Lb - 1e-3 * np.maximum(Lb, 1e-3))
    assert np.max(_circ(r["state"].t[:, 0] - tb, T)) <= 0.05


def test_start_points_closed_form():
    """Start s puts point k at (s T / S + k T / K) mod T; a noiseless atom sitting exactly at a
    start gets its amplitude back from the single-atom least-squares fit."""
    T, m, K, S = 600, 6, 2, 4
    p = O.Params(T, m, K)
    hhat = OM.irf_spectrum([1.0], 0, T, m)          # delta response, m even: atoms T/2 apart
                                                    # are orthogonal
    t_true = np.array([[150.0, 450.0]])             # start 1 of 4: 150 and 150 + 300
    a_true = np.array([[0.35, 0.25]])
    z = OM.model_sketch(t_true, a_true, np.ones((1, 2), bool), hhat, T)
    init = O.init_points(z, np.array([100]), hhat, p)
    st = OS.start_points(z, np.array([100]), hhat, p, 1, S, init)
    np.testing.assert_allclose(st.t, t_true, atol=1e-12)
    np.testing.assert_allclose(st.alpha, a_true, atol=1e-12)
    st2 = OS.start_points(z, np.array([100]), hhat, p, 3, S, init)
    np.testing.assert_allclose(st2.t, [[450.0, 150.0]], atol=1e-12)
    st0 = OS.start_points(z, np.array([100]), hhat, p, 0, S, init)
    np.testing.assert_array_equal(st0.t, init.t)
    # no photons: the start has no active point
    st3 = OS.start_points(z, np.array([0]), hhat, p, 2, S, init)
    assert not st3.active.any() and not st3.alpha.any()


def test_descent_never_increases_the_loss_and_selection_is_the_minimum():
    T, m, P, K = 256, 6, 30, 2
    rng = np.random.default_rng(4)
    h, o = _gauss_irf(2.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    p = O.Params(T, m, K)
    z = rng.normal(0, 0.3, (P, m)) + 1j * rng.normal(0, 0.3, (P, m))
    n = rng.integers(0, 300, P)
    n[:3] = 0
    init = O.init_points(z, n, hhat, p)
    S = 5
    for s in range(S):
        st = OS.start_points(z, n, hhat, p, s, S, init)
        L0 = OM.loss(z, n, st.t, st.alpha, st.active, hhat, T)
        st1 = OS.descend(st, z, n, hhat, p, 1)
        L1 = OM.loss(z, n, st1.t, st1.alpha, st1.active, hhat, T)
        assert np.all(L1 <= L0 + 1e-12)
    r = OS.smle(z, n, h, o, p, starts=S, iters=30)
    L = r["losses"]
    np.testing.assert_array_equal(r["loss"], L.min(0))
    np.testing.assert_array_equal(r["start"], np.argmin(L, axis=0))      # earliest on ties
    np.testing.assert_allclose(r["loss"], OM.loss(z, n, r["state"].t, r["state"].alpha, r["state"].active, hhat, T))
    assert np.all(r["loss"][:3] == 0)
