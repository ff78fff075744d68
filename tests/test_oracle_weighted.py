"""Pins of the precision-weighted pixelwise estimator (eq. 6 with W = Sigma^{-1}): the covariance
against brute-force expectation over the mixture pmf of eq. (1), its reduction to a multiple of
the identity without signal, the Jacobian against finite differences, and the weighted fit
against the W = I minimum and against noiseless sketches."""
import numpy as np
import pytest

from oracle import model as OM
from oracle import smle as OSM
from oracle import srt3d as O
from oracle import weighted as OW


def _mixture_pmf(T, h, o, t, alpha, alpha0):
    """pi(x) of eq. (1) on x = 0..T-1 for integer depths, impulse response wrapped mod T."""
    pi = np.full(T, alpha0 / T)
    h = np.asarray(h, dtype=np.float64) / np.sum(h)
    for tk, ak in zip(t, alpha):
        for i, hi in enumerate(h):
            pi[(tk + i - o) % T] += ak * hi
    return pi


@pytest.mark.parametrize("T,m", [(64, 7), (4613, 12), (1000, 31)])
def test_covariance_is_the_expected_outer_product(T, m):
    """Sigma = sum_x pi(x) phi(x) phi(x)^T - mu mu^T with phi = [cos w_l x, sin w_l x] by brute
    force over the support of eq. (1)'s pmf."""
    rng = np.random.default_rng(T + m)
    h = rng.uniform(0, 1, 9)
    o = 4
    t = rng.integers(0, T, 3)
    alpha = np.array([0.3, 0.2, 0.1])
    pi = _mixture_pmf(T, h, o, t, alpha, 0.4)
    x = np.arange(T)
    w = 2 * np.pi * np.arange(1, m + 1) / T
    phi = np.concatenate([np.cos(np.outer(x, w)), np.sin(np.outer(x, w))], 1)      # [T, 2m]
    mu = pi @ phi
    S_bf = (phi * pi[:, None]).T @ phi - np.outer(mu, mu)
    hhat2 = OM.irf_spectrum(h, o, T, 2 * m)
    S = OW.covariance(t[None].astype(float), alpha[None], np.ones((1, 3), bool), hhat2, T, m)[0]
    np.testing.assert_allclose(S, S_bf, atol=1e-12)
    assert np.allclose(S, S.T) and np.min(np.linalg.eigvalsh(S)) > -1e-12


def test_no_signal_reduces_to_identity():
    """alpha = 0: Psi_j = 0 for 0 < j <= 2m, Sigma = I / 2 exactly, and the weighted fit takes
    exactly the W = I steps (the loss is scaled by 2)."""
    T, m, P = 300, 6, 5
    hhat2 = OM.irf_spectrum([0.2, 1.0, 0.5], 1, T, 2 * m)
    t = np.random.default_rng(0).uniform(0, T, (P, 2))
    S = OW.covariance(t, np.zeros((P, 2)), np.ones((P, 2), bool), hhat2, T, m)
    np.testing.assert_array_equal(S, np.broadcast_to(0.5 * np.eye(2 * m), S.shape))
    rng = np.random.default_rng(1)
    hhat = hhat2[:m]
    z = rng.normal(0, 0.3, (P, m)) + 1j * rng.normal(0, 0.3, (P, m))
    n = rng.integers(10, 500, P)
    st0 = O.State(rng.uniform(0, T, (P, 2)), np.full((P, 2), 0.2), np.ones((P, 2), bool))
    Lh = np.broadcast_to(np.sqrt(0.5) * np.eye(2 * m), (P, 2 * m, 2 * m))
    L1 = np.broadcast_to(np.eye(2 * m), (P, 2 * m, 2 * m))
    a, la = OW.weighted_fit(z, n, st0, hhat, Lh, T, 15)
    b, lb = OW.weighted_fit(z, n, st0, hhat, L1, T, 15)
    np.testing.assert_allclose(a.t, b.t, atol=1e-10)
    np.testing.assert_allclose(a.alpha, b.alpha, atol=1e-12)
    np.testing.assert_allclose(la, 2 * lb, rtol=1e-10)


def test_jacobian_matches_finite_differences():
    T, m, P, K = 500, 5, 4, 3
    rng = np.random.default_rng(2)
    hhat = OM.irf_spectrum(rng.uniform(0, 1, 7), 3, T, m)
    t = rng.uniform(0, T, (P, K))
    alpha = rng.uniform(0.05, 0.3, (P, K))
    act = np.array([[True, True, False]] * P)
    z = np.zeros((P, m), complex)
    _, J = OW.residual_and_jacobian(z, t, alpha, act, hhat, T)
    eps = 1e-6
    for k in range(K):
        for which, base in ((0, t), (1, alpha)):
            up, dn = base.copy(), base.copy()
            up[:, k] += eps
            dn[:, k] -= eps
            args_up = (up, alpha) if which == 0 else (t, up)
            args_dn = (dn, alpha) if which == 0 else (t, dn)
            ru, _ = OW.residual_and_jacobian(z, *args_up, act, hhat, T)
            rd, _ = OW.residual_and_jacobian(z, *args_dn, act, hhat, T)
            fd = -(ru - rd) / (2 * eps)                       # r = z - Phi
            col = J[:, :, which * K + k]
            if act[0, k]:
                np.testing.assert_allclose(col, fd, atol=1e-7)
            else:
                assert not col.any()


def test_identity_weighting_reaches_the_unweighted_minimum():
    """With L = I the fit minimises the W = I loss: from a perturbed start it lands on the
    pixelwise W = I estimate."""
    T, m, P = 512, 6, 30
    rng = np.random.default_rng(3)
    sig = 2.5
    o = int(np.ceil(6 * sig))
    h = np.exp(-0.5 * (np.arange(-o, o + 1) / sig) ** 2)
    hhat = OM.irf_spectrum(h, o, T, m)
    t = rng.uniform(0, T, (P, 1))
    alpha = rng.uniform(0.3, 0.8, (P, 1))
    n = rng.integers(50, 400, P)
    z = OM.model_sketch(t, alpha, np.ones((P, 1), bool), hhat, T)
    z = z + (rng.normal(0, 1, z.shape) + 1j * rng.normal(0, 1, z.shape)) * 0.5 / np.sqrt(n)[:, None]
    ref = OSM.smle(z, n, h, o, O.Params(T, m, 1), starts=4, iters=2000)["state"]
    start = O.State(ref.t + rng.uniform(-1, 1, (P, 1)), np.clip(ref.alpha * 0.8, 0, 1), ref.active.copy())
    L1 = np.broadcast_to(np.eye(2 * m), (P, 2 * m, 2 * m))
    st, _ = OW.weighted_fit(z, n, start, hhat, L1, T, 60)
    d = np.mod(st.t - ref.t + T / 2, T) - T / 2
    assert np.max(np.abs(d)) < 1e-5
    np.testing.assert_allclose(st.alpha, ref.alpha, atol=1e-6)


def test_noiseless_sketch_is_a_fixed_point_and_is_reached():
    T, m, P = 1024, 8, 20
    rng = np.random.default_rng(4)
    sig = 3.0
    o = int(np.ceil(6 * sig))
    h = np.exp(-0.5 * (np.arange(-o, o + 1) / sig) ** 2)
    hhat = OM.irf_spectrum(h, o, T, m)
    hhat2 = OM.irf_spectrum(h, o, T, 2 * m)
    t = rng.uniform(0, T, (P, 2))
    alpha = rng.uniform(0.15, 0.45, (P, 2))
    act = np.ones((P, 2), bool)
    z = OM.model_sketch(t, alpha, act, hhat, T)
    n = np.full(P, 300)
    start = O.State(t + rng.uniform(-0.5, 0.5, (P, 2)), alpha * 0.9, act)
    L = OW.whitener(OW.covariance(start.t, start.alpha, act, hhat2, T, m))
    st, loss = OW.weighted_fit(z, n, start, hhat, L, T, 60)
    assert np.max(loss) < 1e-12
    np.testing.assert_allclose(np.mod(st.t - t + T / 2, T) - T / 2, 0, atol=1e-6)
    np.testing.assert_allclose(st.alpha, alpha, atol=1e-8)
