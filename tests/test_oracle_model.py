"""Pins of the model oracle: eq. (1), eq. (4), eq. (6) with W = I and its gradients."""
import numpy as np
import pytest

from oracle import model as OM
from oracle import sketch as OS


def test_golden_irf_spectrum(golden):
    for (T, m, o), h, expect in golden("irf_spectrum_small.txt"):
        np.testing.assert_allclose(OM.irf_spectrum(h, o, T, m), expect, atol=1e-15)


def test_delta_irf_and_symmetry():
    T, m = 256, 20
    np.testing.assert_allclose(OM.irf_spectrum([0, 0, 5.0, 0], 2, T, m), 1.0, atol=1e-15)
    h = np.exp(-0.5 * (np.arange(-40, 41) / 4.0) ** 2)
    hh = OM.irf_spectrum(h, 40, T, m)
    assert np.max(np.abs(hh.imag)) < 1e-14           # symmetric about its origin -> real
    assert np.all(np.abs(hh) <= 1.0 + 1e-15)
    assert OM.irf_sigma(h, 40) == pytest.approx(4.0, rel=1e-9)


def _mixture_pmf(T, h, o, t, alpha, alpha0):
    """pi(x) of eq. (1) on x = 0..T-1 for integer depths, impulse response wrapped mod T."""
    pi = np.full(T, alpha0 / T)
    h = np.asarray(h, dtype=np.float64) / np.sum(h)
    for tk, ak in zip(t, alpha):
        for i, hi in enumerate(h):
            pi[(tk + i - o) % T] += ak * hi
    return pi


@pytest.mark.parametrize("T,m", [(64, 31), (1024, 16), (4613, 10)])
def test_model_is_expected_sketch(T, m):
    """E z_l = sum_x pi(x) e^{i w_l x} equals Phi_l = hhat_l sum_k alpha_k e^{i w_l t_k}:
    the background term drops out at w_l = 2 pi l / T (eq. 4)."""
    rng = np.random.default_rng(T)
    h = rng.uniform(0, 1, 9)
    o = 3
    t = rng.integers(0, T, 3)
    alpha = np.array([0.3, 0.2, 0.1])
    pi = _mixture_pmf(T, h, o, t, alpha, 0.4)
    assert pi.sum() == pytest.approx(1.0)
    ez = np.array([np.sum(pi * np.exp(1j * 2 * np.pi * ell * np.arange(T) / T)) for ell in range(1, m + 1)])
    hhat = OM.irf_spectrum(h, o, T, m)
    phi = OM.model_sketch(t[None].astype(float), alpha[None], np.ones((1, 3), bool), hhat, T)[0]
    np.testing.assert_allclose(phi, ez, atol=1e-12)


def _rand_problem(rng, P=6, K=3, m=7, T=300):
    h = rng.uniform(0, 1, 11)
    hhat = OM.irf_spectrum(h, 5, T, m)
    t = rng.uniform(0, T, (P, K))
    alpha = rng.uniform(0.05, 0.3, (P, K))
    active = rng.uniform(size=(P, K)) < 0.8
    z = rng.normal(size=(P, m)) * 0.3 + 1j * rng.normal(size=(P, m)) * 0.3
    n = rng.integers(1, 1000, P)
    return z, n, t, alpha, active, hhat, T


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(7)
    z, n, t, alpha, active, hhat, T = _rand_problem(rng)
    gt, ga = OM.gradients(z, n, t, alpha, active, hhat, T)
    P, K = t.shape
    h = 1e-6
    for k in range(K):
        dt = np.zeros_like(t)
        dt[:, k] = h
        fd = (OM.loss(z, n, t + dt, alpha, active, hhat, T) - OM.loss(z, n, t - dt, alpha, active, hhat, T)) / (2 * h)
        np.testing.assert_allclose(gt[:, k], np.where(active[:, k], fd, 0.0), rtol=1e-6, atol=1e-6)
        da = np.zeros_like(alpha)
        da[:, k] = h
        fd = (OM.loss(z, n, t, alpha + da, active, hhat, T) - OM.loss(z, n, t, alpha - da, active, hhat, T)) / (2 * h)
        np.testing.assert_allclose(ga[:, k], np.where(active[:, k], fd, 0.0), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("T", [16, 64, 200])
def test_loss_parseval_identity(T):
    """At m = T/2 the sketched loss equals a histogram-domain quantity:
    n sum_{l=1}^{T/2} |z_l - Phi_l|^2 = (T ||D||^2 - (sum D)^2 + |sum_x D_x (-1)^x|^2) / (2n),
    D = y - n pi, with y the photon histogram and pi the mixture pmf of eq. (1)."""
    rng = np.random.default_rng(T)
    m = T // 2
    h = rng.uniform(0, 1, 5)
    o = 2
    t = rng.integers(0, T, 2)
    alpha = np.array([0.35, 0.25])
    x = rng.integers(0, T, 300)
    z, n = OS.sketch(x, np.array([0, x.size]), T, m)
    hhat = OM.irf_spectrum(h, o, T, m)
    L = OM.loss(z, n, t[None].astype(float), alpha[None], np.ones((1, 2), bool), hhat, T)[0]
    y = np.bincount(x, minlength=T).astype(float)
    D = y - n[0] * _mixture_pmf(T, h, o, t, alpha, 0.4)
    alt = (T * np.sum(D ** 2) - D.sum() ** 2 + np.sum(D * (-1.0) ** np.arange(T)) ** 2) / (2 * n[0])
    assert L == pytest.approx(alt, rel=1e-10)


def test_noiseless_fixed_point_and_m1_closed_form():
    rng = np.random.default_rng(8)
    T, m = 4096, 12
    h = np.exp(-0.5 * (np.arange(-30, 31) / 5.0) ** 2)
    hhat = OM.irf_spectrum(h, 30, T, m)
    t = np.array([[1234.567, 3001.25]])
    alpha = np.array([[0.4, 0.3]])
    act = np.ones((1, 2), bool)
    z = OM.model_sketch(t, alpha, act, hhat, T)
    gt, ga = OM.gradients(z, np.array([500]), t, alpha, act, hhat, T)
    assert np.max(np.abs(gt)) < 1e-9 and np.max(np.abs(ga)) < 1e-9
    # m = 1, one surface: t = (T / 2pi) arg(z_1 / hhat_1) mod T, alpha = |z_1| / |hhat_1|
    z1 = OM.model_sketch(t[:, :1], alpha[:, :1], act[:, :1], hhat[:1], T)[0, 0]
    r = z1 / hhat[0]
    assert (np.angle(r) * T / (2 * np.pi)) % T == pytest.approx(1234.567, abs=1e-9)
    assert abs(r) == pytest.approx(0.4, abs=1e-14)
