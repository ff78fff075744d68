"""Observation model, its characteristic function and the sketched loss.

Section 2, eq. (1): a photon comes from surface k with probability alpha_k
(stamp distribution h(x - t_k)/H, H = sum h) or from the background with
probability alpha_0 (uniform on {0..T-1}), sum_{k=0..K} alpha_k = 1.

Eq. (4): the characteristic function sampled at w_l is
  Psi_l = sum_k alpha_k * hhat_l * exp(i w_l t_k) + alpha_0 * (background CF).
With w_l = 2*pi*l/T and 1 <= l <= T-1 the background term vanishes (the sum of
exp(i w_l x) over x = 0..T-1 is zero), so the model sketch is
  Phi_l = hhat_l * sum_k alpha_k exp(i w_l t_k).
Readings: the exponent of eq. (4) carries t_k (one term per surface); hhat is
the impulse-response transform normalised by H (so that pi_s = h/H has hhat at
w = 0 equal to 1); h is indexed by lag i - o with an explicit origin o.

Eq. (6) with W = I and the weight n of eq. (8): L = n * sum_l |Phi_l - z_l|^2.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np


def omega(T: int, m: int) -> np.ndarray:
    """w_l = 2*pi*l/T for l = 1..m (Section 2, sampling scheme)."""
    return 2.0 * np.pi * np.arange(1, m + 1, dtype=np.float64) / T


def irf_spectrum(h, origin: int, T: int, m: int) -> np.ndarray:
    """hhat_l = sum_i h_i exp(i w_l (i - origin)) / sum_i h_i, l = 1..m, exact phases."""
    h = np.asarray(h, dtype=np.float64)
    lag = np.arange(h.size, dtype=np.int64) - origin
    ell = np.arange(1, m + 1, dtype=np.int64)
    k = np.mod(ell[:, None] * lag[None, :], T)
    return (np.exp(1j * 2.0 * np.pi * k / T) @ h) / h.sum()


def irf_sigma(h, origin: int) -> float:
    """Standard deviation (bins) of the normalised impulse response."""
    h = np.asarray(h, dtype=np.float64)
    lag = np.arange(h.size, dtype=np.float64) - origin
    H = h.sum()
    mu = (h * lag).sum() / H
    return float(np.sqrt((h * (lag - mu) ** 2).sum() / H))


def unit_phasors(t, T: int, m: int) -> np.ndarray:
    """exp(i w_l t) for every entry of t: shape t.shape + (m,); phase reduced mod T."""
    t = np.asarray(t, dtype=np.float64)
    ell = np.arange(1, m + 1, dtype=np.float64)
    ph = np.mod(t[..., None] * ell, T)
    return np.exp(1j * 2.0 * np.pi * ph / T)


def atoms(t, hhat, T: int) -> np.ndarray:
    """g[..., k, l] = hhat_l * exp(i w_l t_k)."""
    return hhat * unit_phasors(t, T, hhat.size)


def model_sketch(t, alpha, active, hhat, T: int) -> np.ndarray:
    """Phi[p, l] = hhat_l * sum over active k of alpha_k exp(i w_l t_k)  (eq. 4)."""
    a = np.where(active, alpha, 0.0)
    return np.einsum("pk,pkl->pl", a, atoms(t, hhat, T))


def loss(z, n, t, alpha, active, hhat, T: int) -> np.ndarray:
    """Per-pixel sketched loss n * ||Phi - z||^2 (eq. 6 with W = I, weight of eq. 8)."""
    e = model_sketch(t, alpha, active, hhat, T) - z
    return np.asarray(n, dtype=np.float64) * (np.abs(e) ** 2).sum(-1)


def gradients(z, n, t, alpha, active, hhat, T: int):
    """dL/dt_k = -2 n alpha_k sum_l w_l Im(conj(e_l) g_lk);  dL/dalpha_k = 2 n sum_l Re(conj(e_l) g_lk).

    Inactive points get zero gradients.
    """
    m = hhat.size
    g = atoms(t, hhat, T)
    e = np.einsum("pk,pkl->pl", np.where(active, alpha, 0.0), g) - z
    ce = np.conj(e)[:, None, :] * g
    n = np.asarray(n, dtype=np.float64)[:, None]
    gt = -2.0 * n * alpha * (ce.imag * omega(T, m)).sum(-1)
    ga = 2.0 * n * ce.real.sum(-1)
    return np.where(active, gt, 0.0), np.where(active, ga, 0.0)
