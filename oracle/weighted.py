"""Eq. (6) with the precision-matrix weighting W = Sigma_theta^{-1} (Section 2: the sketch is
asymptotically normal with covariance Sigma_theta / n, eq. (5), and the loss of eq. (6) may
weight the residual by a positive definite W, the precision matrix being the statistically
efficient choice), pixel by pixel.

Reading of Sigma: the covariance of the sketch's 2m real coordinates.  The sketch is a mean of
phi(x) = [cos w_l x, sin w_l x], l = 1..m, whose distribution is not circularly symmetric, so
the efficient weighting needs the covariance of the real and imaginary parts together; the
Hermitian m x m matrix E[(e - Psi)(e - Psi)^H] alone does not determine it (weighting by its
inverse alone was measured worse than W = I).  Expectations of products of harmonics are values
of the characteristic function at sums and differences of frequencies (eq. 4 at w_a +- w_b, with
Psi_0 = 1 and Psi_{-j} = conj(Psi_j)):
    E[cos_a cos_b] = Re(Psi_{a+b} + Psi_{a-b}) / 2,  E[sin_a sin_b] = Re(Psi_{a-b} - Psi_{a+b}) / 2,
    E[cos_a sin_b] = Im(Psi_{a+b} - Psi_{a-b}) / 2,   E[phi] = [Re Psi_l, Im Psi_l],
so Sigma needs the impulse-response spectrum up to harmonic 2m (and 2m < T).  A pixel with no
signal (alpha = 0) has Psi_j = 0 for 0 < j <= 2m and Sigma = I / 2: the weighting reduces to a
multiple of W = I.

Readings of what the paper leaves open (used identically by the HIP path):
  two steps   Sigma is evaluated at a first estimate theta_1 -- the pixelwise estimator with
              W = I (oracle.smle) -- and held fixed; the weighted loss
              L_W = n ||L^{-1} r||^2, r = [Re(z - Phi), Im(z - Phi)], L L^T = Sigma(theta_1), is
              then minimised from theta_1 (the classical two-step efficient estimator)
  ridge       Sigma + (1e-5 tr(Sigma) / (2m)) I, so that the factor exists when a pixel's
              photons are nearly deterministic in some harmonic
  minimiser   Levenberg-Marquardt on the whitened residual rw = L^{-1} r: the step solves
              (A + mu (diag A + 1e-12)) d = g with A = Jw^T Jw, g = Jw^T rw, Jw = L^{-1} J and J
              the real Jacobian of Phi in (t_k, alpha_k) over the active points; t wraps onto
              [0, T), alpha is projected onto {alpha >= 0, sum alpha <= 1}; a step is kept iff it
              lowers L_W (then mu / 10, floored at 1e-7), else mu * 10 (capped at 1e7); mu starts
              at 1e-3; inactive points stay fixed

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .model import irf_spectrum, model_sketch, unit_phasors
from .smle import smle
from .srt3d import Params, State, project_capped_simplex, wrap

RIDGE = 1e-5
MU0, MU_MIN, MU_MAX = 1e-3, 1e-7, 1e7


def covariance(t, alpha, active, hhat2, T: int, m: int) -> np.ndarray:
    """Sigma [P, 2m, 2m] of phi(x) under pi_theta; hhat2 holds hhat_1 .. hhat_2m."""
    assert hhat2.size >= 2 * m and 2 * m < T
    psi = model_sketch(t, alpha, active, hhat2[: 2 * m], T)           # Psi_1 .. Psi_2m
    P = psi.shape[0]
    full = np.concatenate([np.ones((P, 1), complex), psi], 1)          # Psi_0 .. Psi_2m

    def at(j):
        v = full[:, np.abs(j)]
        return np.where(j >= 0, v, np.conj(v))

    a = np.arange(1, m + 1)
    S = at(a[:, None] + a[None, :])                                    # Psi_{a+b}  [P, m, m]
    D = at(a[:, None] - a[None, :])                                    # Psi_{a-b}
    Ecc = 0.5 * (S + D).real
    Ess = 0.5 * (D - S).real
    Ecs = 0.5 * (S - D).imag                                           # Ecs[a, b] = E[cos_a sin_b]
    C = np.concatenate([np.concatenate([Ecc, Ecs], 2), np.concatenate([np.swapaxes(Ecs, 1, 2), Ess], 2)], 1)
    mu = np.concatenate([psi[:, :m].real, psi[:, :m].imag], 1)
    return C - mu[:, :, None] * mu[:, None, :]


def whitener(Sigma: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor L (L L^T) of the ridged Sigma."""
    d = Sigma.shape[-1]
    tr = np.trace(Sigma, axis1=1, axis2=2)
    return np.linalg.cholesky(Sigma + (RIDGE * tr / d)[:, None, None] * np.eye(d))


def residual_and_jacobian(z, t, alpha, active, hhat, T: int):
    """r = [Re(z - Phi), Im(z - Phi)] [P, 2m] and J = dPhi / d(t_1..t_K, alpha_1..alpha_K) in the
    same real layout [P, 2m, 2K] (zero columns for inactive points)."""
    m = hhat.size
    w = 2.0 * np.pi * np.arange(1, m + 1) / T
    g = hhat * unit_phasors(t, T, m)                                   # [P, K, m]
    a = np.where(active, alpha, 0.0)
    r = np.asarray(z) - np.einsum("pk,pkl->pl", a, g)
    dt = (a[..., None] * 1j * w) * g                                   # dPhi / dt_k
    da = np.where(active[..., None], g, 0.0)                           # dPhi / dalpha_k
    cols = np.concatenate([dt, da], 1)                                 # [P, 2K, m]
    J = np.concatenate([cols.real, cols.imag], 2).transpose(0, 2, 1)   # [P, 2m, 2K]
    return np.concatenate([r.real, r.imag], 1), J


def weighted_loss(z, n, st: State, hhat, L, T: int) -> np.ndarray:
    r, _ = residual_and_jacobian(z, st.t, st.alpha, st.active, hhat, T)
    rw = np.linalg.solve(L, r[..., None])[..., 0]
    return np.asarray(n, np.float64) * np.sum(rw * rw, 1)


def weighted_fit(z, n, st1: State, hhat, L, T: int, iters: int):
    """Levenberg-Marquardt on n ||L^{-1} r||^2 from st1.  Returns (state, loss)."""
    P, K = st1.t.shape
    st = st1.copy()
    loss = weighted_loss(z, n, st, hhat, L, T)
    mu = np.full(P, MU0)
    for _ in range(iters):
        r, J = residual_and_jacobian(z, st.t, st.alpha, st.active, hhat, T)
        rw = np.linalg.solve(L, r[..., None])[..., 0]
        Jw = np.linalg.solve(L, J)
        A = np.einsum("pia,pib->pab", Jw, Jw)
        g = np.einsum("pia,pi->pa", Jw, rw)
        dA = np.einsum("paa->pa", A)
        M = A + (mu[:, None] * (dA + 1e-12))[:, :, None] * np.eye(2 * K)
        d = np.linalg.solve(M, g[..., None])[..., 0]
        t_new = np.where(st.active, wrap(st.t + d[:, :K], T), st.t)
        a_new = project_capped_simplex(np.where(st.active, st.alpha + d[:, K:], 0.0), st.active)
        trial = State(t_new, a_new, st.active.copy())
        L_new = weighted_loss(z, n, trial, hhat, L, T)
        keep = L_new < loss
        st = State(np.where(keep[:, None], trial.t, st.t), np.where(keep[:, None], trial.alpha, st.alpha),
                   st.active.copy())
        loss = np.where(keep, L_new, loss)
        mu = np.where(keep, np.maximum(mu / 10, MU_MIN), np.minimum(mu * 10, MU_MAX))
    return st, loss


def smle_weighted(z, n, irf, origin: int, p: Params, starts: int, witers: int, iters=None):
    """The W = I pixelwise estimate, then eq. (6) with W = Sigma(theta_1)^{-1}.  Returns
    dict(state, loss (weighted), first (the W = I result), L (whitening factors), hhat)."""
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n, dtype=np.int64)
    first = smle(z, n, irf, origin, p, starts, iters)
    st1 = first["state"]
    hhat = irf_spectrum(irf, origin, p.T, p.m)
    hhat2 = irf_spectrum(irf, origin, p.T, 2 * p.m)
    L = whitener(covariance(st1.t, st1.alpha, st1.active, hhat2, p.T, p.m))
    st, loss = weighted_fit(z, n, st1, hhat, L, p.T, witers)
    return dict(state=st, loss=loss, first=first, L=L, hhat=hhat)


__all__ = ["covariance", "whitener", "residual_and_jacobian", "weighted_loss", "weighted_fit", "smle_weighted"]
