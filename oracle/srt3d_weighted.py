"""SRT3D with the precision weighting inside its data step: eq. (8) with a per-pixel W.

Section 2 allows any positive definite W in the sketched loss of eq. (6) and names the precision
matrix W = Sigma_theta^{-1} (eq. 5) as the statistically efficient choice; Section 3's SRT3D
takes W = I.  This module is the SRT3D iteration of `oracle.srt3d` with only the data step
changed: its loss is n e^T W e, with e = [Re(Phi - z), Im(Phi - z)] the sketch residual in the
2m real coordinates of `oracle.weighted` and W_p = Sigma(theta_0)^{-1} for each pixel.

Readings (the paper gives no algorithm for a weighted SRT3D):
  weights     W_p is the inverse of the ridged covariance of `oracle.weighted` (reading 20-21 of
              the pixelwise weighted estimator) evaluated at the SRT3D initialisation theta_0 of
              the pixel and held fixed through the iterations (a two-step weighting)
  gradient    dL/dtheta = 2 n J^T W e, J = dPhi/d(t, alpha) in the same real layout; with W = I
              it is the W = I gradient of `oracle.model.gradients`
  step sizes  the W = I Lipschitz steps (reading 10) with n_max replaced by
              n_w = max_p n_p G_p, G_p = max_i sum_j |W_p,ij| (Gershgorin, >= the largest
              eigenvalue of W_p and equal to c for W_p = c I): the weighted data term's block
              Lipschitz constants are at most G_p times the unweighted ones
  the rest    data step order (t, then alpha at the new t, projection), denoisers, background and
              output are SRT3D's; with every W_p = c I the iteration is exactly SRT3D's

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .model import irf_spectrum
from .srt3d import (Params, State, background, default_tau_z, depth_denoise, init_points, intensity_denoise,
                    output, project_capped_simplex, step_sizes, wrap)
from .weighted import covariance, residual_and_jacobian, whitener


def weight_matrices(st0: State, hhat2, p: Params) -> np.ndarray:
    """W_p = (ridged Sigma(theta_0))^{-1} [P, 2m, 2m], through its Cholesky factor."""
    L = whitener(covariance(st0.t, st0.alpha, st0.active, hhat2, p.T, p.m))
    Linv = np.linalg.inv(L)
    return np.einsum("pki,pkj->pij", Linv, Linv)


def gershgorin(W) -> np.ndarray:
    """Per pixel max_i sum_j |W_ij|, an upper bound of the largest eigenvalue of W."""
    return np.abs(W).sum(2).max(1)


def weighted_step_sizes(n, hhat, W, p: Params):
    """The W = I steps with n_max replaced by n_w = max_p n_p G_p."""
    n = np.asarray(n, dtype=np.float64)
    n_w = float(np.max(n * gershgorin(W))) if n.size else 0.0
    if n_w <= 0:
        return 0.0, 0.0
    gt, ga = step_sizes(n, hhat, p)
    n_max = float(np.max(n))
    return gt * n_max / n_w, ga * n_max / n_w


def weighted_loss(z, n, t, alpha, active, hhat, W, T: int) -> np.ndarray:
    """n e^T W e per pixel, e = [Re(Phi - z), Im(Phi - z)]."""
    r, _ = residual_and_jacobian(z, t, alpha, active, hhat, T)          # r = z - Phi
    return np.asarray(n, np.float64) * np.einsum("pi,pij,pj->p", r, W, r)


def weighted_gradients(z, n, t, alpha, active, hhat, W, T: int):
    """(dL/dt, dL/dalpha) [P, K] of n e^T W e: 2 n J^T W e, zero for inactive points."""
    r, J = residual_and_jacobian(z, t, alpha, active, hhat, T)
    v = np.einsum("pij,pj->pi", W, -r)                                   # W e
    g = 2.0 * np.asarray(n, np.float64)[:, None] * np.einsum("pic,pi->pc", J, v)
    K = np.shape(t)[1]
    return np.where(active, g[:, :K], 0.0), np.where(active, g[:, K:], 0.0)


def data_step_weighted(st: State, z, n, hhat, W, p: Params, gam_t: float, gam_a: float) -> State:
    """t <- t - gam_t dL/dt; then alpha <- proj(alpha - gam_a dL/dalpha) at the new t."""
    gt, _ = weighted_gradients(z, n, st.t, st.alpha, st.active, hhat, W, p.T)
    t = np.where(st.active, wrap(st.t - gam_t * gt, p.T), st.t)
    _, ga = weighted_gradients(z, n, t, st.alpha, st.active, hhat, W, p.T)
    a = np.where(st.active, st.alpha - gam_a * ga, st.alpha)
    return State(t, project_capped_simplex(a, st.active), st.active.copy())


def iterate_weighted(st: State, z, n, hhat, W, rows, cols, p: Params, tau_z: float, iters: int) -> State:
    """`iters` x (weighted data step, depth denoiser, intensity denoiser)."""
    gam_t, gam_a = weighted_step_sizes(n, hhat, W, p)
    for _ in range(iters):
        st = data_step_weighted(st, z, n, hhat, W, p, gam_t, gam_a)
        st = depth_denoise(st, rows, cols, p, tau_z)
        st = intensity_denoise(st, n, rows, cols, p, tau_z)
    return st


def reconstruct_weighted(z, n, irf, origin: int, rows: int, cols: int, p: Params, iters=None):
    """Initialisation, W_p at it, `iters` weighted iterations, background and output."""
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n, dtype=np.int64)
    hhat = irf_spectrum(irf, origin, p.T, p.m)
    hhat2 = irf_spectrum(irf, origin, p.T, 2 * p.m)
    tau_z = default_tau_z(irf, origin, p)
    st0 = init_points(z, n, hhat, p)
    W = weight_matrices(st0, hhat2, p)
    st = iterate_weighted(st0, z, n, hhat, W, rows, cols, p, tau_z, p.iters if iters is None else iters)
    depth, inten, act = output(st, n)
    return dict(depth=depth, intensity=inten, active=act, bg=background(st, n, rows, cols, p), state=st,
                init=st0, W=W, hhat=hhat, tau_z=tau_z)


__all__ = ["weight_matrices", "gershgorin", "weighted_step_sizes", "weighted_loss", "weighted_gradients",
           "data_step_weighted", "iterate_weighted", "reconstruct_weighted"]
