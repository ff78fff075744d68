"""Pixelwise sketched estimator (SMLE), the comparison system of Sections 1 and 4: each pixel's
sketched loss (eq. 6 with W = I) minimised on its own, with no spatial prior -- SRT3D with the
denoisers turned off -- from several starting points, keeping the start with the lowest loss.

Readings of what the paper leaves open (used identically by the HIP path):
  starts      start 0 is the SRT3D initialisation (greedy sketched matched filter); start
              s = 1..S-1 puts point k at t_k = (s T / S + k T / K) mod T with the single-atom
              least-squares amplitude a_k = max(0, Re sum_l conj(hhat_l e^{i w_l t_k}) z_l /
              sum_l |hhat_l|^2), alpha = the projection of a onto {alpha >= 0, sum alpha <= 1},
              and every point active where n > 0
  steps       per pixel: the SRT3D data step with the pixel's own n in the Lipschitz bounds, so
              every pixel moves at the rate of a pixel with n photons in SRT3D's per-frame steps
              (gamma_t = eta_t / (2 sum w^2 |hhat|^2), gamma_a = eta_a / (2 K sum |hhat|^2) on
              the loss divided by n); points are never removed
  selection   the lowest loss n ||Phi - z||^2 after `iters` steps, the earliest start on ties

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .model import irf_spectrum, loss, omega, unit_phasors
from .srt3d import Params, State, data_step, init_points, project_capped_simplex


def start_points(z, n, hhat, p: Params, s: int, S: int, init: State) -> State:
    """Start s of S (see the module docstring); start 0 is `init`."""
    if s == 0:
        return init.copy()
    T, K = p.T, p.K_max
    P = z.shape[0]
    k = np.arange(K, dtype=np.float64)
    t = np.mod(s * T / S + k * T / K, T)
    t = np.broadcast_to(t, (P, K)).copy()
    e2 = float(np.sum(np.abs(hhat) ** 2))
    g = hhat * unit_phasors(t, T, p.m)                          # [P, K, m]
    c = (np.conj(g) * np.asarray(z)[:, None, :]).sum(-1).real
    a = np.maximum(0.0, c / e2)
    active = np.broadcast_to((np.asarray(n) > 0)[:, None], (P, K)).copy()
    alpha = project_capped_simplex(a, active)
    return State(t, np.where(active, alpha, 0.0), active)


def unit_steps(hhat, p: Params):
    """Steps on the loss divided by n: the SRT3D bounds with n_max = 1."""
    e2 = float(np.sum(np.abs(hhat) ** 2))
    et = float(np.sum(omega(p.T, p.m) ** 2 * np.abs(hhat) ** 2))
    return p.eta_t / (2.0 * et), p.eta_a / (2.0 * p.K_max * e2)


def descend(st: State, z, n, hhat, p: Params, iters: int) -> State:
    """`iters` data steps with per-pixel steps (the gradient of the loss / n)."""
    gam_t, gam_a = unit_steps(hhat, p)
    unit_n = (np.asarray(n) > 0).astype(np.float64)
    for _ in range(iters):
        st = data_step(st, z, unit_n, hhat, p, gam_t, gam_a)
    return st


def smle(z, n, irf, origin: int, p: Params, starts: int, iters=None):
    """Returns dict(state, loss [P], start [P] index of the chosen start, losses [S, P])."""
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n, dtype=np.int64)
    hhat = irf_spectrum(irf, origin, p.T, p.m)
    iters = p.iters if iters is None else iters
    init = init_points(z, n, hhat, p)
    best, best_loss, best_s, losses = None, None, None, []
    for s in range(starts):
        st = descend(start_points(z, n, hhat, p, s, starts, init), z, n, hhat, p, iters)
        L = loss(z, n, st.t, st.alpha, st.active, hhat, p.T)
        losses.append(L)
        if best is None:
            best, best_loss, best_s = st, L, np.zeros(L.shape, np.int64)
            continue
        take = L < best_loss
        best = State(np.where(take[:, None], st.t, best.t), np.where(take[:, None], st.alpha, best.alpha),
                     np.where(take[:, None], st.active, best.active))
        best_loss = np.where(take, L, best_loss)
        best_s = np.where(take, s, best_s)
    return dict(state=best, loss=best_loss, start=best_s, losses=np.array(losses), hhat=hhat)


__all__ = ["start_points", "unit_steps", "descend", "smle"]
