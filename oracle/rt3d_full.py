"""Full-data RT3D: the per-photon likelihood that SRT3D replaces (Section 3), on tiny frames.

Section 3 contrasts SRT3D's sketched data term (eq. 8) with RT3D's, which uses every photon
through the likelihood of eq. (1) and so costs time in proportion to the photon count; Section 4
reports reconstructions of similar quality.  This module keeps everything of the SRT3D oracle
except the data term -- the initialisation, the depth and intensity denoisers, the background,
the output and the order of the steps are `oracle.srt3d`'s -- and takes the data step on the
negative log-likelihood of each pixel's full ToA histogram instead.  It is a quality reference,
not a parity target: the two losses differ, so the two reconstructions are compared with the
synthetic truth, not with each other.

Data term (eq. 1, histogram of eq. 2 with unit bins).  The photons of a pixel are i.i.d. on the
bins x = 0..T-1 with pmf
    pi_x = sum_k alpha_k h~(x - t_k) + alpha_0 / T,     alpha_0 = 1 - sum_k alpha_k,
h~ = h / sum h.  With mu_x = n pi_x (surface counts r_k = n alpha_k, background b = n alpha_0 / T)
the Poisson negative log-likelihood of the histogram y is
    L = sum_x [mu_x - y_x log mu_x] = n - n log n - sum_x y_x log pi_x,
because sum_x mu_x = n for every theta.  `nll` evaluates it on the dense histogram (every bin),
the brute-force form; the iteration uses the same sum restricted to the non-empty bins
(`Photons`), which the tests pin against the dense form.

Readings (the paper does not describe RT3D's data step):
  - h at a non-integer lag is the linear interpolation between its integer lags; lags are
    circular with period T (stamps are folded mod T, as for the sketch).
  - The data step is a gradient step on the depths, then a projected gradient step on alpha onto
    {alpha >= 0, sum alpha <= 1}, as SRT3D's; the step size is found per pixel by backtracking
    (halving from twice the pixel's last accepted step until the quadratic upper-bound condition
    L(x+) <= L(x) + g.(x+ - x) + |x+ - x|^2 / (2 gamma) holds; no move after 40 halvings).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from .model import irf_spectrum
from .srt3d import (Params, State, background, circ_diff, default_tau_z, depth_denoise, init_points,
                    intensity_denoise, output, project_capped_simplex, wrap)

MAX_HALVINGS = 40
START_STEP_T = 1.0      # first trial step of a pixel's depth update (bins^2 per unit of L)
START_STEP_A = 1e-3     # first trial step of a pixel's alpha update


def irf_at(h, origin: int, u):
    """h~(u) = h(u) / sum h at real lags u (linear interpolation of the integer lags, zero outside
    the support), and its derivative dh~/du on the interval containing u."""
    h = np.asarray(h, dtype=np.float64) / float(np.sum(h))
    u = np.asarray(u, dtype=np.float64)
    u0 = np.floor(u)
    f = u - u0
    i0 = u0.astype(np.int64) + origin
    pad = np.concatenate([[0.0], h, [0.0]])               # index j + 1 holds lag j - origin
    lo = pad[np.clip(i0 + 1, 0, h.size + 1)]
    hi = pad[np.clip(i0 + 2, 0, h.size + 1)]
    inside_lo = (i0 >= 0) & (i0 < h.size)
    inside_hi = (i0 + 1 >= 0) & (i0 + 1 < h.size)
    lo = np.where(inside_lo, lo, 0.0)
    hi = np.where(inside_hi, hi, 0.0)
    return (1.0 - f) * lo + f * hi, hi - lo


def pmf(t, alpha, active, h, origin: int, T: int):
    """pi[p, x] of eq. (1) on every bin, with the per-surface shapes H[p, k, x] = h~(x - t_k) and
    their derivatives dH/dt_k = -h~'(x - t_k)."""
    x = np.arange(T, dtype=np.float64)
    u = circ_diff(x[None, None, :] - np.asarray(t, dtype=np.float64)[:, :, None], T)
    H, dH = irf_at(h, origin, u)
    a = np.where(active, alpha, 0.0)
    a0 = 1.0 - a.sum(1)
    pi = np.einsum("pk,pkx->px", a, H) + a0[:, None] / T
    return pi, H, -dH


def nll(y, n, t, alpha, active, h, origin: int, T: int):
    """Per-pixel Poisson negative log-likelihood sum_x [mu_x - y_x log mu_x], mu = n pi (bins
    with y_x = 0 contribute mu_x only)."""
    y = np.asarray(y, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    pi, _, _ = pmf(t, alpha, active, h, origin, T)
    mu = n[:, None] * pi
    ylog = np.where(y > 0, y * np.log(np.where(mu > 0, mu, 1.0)), 0.0)
    return mu.sum(1) - ylog.sum(1)


def nll_gradients(y, n, t, alpha, active, h, origin: int, T: int):
    """dL/dt_k = -sum_x y_x alpha_k dH_kx/dt_k / pi_x;  dL/dalpha_k = -sum_x y_x (H_kx - 1/T) / pi_x.
    (The mu_x term contributes nothing: sum_x pi_x = 1 for every theta.)  Inactive points get 0."""
    y = np.asarray(y, dtype=np.float64)
    pi, H, dHdt = pmf(t, alpha, active, h, origin, T)
    w = np.where(y > 0, y / np.where(pi > 0, pi, 1.0), 0.0)          # y_x / pi_x
    gt = -np.asarray(alpha, dtype=np.float64) * np.einsum("px,pkx->pk", w, dHdt)
    ga = -np.einsum("px,pkx->pk", w, H - 1.0 / T)
    return np.where(active, gt, 0.0), np.where(active, ga, 0.0)


class Photons:
    """The non-empty bins of each pixel's histogram: pixel index, bin and count per entry.  The
    likelihood only needs pi at these bins, because sum_x mu_x = n for every theta."""

    def __init__(self, y):
        y = np.asarray(y, dtype=np.float64)
        self.P = y.shape[0]
        self.pix, self.x = np.nonzero(y)
        self.cnt = y[self.pix, self.x]
        self.n = y.sum(1)

    def pi(self, t, alpha, active, h, origin: int, T: int):
        """pi at the non-empty bins, the shapes H[e, k] and dH/dt_k there."""
        t = np.asarray(t, dtype=np.float64)[self.pix]
        a = np.where(active, alpha, 0.0)[self.pix]
        u = circ_diff(self.x[:, None] - t, T)
        H, dH = irf_at(h, origin, u)
        return (a * H).sum(1) + (1.0 - a.sum(1)) / T, H, -dH

    def nll(self, t, alpha, active, h, origin: int, T: int):
        """Per pixel n - sum_x y_x log(n pi_x): the Poisson NLL of `nll` on the non-empty bins."""
        pi, _, _ = self.pi(t, alpha, active, h, origin, T)
        mu = self.n[self.pix] * pi
        term = self.cnt * np.log(np.where(mu > 0, mu, 1.0))
        return self.n - np.bincount(self.pix, weights=term, minlength=self.P)

    def gradients(self, t, alpha, active, h, origin: int, T: int):
        """`nll_gradients` on the non-empty bins."""
        pi, H, dHdt = self.pi(t, alpha, active, h, origin, T)
        w = self.cnt / np.where(pi > 0, pi, 1.0)
        K = np.shape(t)[1]
        gt = np.zeros((self.P, K))
        ga = np.zeros((self.P, K))
        for k in range(K):
            gt[:, k] = -np.bincount(self.pix, weights=w * dHdt[:, k], minlength=self.P)
            ga[:, k] = -np.bincount(self.pix, weights=w * (H[:, k] - 1.0 / T), minlength=self.P)
        gt *= np.asarray(alpha, dtype=np.float64)
        return np.where(active, gt, 0.0), np.where(active, ga, 0.0)


def _backtrack(ph: Photons, st: State, h, origin, T, gam, which: str):
    """One projected gradient step per pixel on `which` ('t' or 'alpha') with backtracking."""
    L0 = ph.nll(st.t, st.alpha, st.active, h, origin, T)
    gt, ga = ph.gradients(st.t, st.alpha, st.active, h, origin, T)
    g = gt if which == "t" else ga
    gam = gam.copy()
    done = ~st.active.any(1) | (np.abs(g).sum(1) == 0)
    t_new, a_new = st.t.copy(), st.alpha.copy()
    for _ in range(MAX_HALVINGS):
        todo = ~done
        if not todo.any():
            break
        if which == "t":
            cand_t = np.where(st.active, wrap(st.t - gam[:, None] * g, T), st.t)
            cand_a = st.alpha
            step = np.where(st.active, -gam[:, None] * g, 0.0)       # L is T-periodic in t: unwrapped
        else:
            cand_t = st.t
            cand_a = project_capped_simplex(np.where(st.active, st.alpha - gam[:, None] * g, 0.0), st.active)
            step = cand_a - st.alpha
        L1 = ph.nll(cand_t, cand_a, st.active, h, origin, T)
        bound = L0 + (g * step).sum(1) + (step ** 2).sum(1) / (2.0 * gam)
        ok = todo & (L1 <= bound)
        t_new[ok] = cand_t[ok]
        a_new[ok] = cand_a[ok]
        done |= ok
        gam = np.where(todo & ~ok, gam * 0.5, gam)
    gam = np.where(done, gam, gam * 2.0 ** MAX_HALVINGS)     # a pixel that never passed keeps its step
    return State(t_new, a_new, st.active.copy()), gam


def data_step(st: State, ph: Photons, h, origin: int, p: Params, gam_t, gam_a):
    """Depth step, then alpha step at the new depths (each with per-pixel backtracking); returns
    the new state and the accepted step sizes."""
    st, gam_t = _backtrack(ph, st, h, origin, p.T, gam_t, "t")
    st, gam_a = _backtrack(ph, st, h, origin, p.T, gam_a, "alpha")
    return State(st.t, project_capped_simplex(st.alpha, st.active), st.active), gam_t, gam_a


def reconstruct(y, z, n, irf, origin: int, rows: int, cols: int, p: Params, iters=None):
    """Full-data RT3D: SRT3D's initialisation from the sketch z of the same photons, then
    `iters` x (full-data step, depth denoiser, intensity denoiser), background and output."""
    ph = Photons(y)
    n = np.asarray(n, dtype=np.int64)
    if not np.array_equal(ph.n, n):
        raise ValueError("photon counts of the histogram and of the sketch differ")
    hhat = irf_spectrum(irf, origin, p.T, p.m)
    tau_z = default_tau_z(irf, origin, p)
    st = init_points(z, n, hhat, p)
    P = st.t.shape[0]
    gam_t = np.full(P, START_STEP_T)
    gam_a = np.full(P, START_STEP_A)
    for _ in range(p.iters if iters is None else iters):
        st, gam_t, gam_a = data_step(st, ph, irf, origin, p, gam_t * 2.0, gam_a * 2.0)
        st = depth_denoise(st, rows, cols, p, tau_z)
        st = intensity_denoise(st, n, rows, cols, p, tau_z)
    depth, inten, act = output(st, n)
    return dict(depth=depth, intensity=inten, active=act, bg=background(st, n, rows, cols, p), state=st)


__all__ = ["irf_at", "pmf", "nll", "nll_gradients", "Photons", "data_step", "reconstruct"]
