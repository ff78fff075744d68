"""Sketched RT3D (SRT3D), Section 3: eq. (8) with W = I, solved RT3D-style.

Eq. (8) minimises sum_ij n_ij ||z_ij - Psi(theta_ij)||^2 + rho(theta).  RT3D
(cited in Section 3, not described in the paper) handles rho with
plug-and-play point-cloud denoisers between gradient steps on the data term.
The paper fixes the data term; everything else below is a reading of what it
leaves open, chosen once and used identically by the HIP path:

  init        sketched matched filter on a grid, greedy pursuit over K_max points
  step sizes  per-frame Lipschitz bounds, so n_ij sets the data/prior balance
  data step   gradient step on depths, then on intensities, then a projection
              of alpha onto {alpha >= 0, sum alpha <= 1} (eq. (1) constraint)
  depth       weighted least-squares height-field fit over a gated window
  intensity   gated weighted mean of photon counts n*alpha, threshold r_min
  background  alpha_0 = 1 - sum alpha (eq. 1), b = n alpha_0 / T, box filter
  output      per-pixel points sorted by depth, inactive slots last
  merge/birth optional, every `birth_every` iterations (RT3D's split and merge of points, not
              described in the paper): points closer than T/(2m) merge; a free slot takes the
              residual's matched-filter peak when it carries at least r_min photons

Depths are in bins on the circle [0, T) (the sketch is periodic in t).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

from .model import atoms, gradients, irf_sigma, irf_spectrum, omega, unit_phasors

CHOL_EPS = 1e-5       # a Cholesky pivot <= CHOL_EPS * trace(M) counts as singular


@dataclass(frozen=True)
class Params:
    T: int
    m: int
    K_max: int = 1
    iters: int = 50
    R: int = 2             # denoiser window radius in pixels
    Rb: int = 1            # background box-filter radius
    init_stride: int = 0   # grid spacing of the initial search; 0 = max(1, T // (8 m))
    eta_t: float = 1.0     # depth step scale
    eta_a: float = 1.0     # intensity step scale
    lambda_z: float = 1.0  # relaxation of the depth denoiser
    tau_z: float = 0.0     # depth gate in bins; 0 = 3 * sigma of the impulse response
    r_min: float = 1.0     # photons below which a point is removed
    birth_every: int = 0   # iterations between merge/birth stages; 0 = none

    @property
    def stride(self) -> int:
        return self.init_stride if self.init_stride > 0 else max(1, self.T // (8 * self.m))


@dataclass
class State:
    t: np.ndarray        # [P, K] float64 depth in bins, [0, T)
    alpha: np.ndarray    # [P, K] float64 probability of each surface (eq. 1)
    active: np.ndarray   # [P, K] bool

    def copy(self) -> "State":
        return State(self.t.copy(), self.alpha.copy(), self.active.copy())


def wrap(t, T: int):
    """Map depths onto [0, T)."""
    r = np.mod(t, T)
    return np.where(r >= T, r - T, r)


def circ_diff(d, T: int):
    """Signed circular difference in (-T/2, T/2]."""
    r = wrap(d, T)
    return np.where(r > T / 2, r - T, r)


# ---------------------------------------------------------------------------
# constraint set of eq. (1): alpha_k >= 0, sum_k alpha_k <= 1 (alpha_0 = rest)
# ---------------------------------------------------------------------------
def project_capped_simplex(v, active):
    """Euclidean projection of each row's active entries onto {a >= 0, sum a <= 1}.

    Clamping at zero is the projection when the clamped sum is <= 1; otherwise
    the sum constraint is tight and the projection is onto the unit simplex,
    found by the sort-and-threshold rule.  Inactive entries are returned as 0.
    """
    v = np.asarray(v, dtype=np.float64)
    active = np.asarray(active, dtype=bool)
    clamped = np.where(active, np.maximum(v, 0.0), 0.0)
    over = clamped.sum(1) > 1.0
    if not over.any():
        return clamped
    K = v.shape[1]
    u = np.where(active, v, -np.inf)
    u = -np.sort(-u, axis=1)                    # descending
    cs = np.cumsum(np.where(np.isfinite(u), u, 0.0), axis=1)
    j = np.arange(1, K + 1, dtype=np.float64)
    cond = np.isfinite(u) & (u - (cs - 1.0) / j > 0.0)
    rho = K - np.argmax(cond[:, ::-1], axis=1)  # last index where cond holds (1-based)
    theta = (cs[np.arange(v.shape[0]), rho - 1] - 1.0) / rho
    simplex = np.where(active, np.maximum(v - theta[:, None], 0.0), 0.0)
    return np.where(over[:, None], simplex, clamped)


# ---------------------------------------------------------------------------
# step sizes
# ---------------------------------------------------------------------------
def step_sizes(n, hhat, p: Params):
    """Per-frame steps from Lipschitz bounds of the data term of eq. (8).

    d2L/dt_k^2 <= 2 n sum_l w_l^2 |hhat_l|^2 (alpha_k <= 1) and the alpha-block
    Hessian norm <= 2 n K sum_l |hhat_l|^2; both use the frame's largest n, so a
    pixel with fewer photons moves less per step and the denoisers weigh more.
    """
    n_max = float(np.max(n)) if np.size(n) else 0.0
    if n_max <= 0:
        return 0.0, 0.0
    e2 = float(np.sum(np.abs(hhat) ** 2))
    et = float(np.sum(omega(p.T, p.m) ** 2 * np.abs(hhat) ** 2))
    return p.eta_t / (2.0 * n_max * et), p.eta_a / (2.0 * n_max * p.K_max * e2)


# ---------------------------------------------------------------------------
# initialisation
# ---------------------------------------------------------------------------
def init_points(z, n, hhat, p: Params) -> State:
    """Greedy sketched matched filter.

    c(tau) = Re sum_l conj(hhat_l) w_l exp(-i w_l tau) on the grid tau = 0, s, 2s, ...
    For k = 1..K_max: take the grid maximum (lowest tau on ties) among points at
    circular distance >= T/m from earlier picks, a_k = max(0, c / sum|hhat|^2)
    (the least-squares amplitude of one atom), and remove a_k * hhat * exp(i w tau)
    from the working sketch w (initially z).  Then alpha = projection of a onto the
    constraint set; a point is active iff n * alpha >= r_min.
    """
    T, m, K = p.T, p.m, p.K_max
    z = np.asarray(z, dtype=np.complex128)
    n = np.asarray(n, dtype=np.int64)
    P = z.shape[0]
    s = p.stride
    G = -(-T // s)
    tau = np.arange(G, dtype=np.int64) * s
    ell = np.arange(1, m + 1, dtype=np.int64)
    Eg = np.exp(-1j * 2.0 * np.pi * np.mod(tau[:, None] * ell[None, :], T) / T)   # [G, m]
    e2 = float(np.sum(np.abs(hhat) ** 2))
    w = z.copy()
    picked = np.zeros((P, K), dtype=np.int64)
    amp = np.zeros((P, K))
    excluded = np.zeros((P, G), dtype=bool)
    rows = np.arange(P)
    for k in range(K):
        c = ((np.conj(hhat) * w) @ Eg.T).real
        c = np.where(excluded, -np.inf, c)
        g = np.argmax(c, axis=1)
        a = np.maximum(0.0, c[rows, g] / e2)
        picked[:, k] = tau[g]
        amp[:, k] = a
        w = w - a[:, None] * hhat * np.exp(1j * 2.0 * np.pi * np.mod(tau[g][:, None] * ell, T) / T)
        d = np.abs(tau[None, :] - tau[g][:, None])
        d = np.minimum(d, T - d)
        excluded |= d * m < T
    alpha = project_capped_simplex(amp, np.ones((P, K), dtype=bool))
    active = (n[:, None] * alpha >= p.r_min) & (n[:, None] > 0)
    return State(picked.astype(np.float64), np.where(active, alpha, 0.0), active)


# ---------------------------------------------------------------------------
# data step on eq. (8), W = I
# ---------------------------------------------------------------------------
def data_step(st: State, z, n, hhat, p: Params, gam_t: float, gam_a: float) -> State:
    """t <- t - gam_t dL/dt; then alpha <- proj(alpha - gam_a dL/dalpha) at the new t."""
    gt, _ = gradients(z, n, st.t, st.alpha, st.active, hhat, p.T)
    t = np.where(st.active, wrap(st.t - gam_t * gt, p.T), st.t)
    _, ga = gradients(z, n, t, st.alpha, st.active, hhat, p.T)
    a = np.where(st.active, st.alpha - gam_a * ga, st.alpha)
    return State(t, project_capped_simplex(a, st.active), st.active.copy())


# ---------------------------------------------------------------------------
# neighbourhoods for the denoisers
# ---------------------------------------------------------------------------
def window_weight(di: int, dj: int, R: int) -> float:
    """Compactly supported spatial weight (1 - r^2/(R+1)^2)^4."""
    return (1.0 - (di * di + dj * dj) / float((R + 1) ** 2)) ** 4


def _shift(a, di, dj, fill):
    """out[i, j] = a[i + di, j + dj] where in frame, else `fill`."""
    rows, cols = a.shape[:2]
    out = np.full_like(a, fill)
    i0, i1 = max(0, -di), min(rows, rows - di)
    j0, j1 = max(0, -dj), min(cols, cols - dj)
    if i0 < i1 and j0 < j1:
        out[i0:i1, j0:j1] = a[i0 + di:i1 + di, j0 + dj:j1 + dj]
    return out


def _gated_pairs(t, act, rows, cols, R, tau_z, T):
    """Yield (di, dj, kk, weight_array, neighbour-index shift) for every gated pair.

    The neighbourhood of active point q = (i, j, k) is every active point
    p = (i+di, j+dj, kk) in frame with |di|, |dj| <= R and circular
    |t_p - t_q| <= tau_z; it includes q itself.
    """
    K = t.shape[-1]
    for di in range(-R, R + 1):
        for dj in range(-R, R + 1):
            w = window_weight(di, dj, R)
            tn = _shift(t, di, dj, 0.0)
            an = _shift(act, di, dj, False)
            for kk in range(K):
                d = circ_diff(tn[..., kk:kk + 1] - t, T)
                gate = act & an[..., kk:kk + 1] & (np.abs(d) <= tau_z)
                yield di, dj, kk, np.where(gate, w, 0.0), d


def chol_solve(M, b, eps=CHOL_EPS):
    """Solve M x = b for a stack of small SPD systems by Cholesky.

    Returns (x, ok); ok is False where a pivot M_jj - sum_k L_jk^2 <= eps * trace(M).
    """
    d = M.shape[-1]
    tr = np.trace(M, axis1=-2, axis2=-1)
    L = np.zeros_like(M)
    ok = np.ones(M.shape[:-2], dtype=bool)
    for j in range(d):
        s = M[..., j, j] - np.sum(L[..., j, :j] ** 2, axis=-1)
        ok &= s > eps * tr
        ljj = np.sqrt(np.where(ok, s, 1.0))
        L[..., j, j] = ljj
        for i in range(j + 1, d):
            L[..., i, j] = (M[..., i, j] - np.sum(L[..., i, :j] * L[..., j, :j], axis=-1)) / ljj
    y = np.zeros(b.shape)
    for j in range(d):
        y[..., j] = (b[..., j] - np.sum(L[..., j, :j] * y[..., :j], axis=-1)) / L[..., j, j]
    x = np.zeros(b.shape)
    for j in range(d - 1, -1, -1):
        x[..., j] = (y[..., j] - np.sum(L[..., j + 1:, j] * x[..., j + 1:], axis=-1)) / L[..., j, j]
    return x, ok


def depth_denoise(st: State, rows: int, cols: int, p: Params, tau_z: float) -> State:
    """Point-cloud denoiser: weighted least-squares height-field fit per point.

    For each active point q, fit d(di, dj) = a + b di + c dj + q (di^2 + dj^2) to the
    centred circular depth offsets d_p = t_p - t_q of its gated neighbourhood with
    the window weights, and move t_q <- t_q + lambda_z * a.  If the 4x4 normal
    matrix is singular by the pivot rule, fit the plane a + b di + c dj; if that is
    singular too, a is the weighted mean offset.  All points read the pre-step depths.
    """
    K = st.t.shape[1]
    t = st.t.reshape(rows, cols, K)
    act = st.active.reshape(rows, cols, K)
    M = np.zeros((rows, cols, K, 4, 4))
    b = np.zeros((rows, cols, K, 4))
    for di, dj, kk, wg, d in _gated_pairs(t, act, rows, cols, p.R, tau_z, p.T):
        phi = np.array([1.0, di, dj, di * di + dj * dj])
        M += wg[..., None, None] * np.outer(phi, phi)
        b += (wg * d)[..., None] * phi
    x4, ok4 = chol_solve(M, b)
    x3, ok3 = chol_solve(M[..., :3, :3], b[..., :3])
    mean = b[..., 0] / np.where(M[..., 0, 0] > 0, M[..., 0, 0], 1.0)
    a = np.where(ok4, x4[..., 0], np.where(ok3, x3[..., 0], mean))
    t_new = np.where(act, wrap(t + p.lambda_z * a, p.T), t)
    return State(t_new.reshape(-1, K), st.alpha.copy(), st.active.copy())


def intensity_denoise(st: State, n, rows: int, cols: int, p: Params, tau_z: float) -> State:
    """Intensity denoiser: gated weighted mean of photon counts r = n * alpha.

    r~_q = sum_p w_p n_p alpha_p / sum_p w_p over the gated neighbourhood (with the
    current, already denoised depths); alpha_q <- r~_q / n_q; the point is removed if
    r~_q < r_min; finally alpha is projected onto the constraint set of eq. (1).
    """
    K = st.t.shape[1]
    t = st.t.reshape(rows, cols, K)
    act = st.active.reshape(rows, cols, K)
    nn = np.asarray(n, dtype=np.float64).reshape(rows, cols, 1)
    r = np.where(act, nn * st.alpha.reshape(rows, cols, K), 0.0)
    num = np.zeros((rows, cols, K))
    den = np.zeros((rows, cols, K))
    for di, dj, kk, wg, _ in _gated_pairs(t, act, rows, cols, p.R, tau_z, p.T):
        num += wg * _shift(r, di, dj, 0.0)[..., kk:kk + 1]
        den += wg
    rt = num / np.where(den > 0, den, 1.0)
    keep = act & (rt >= p.r_min)
    alpha = np.where(keep, rt / np.where(nn > 0, nn, 1.0), 0.0).reshape(-1, K)
    keep = keep.reshape(-1, K)
    return State(st.t.copy(), project_capped_simplex(alpha, keep), keep)


# ---------------------------------------------------------------------------
# background and output
# ---------------------------------------------------------------------------
def background(st: State, n, rows: int, cols: int, p: Params):
    """b = n * alpha_0 / T photons per bin, alpha_0 = max(0, 1 - sum alpha), then a
    (2 Rb + 1)^2 box mean over the in-frame pixels."""
    a0 = np.maximum(0.0, 1.0 - np.where(st.active, st.alpha, 0.0).sum(1))
    braw = (np.asarray(n, dtype=np.float64) * a0 / p.T).reshape(rows, cols)
    s = np.zeros((rows, cols))
    c = np.zeros((rows, cols))
    for di in range(-p.Rb, p.Rb + 1):
        for dj in range(-p.Rb, p.Rb + 1):
            s += _shift(braw, di, dj, 0.0)
            c += _shift(np.ones((rows, cols)), di, dj, 0.0)
    return (s / c).reshape(-1)


def output(st: State, n):
    """Per-pixel slots sorted by depth, inactive slots last (depth 0, intensity 0)."""
    key = np.where(st.active, st.t, np.inf)
    order = np.argsort(key, axis=1, kind="stable")
    take = lambda a: np.take_along_axis(a, order, axis=1)  # noqa: E731
    act = take(st.active)
    depth = np.where(act, take(st.t), 0.0)
    inten = np.where(act, take(np.asarray(n, dtype=np.float64)[:, None] * st.alpha), 0.0)
    return depth, inten, act


def default_tau_z(irf, origin: int, p: Params) -> float:
    return p.tau_z if p.tau_z > 0 else 3.0 * irf_sigma(irf, origin)


# ---------------------------------------------------------------------------
# merge and birth of points
# ---------------------------------------------------------------------------
def merge_points(st: State, p: Params) -> State:
    """Two active points of a pixel closer than T/(2m) (circular) become one, in slot order: the
    lower slot k takes t = the alpha-weighted circular mean, alpha = the sum; the other slot is
    cleared."""
    T, K = p.T, st.t.shape[1]
    t, a, act = st.t.copy(), st.alpha.copy(), st.active.copy()
    for k in range(K):
        for q in range(k + 1, K):
            d = circ_diff(t[:, q] - t[:, k], T)                          # signed, (-T/2, T/2]
            both = act[:, k] & act[:, q] & (np.abs(d) * 2 * p.m < T)
            s = a[:, k] + a[:, q]
            w = np.where(s > 0, a[:, q] / np.where(s > 0, s, 1.0), 0.5)
            t[:, k] = np.where(both, wrap(t[:, k] + w * d, T), t[:, k])
            a[:, k] = np.where(both, s, a[:, k])
            a[:, q] = np.where(both, 0.0, a[:, q])
            act[:, q] &= ~both
    return State(t, a, act)


def birth_correlation(st: State, z, hhat, p: Params):
    """The birth step's sketched matched filter: on the grid tau = 0, s, 2s, ... the correlation
    c[p, g] = Re sum_l conj(hhat_l) w_l exp(-i w_l tau_g) of the residual w = z - Phi(theta), -inf
    at grid points closer than T/m (circularly) to an active point.  Also returns
    sum_l |conj(hhat_l) w_l| per pixel, which bounds |c|.  Returns (tau [G], c [P, G], cabs [P])."""
    T, m = p.T, p.m
    z = np.asarray(z, dtype=np.complex128)
    s = p.stride
    G = -(-T // s)
    tau = np.arange(G, dtype=np.int64) * s
    ell = np.arange(1, m + 1, dtype=np.int64)
    Eg = np.exp(-1j * 2.0 * np.pi * np.mod(tau[:, None] * ell[None, :], T) / T)    # [G, m]
    w = z - np.einsum("pk,pkl->pl", np.where(st.active, st.alpha, 0.0), atoms(st.t, hhat, T))
    c = ((np.conj(hhat) * w) @ Eg.T).real                                       # [P, G]
    dist = np.abs(circ_diff(tau[None, None, :] - st.t[:, :, None], T))          # [P, K, G]
    excluded = np.any(st.active[:, :, None] & (dist * m < T), axis=1)
    return tau, np.where(excluded, -np.inf, c), np.abs(np.conj(hhat) * w).sum(1)


def birth_points(st: State, z, n, hhat, p: Params) -> State:
    """Where a pixel has a free slot and photons: the sketched matched filter of the init
    (grid 0, s, 2s, ...) on the residual z - Phi(theta), restricted to grid points at circular
    distance >= T/m from every active point; the maximum (lowest tau on ties) with amplitude
    a = max(0, c / sum |hhat|^2) becomes a point in the first free slot iff n a >= r_min; then
    alpha is projected onto {alpha >= 0, sum alpha <= 1}."""
    n = np.asarray(n, dtype=np.int64)
    P = st.t.shape[0]
    e2 = float(np.sum(np.abs(hhat) ** 2))
    tau, c, _ = birth_correlation(st, z, hhat, p)
    g = np.argmax(c, axis=1)
    rows = np.arange(P)
    best = c[rows, g]
    a = np.where(np.isfinite(best), np.maximum(0.0, best / e2), 0.0)
    free = ~st.active
    slot = np.argmax(free, axis=1)
    born = free.any(1) & (n > 0) & np.isfinite(best) & (n * a >= p.r_min)
    t, al, act = st.t.copy(), st.alpha.copy(), st.active.copy()
    t[rows[born], slot[born]] = tau[g[born]]
    al[rows[born], slot[born]] = a[born]
    act[rows[born], slot[born]] = True
    return State(t, project_capped_simplex(np.where(act, al, 0.0), act), act)


def iterate(st: State, z, n, hhat, rows, cols, p: Params, tau_z: float, iters: int) -> State:
    """`iters` x (data step, depth denoiser, intensity denoiser); with birth_every = B > 0, after
    iteration i (counted from 1 in this call) with i % B == 0 and i < iters, merge then birth."""
    gam_t, gam_a = step_sizes(n, hhat, p)
    for it in range(iters):
        st = data_step(st, z, n, hhat, p, gam_t, gam_a)
        st = depth_denoise(st, rows, cols, p, tau_z)
        st = intensity_denoise(st, n, rows, cols, p, tau_z)
        if p.birth_every > 0 and (it + 1) % p.birth_every == 0 and it + 1 < iters:
            st = birth_points(merge_points(st, p), z, n, hhat, p)
    return st


def reconstruct(z, n, irf, origin: int, rows: int, cols: int, p: Params, iters=None):
    """Full SRT3D: spectrum, init, `iters` x (data, depth, intensity), background, output."""
    hhat = irf_spectrum(irf, origin, p.T, p.m)
    tau_z = default_tau_z(irf, origin, p)
    st0 = init_points(z, n, hhat, p)
    st = iterate(st0, z, n, hhat, rows, cols, p, tau_z, p.iters if iters is None else iters)
    depth, inten, act = output(st, n)
    return dict(depth=depth, intensity=inten, active=act, bg=background(st, n, rows, cols, p),
                state=st, init=st0, hhat=hhat, tau_z=tau_z)


# ---------------------------------------------------------------------------
# per-point loops (tiny frames): the same denoisers written point by point
# ---------------------------------------------------------------------------
def _small_solve(M, b, eps=CHOL_EPS):
    d = len(b)
    tr = sum(M[i][i] for i in range(d))
    L = [[0.0] * d for _ in range(d)]
    for j in range(d):
        s = M[j][j] - sum(L[j][k] ** 2 for k in range(j))
        if not s > eps * tr:
            return None
        L[j][j] = math.sqrt(s)
        for i in range(j + 1, d):
            L[i][j] = (M[i][j] - sum(L[i][k] * L[j][k] for k in range(j))) / L[j][j]
    y = [0.0] * d
    for j in range(d):
        y[j] = (b[j] - sum(L[j][k] * y[k] for k in range(j))) / L[j][j]
    x = [0.0] * d
    for j in reversed(range(d)):
        x[j] = (y[j] - sum(L[k][j] * x[k] for k in range(j + 1, d))) / L[j][j]
    return x


def _neighbours_loop(t, act, i, j, k, rows, cols, R, tau_z, T):
    out = []
    for di in range(-R, R + 1):
        for dj in range(-R, R + 1):
            ii, jj = i + di, j + dj
            if not (0 <= ii < rows and 0 <= jj < cols):
                continue
            for kk in range(t.shape[2]):
                if not act[ii, jj, kk]:
                    continue
                d = (t[ii, jj, kk] - t[i, j, k]) % T
                if d > T / 2:
                    d -= T
                if abs(d) <= tau_z:
                    out.append((di, dj, kk, window_weight(di, dj, R), d))
    return out


def depth_denoise_loop(st: State, rows, cols, p: Params, tau_z: float) -> State:
    K = st.t.shape[1]
    t = st.t.reshape(rows, cols, K)
    act = st.active.reshape(rows, cols, K)
    t_new = t.copy()
    for i in range(rows):
        for j in range(cols):
            for k in range(K):
                if not act[i, j, k]:
                    continue
                nb = _neighbours_loop(t, act, i, j, k, rows, cols, p.R, tau_z, p.T)
                a = None
                for dim in (4, 3):
                    M = [[0.0] * dim for _ in range(dim)]
                    b = [0.0] * dim
                    for di, dj, _, w, d in nb:
                        phi = [1.0, di, dj, di * di + dj * dj][:dim]
                        for r_ in range(dim):
                            b[r_] += w * phi[r_] * d
                            for c_ in range(dim):
                                M[r_][c_] += w * phi[r_] * phi[c_]
                    x = _small_solve(M, b)
                    if x is not None:
                        a = x[0]
                        break
                if a is None:
                    a = sum(w * d for *_, w, d in nb) / sum(w for *_, w, _ in nb)
                v = (t[i, j, k] + p.lambda_z * a) % p.T
                t_new[i, j, k] = v - p.T if v >= p.T else v
    return State(t_new.reshape(-1, K), st.alpha.copy(), st.active.copy())


def intensity_denoise_loop(st: State, n, rows, cols, p: Params, tau_z: float) -> State:
    K = st.t.shape[1]
    t = st.t.reshape(rows, cols, K)
    act = st.active.reshape(rows, cols, K)
    nn = np.asarray(n, dtype=np.float64).reshape(rows, cols)
    al = st.alpha.reshape(rows, cols, K)
    alpha = np.zeros((rows, cols, K))
    keep = np.zeros((rows, cols, K), dtype=bool)
    for i in range(rows):
        for j in range(cols):
            for k in range(K):
                if not act[i, j, k]:
                    continue
                nb = _neighbours_loop(t, act, i, j, k, rows, cols, p.R, tau_z, p.T)
                num = sum(w * nn[i + di, j + dj] * al[i + di, j + dj, kk] for di, dj, kk, w, _ in nb)
                den = sum(w for *_, w, _ in nb)
                rt = num / den
                if rt >= p.r_min:
                    keep[i, j, k] = True
                    alpha[i, j, k] = rt / nn[i, j]
    keep = keep.reshape(-1, K)
    return State(st.t.copy(), project_capped_simplex(alpha.reshape(-1, K), keep), keep)


def with_params(p: Params, **kw) -> Params:
    return replace(p, **kw)


__all__ = [
    "Params", "State", "wrap", "circ_diff", "project_capped_simplex", "step_sizes", "init_points",
    "data_step", "depth_denoise", "intensity_denoise", "background", "output", "iterate",
    "reconstruct", "chol_solve", "window_weight", "depth_denoise_loop", "intensity_denoise_loop",
    "default_tau_z", "irf_spectrum", "atoms", "unit_phasors", "merge_points", "birth_correlation", "birth_points",
]
