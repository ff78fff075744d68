"""Pins of the SRT3D iteration oracle: constraint projection, init, data step,
denoisers, background, output and the whole iteration."""
import itertools

import numpy as np
import pytest

import synth
from oracle import model as OM
from oracle import srt3d as O


# ------------------------------------------------------------------ projection
def test_projection_brute_force():
    """Projection onto {a >= 0, sum a <= 1}: feasible, and (v - x).(y - x) <= 0 for all y in
    the set (variational inequality), checked on the set's vertices and a dense grid."""
    rng = np.random.default_rng(0)
    for K in (1, 2, 3):
        grid = np.array([g for g in itertools.product(np.linspace(0, 1, 21), repeat=K) if sum(g) <= 1 + 1e-12])
        for _ in range(200):
            v = rng.normal(0.3, 0.8, (1, K))
            x = O.project_capped_simplex(v, np.ones((1, K), bool))[0]
            assert np.all(x >= -1e-15) and x.sum() <= 1 + 1e-12
            assert np.max((grid - x) @ (v[0] - x)) <= 1e-12
            # brute force: no grid point is closer than x (up to grid resolution)
            assert np.sum((v[0] - x) ** 2) <= np.min(np.sum((grid - v[0]) ** 2, 1)) + 1e-12


def test_projection_respects_active_mask():
    v = np.array([[0.9, 0.8, 0.7]])
    act = np.array([[True, False, True]])
    x = O.project_capped_simplex(v, act)
    np.testing.assert_allclose(x, [[0.6, 0.0, 0.4]], atol=1e-15)


# ------------------------------------------------------------------ helpers
def _gauss_irf(sigma):
    o = int(np.ceil(6 * sigma))
    return np.exp(-0.5 * (np.arange(-o, o + 1) / sigma) ** 2), o


def _noiseless(t, alpha, active, hhat, T):
    return OM.model_sketch(t, alpha, active, hhat, T)


# ------------------------------------------------------------------ init
def test_init_recovers_grid_surface():
    T, m = 1024, 8
    p = O.Params(T, m, 1)
    h, o = _gauss_irf(3.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    s = p.stride
    t = (np.arange(20) * 7 % (T // s) * s).astype(float)[:, None]
    alpha = np.linspace(0.1, 0.9, 20)[:, None]
    act = np.ones((20, 1), bool)
    z = _noiseless(t, alpha, act, hhat, T)
    st = O.init_points(z, np.full(20, 100), hhat, p)
    np.testing.assert_array_equal(st.t, t)
    np.testing.assert_allclose(st.alpha, alpha, atol=1e-12)
    assert st.active.all()


def test_init_greedy_two_orthogonal_atoms():
    """Delta response, m even, surfaces T/2 apart: the atoms are orthogonal, so greedy
    pursuit returns both amplitudes exactly, strongest first."""
    T, m = 480, 6
    p = O.Params(T, m, 2)
    assert p.stride == 10
    hhat = OM.irf_spectrum([1.0], 0, T, m)
    t = np.array([[60.0, 60.0 + T / 2]])
    alpha = np.array([[0.25, 0.45]])
    z = _noiseless(t, alpha, np.ones((1, 2), bool), hhat, T)
    st = O.init_points(z, np.array([50]), hhat, p)
    np.testing.assert_array_equal(st.t, [[60.0 + T / 2, 60.0]])
    np.testing.assert_allclose(st.alpha, [[0.45, 0.25]], atol=1e-12)


def test_init_empty_and_threshold():
    T, m = 256, 4
    p = O.Params(T, m, 1, r_min=5.0)
    hhat = OM.irf_spectrum([1.0], 0, T, m)
    z = _noiseless(np.array([[32.0], [64.0]]), np.array([[0.5], [0.5]]), np.ones((2, 1), bool), hhat, T)
    z[0] = 0
    st = O.init_points(z, np.array([0, 8]), hhat, p)     # n=0, and 8 * 0.5 = 4 < r_min
    assert not st.active.any()
    assert np.all(st.alpha == 0)


# ------------------------------------------------------------------ data step
def test_data_step_noiseless_fixed_point_and_convergence():
    T, m = 4096, 16
    p = O.Params(T, m, 1)
    h, o = _gauss_irf(8.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    P = 50
    rng = np.random.default_rng(1)
    t = rng.uniform(100, 4000, (P, 1))
    alpha = rng.uniform(0.3, 0.9, (P, 1))
    act = np.ones((P, 1), bool)
    n = np.full(P, 1000)
    z = _noiseless(t, alpha, act, hhat, T)
    gt, ga = O.step_sizes(n, hhat, p)
    st = O.data_step(O.State(t.copy(), alpha.copy(), act.copy()), z, n, hhat, p, gt, ga)
    np.testing.assert_allclose(st.t, t, atol=1e-9)
    np.testing.assert_allclose(st.alpha, alpha, atol=1e-12)
    st = O.State(t + rng.uniform(-6, 6, (P, 1)), alpha * 0.8, act.copy())
    L0 = OM.loss(z, n, st.t, st.alpha, act, hhat, T)
    for _ in range(300):
        st = O.data_step(st, z, n, hhat, p, gt, ga)
    assert np.all(OM.loss(z, n, st.t, st.alpha, act, hhat, T) <= L0)
    np.testing.assert_allclose(O.circ_diff(st.t - t, T), 0, atol=1e-3)
    np.testing.assert_allclose(st.alpha, alpha, atol=1e-4)


def test_step_sizes_are_the_curvature_of_the_data_term():
    """The steps are eta / L with L bounds of the data term's curvature (reading 10).  At a
    noiseless state with one point of intensity 1 in every pixel the bounds are attained: the
    second differences of the loss along t and along alpha equal L_t and L_alpha.  With two
    points and alpha in the simplex they bound the curvature: the t second differences and the
    largest eigenvalue of the alpha-block Hessian stay below them."""
    T, m, P = 256, 6, 40
    rng = np.random.default_rng(3)
    h, o = synth.binned_gaussian_irf(3.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    n = np.full(P, 500)
    for K in (1, 2):
        p = O.Params(T, m, K, eta_t=0.7, eta_a=1.3)
        gt, ga = O.step_sizes(n, hhat, p)
        Lt, La = p.eta_t / gt, p.eta_a / ga
        t = rng.uniform(0, T, (P, K))
        act = np.ones((P, K), bool)
        alpha = np.ones((P, K)) if K == 1 else rng.dirichlet([1.0] * K, P)
        z = OM.model_sketch(t, alpha, act, hhat, T)
        loss = lambda tt, aa: OM.loss(z, n, tt, aa, act, hhat, T)       # noqa: E731
        e = 1e-3
        L0 = loss(t, alpha)
        d2t = np.empty((P, K))
        H = np.empty((P, K, K))
        for k in range(K):
            d = np.zeros((P, K))
            d[:, k] = e
            d2t[:, k] = (loss(t + d, alpha) - 2 * L0 + loss(t - d, alpha)) / e**2
            for j in range(K):
                dj = np.zeros((P, K))
                dj[:, j] = e
                H[:, k, j] = (loss(t, alpha + d + dj) - loss(t, alpha + d - dj) - loss(t, alpha - d + dj)
                              + loss(t, alpha - d - dj)) / (4 * e**2)
        lam = np.linalg.eigvalsh(H).max(1)
        if K == 1:
            np.testing.assert_allclose(d2t[:, 0], Lt, rtol=1e-5)
            np.testing.assert_allclose(lam, La, rtol=1e-6)
        else:
            assert np.all(d2t <= Lt * (1 + 1e-6)) and np.all(lam <= La * (1 + 1e-9))
            assert d2t.max() > 0.2 * Lt and lam.max() > 0.3 * La          # and not vacuous
    assert O.step_sizes(np.zeros(3), hhat, O.Params(T, m, 1)) == (0.0, 0.0)


# ------------------------------------------------------------------ depth denoiser
def _grid_state(tmap, active=None):
    rows, cols = tmap.shape
    act = np.ones((rows * cols, 1), bool) if active is None else active.reshape(-1, 1)
    return O.State(tmap.reshape(-1, 1).astype(float), np.full((rows * cols, 1), 0.5), act)


def test_depth_denoiser_plane_and_paraboloid_fixed_points():
    rows, cols, T = 12, 9, 4096
    p = O.Params(T, 8, 1)
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    for tmap in (1000.3 + 0.37 * ii - 0.21 * jj, 2000.0 + 0.02 * ((ii - 4.5) ** 2 + (jj - 3.0) ** 2) + 0.1 * ii):
        st = O.depth_denoise(_grid_state(tmap), rows, cols, p, tau_z=20.0)
        np.testing.assert_allclose(st.t.reshape(rows, cols), tmap, atol=1e-9)


def test_depth_denoiser_matches_weighted_lstsq():
    """Centre of a full window: a equals the intercept of the weighted least-squares fit
    solved by numpy's lstsq on sqrt(w)-scaled rows."""
    rng = np.random.default_rng(2)
    rows = cols = 5
    T = 4096
    p = O.Params(T, 8, 1)
    tmap = 500 + rng.normal(0, 2, (rows, cols))
    st = O.depth_denoise(_grid_state(tmap), rows, cols, p, tau_z=50.0)
    A, b, sw = [], [], []
    for di in range(-2, 3):
        for dj in range(-2, 3):
            A.append([1, di, dj, di * di + dj * dj])
            b.append(tmap[2 + di, 2 + dj] - tmap[2, 2])
            sw.append(np.sqrt(O.window_weight(di, dj, 2)))
    sw = np.array(sw)
    coef = np.linalg.lstsq(np.array(A) * sw[:, None], np.array(b) * sw, rcond=None)[0]
    assert st.t.reshape(rows, cols)[2, 2] == pytest.approx(tmap[2, 2] + coef[0], abs=1e-9)


def test_depth_denoiser_isolated_point_and_gate():
    rows, cols, T = 7, 7, 1024
    p = O.Params(T, 4, 1)
    tmap = np.full((rows, cols), 300.0)
    tmap[3, 3] = 700.0                       # far outside the gate: its own neighbourhood is itself
    tmap[0, 0] = 310.0                       # inside the gate, pulled toward the plane
    st = O.depth_denoise(_grid_state(tmap), rows, cols, p, tau_z=15.0)
    out = st.t.reshape(rows, cols)
    assert out[3, 3] == 700.0
    assert 300.0 < out[0, 0] < 310.0


def test_depth_denoiser_shift_equivariance_and_wrap():
    rng = np.random.default_rng(3)
    rows, cols, T = 10, 11, 2048
    p = O.Params(T, 8, 1)
    tmap = rng.uniform(0, 30, (rows, cols)) + 5
    act = rng.uniform(size=(rows, cols)) < 0.8
    a = O.depth_denoise(_grid_state(tmap, act), rows, cols, p, tau_z=12.0)
    for D in (100, T - 10):                  # T - 10 wraps part of the frame across 0
        b = O.depth_denoise(_grid_state((tmap + D) % T, act), rows, cols, p, tau_z=12.0)
        np.testing.assert_allclose(O.circ_diff(b.t - a.t - D, T), 0, atol=1e-9)


def test_depth_denoiser_vectorised_matches_loop():
    rng = np.random.default_rng(4)
    rows, cols, T, K = 9, 8, 512, 2
    p = O.Params(T, 8, K)
    t = rng.uniform(0, 40, (rows * cols, K)) + np.array([100.0, 400.0])
    t[rng.uniform(size=t.shape) < 0.1] += 200               # some outliers beyond the gate
    act = rng.uniform(size=t.shape) < 0.85
    st = O.State(t, np.full(t.shape, 0.3), act)
    a = O.depth_denoise(st, rows, cols, p, tau_z=10.0)
    b = O.depth_denoise_loop(st, rows, cols, p, tau_z=10.0)
    np.testing.assert_allclose(a.t, b.t, atol=1e-9)


# ------------------------------------------------------------------ intensity denoiser
def test_intensity_denoiser_constant_fixed_point_and_removal():
    rows, cols, T = 8, 8, 1024
    p = O.Params(T, 4, 1, r_min=3.0)
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    st = O.State((300 + 0.2 * ii + 0.1 * jj).reshape(-1, 1), np.full((64, 1), 0.25), np.ones((64, 1), bool))
    n = np.full(64, 40)
    out = O.intensity_denoise(st, n, rows, cols, p, tau_z=10.0)
    np.testing.assert_allclose(out.alpha, st.alpha, atol=1e-15)
    assert out.active.all()
    st.t[27, 0] = 900.0                      # isolated point with r = 40 * 0.05 = 2 < r_min
    st.alpha[27, 0] = 0.05
    out = O.intensity_denoise(st, n, rows, cols, p, tau_z=10.0)
    assert not out.active[27, 0] and out.alpha[27, 0] == 0
    assert out.active.sum() == 63


def test_intensity_denoiser_weighted_mean_and_loop():
    rng = np.random.default_rng(5)
    rows, cols, T, K = 7, 9, 512, 2
    p = O.Params(T, 8, K, r_min=2.0)
    t = rng.uniform(0, 20, (rows * cols, K)) + np.array([100.0, 300.0])
    act = rng.uniform(size=t.shape) < 0.8
    alpha = rng.uniform(0.05, 0.5, t.shape)
    n = rng.integers(1, 60, rows * cols)
    st = O.State(t, alpha, act)
    a = O.intensity_denoise(st, n, rows, cols, p, tau_z=8.0)
    b = O.intensity_denoise_loop(st, n, rows, cols, p, tau_z=8.0)
    np.testing.assert_array_equal(a.active, b.active)
    np.testing.assert_allclose(a.alpha, b.alpha, atol=1e-12)


# ------------------------------------------------------------------ background / output
def test_background_closed_form():
    rows, cols, T = 5, 6, 1000
    p = O.Params(T, 4, 2, Rb=1)
    alpha = np.tile([0.3, 0.2], (30, 1))
    st = O.State(np.zeros((30, 2)), alpha, np.ones((30, 2), bool))
    n = np.arange(30) + 10
    b = O.background(st, n, rows, cols, p).reshape(rows, cols)
    raw = (n * 0.5 / T).reshape(rows, cols)
    for i in range(rows):
        for j in range(cols):
            win = raw[max(0, i - 1):i + 2, max(0, j - 1):j + 2]
            assert b[i, j] == pytest.approx(win.mean(), rel=1e-13)


def test_output_sorted_inactive_last():
    st = O.State(np.array([[50.0, 10.0, 30.0], [5.0, 1.0, 2.0]]), np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3]]),
                 np.array([[True, True, False], [False, True, True]]))
    d, r, a = O.output(st, np.array([100, 10]))
    np.testing.assert_array_equal(d, [[10.0, 50.0, 0.0], [1.0, 2.0, 0.0]])
    np.testing.assert_allclose(r, [[20.0, 10.0, 0.0], [2.0, 3.0, 0.0]])
    np.testing.assert_array_equal(a, [[True, True, False], [True, True, False]])


# ------------------------------------------------------------------ whole iteration
def test_noiseless_planar_scene_converges():
    """z = Phi(theta*) for a plane of constant intensity: a fixed point of all three steps,
    reached from the grid initialisation."""
    rows, cols, T, m = 16, 16, 4096, 8
    p = O.Params(T, m, 1, iters=200)
    h, o = _gauss_irf(6.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    t = (2000.4 + 0.3 * ii - 0.2 * jj).reshape(-1, 1)
    alpha = np.full((rows * cols, 1), 0.6)
    act = np.ones_like(alpha, bool)
    n = np.full(rows * cols, 800)
    z = _noiseless(t, alpha, act, hhat, T)
    r = O.reconstruct(z, n, h, o, rows, cols, p)
    np.testing.assert_allclose(O.circ_diff(r["depth"] - t, T), 0, atol=1e-3)
    np.testing.assert_allclose(r["intensity"], 480.0, rtol=1e-3)
    np.testing.assert_allclose(r["bg"], 800 * 0.4 / T, rtol=1e-3)


def test_reconstruction_shift_equivariance():
    """Shifting every stamp by D (a multiple of the init grid step) shifts every depth by D."""
    rng = np.random.default_rng(6)
    rows, cols, T, m = 10, 10, 1024, 6
    p = O.Params(T, m, 1, iters=10)
    h, o = _gauss_irf(4.0)
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    tt = (400 + 0.5 * ii + 0.3 * jj).reshape(-1)
    x = [np.concatenate([np.rint(t0 + 4 * rng.normal(size=60)), rng.integers(0, T, 40)]).astype(int) for t0 in tt]
    off = np.concatenate([[0], np.cumsum([len(v) for v in x])])
    from oracle import sketch as OS
    z0, n = OS.sketch(np.concatenate(x), off, T, m)
    D = 5 * p.stride
    z1, _ = OS.sketch((np.concatenate(x) + D) % T, off, T, m)
    a = O.reconstruct(z0, n, h, o, rows, cols, p)
    b = O.reconstruct(z1, n, h, o, rows, cols, p)
    np.testing.assert_array_equal(a["active"], b["active"])
    np.testing.assert_allclose(O.circ_diff(b["depth"] - a["depth"] - D, T)[a["active"]], 0, atol=1e-6)
    np.testing.assert_allclose(b["intensity"], a["intensity"], atol=1e-6)


# ------------------------------------------------------------------ merge and birth
def test_birth_adds_the_missing_orthogonal_surface():
    """Delta response, m even, surfaces T/2 apart: with only the first active, the residual is
    exactly the second atom, whose grid position and amplitude the birth returns exactly."""
    T, m = 480, 6
    p = O.Params(T, m, 2)
    hhat = OM.irf_spectrum([1.0], 0, T, m)
    t = np.array([[60.0, 300.0]])
    alpha = np.array([[0.25, 0.45]])
    z = _noiseless(t, alpha, np.ones((1, 2), bool), hhat, T)
    st = O.State(np.array([[60.0, 0.0]]), np.array([[0.25, 0.0]]), np.array([[True, False]]))
    b = O.birth_points(st, z, np.array([50]), hhat, p)
    np.testing.assert_array_equal(b.active, [[True, True]])
    np.testing.assert_allclose(b.t, t, atol=1e-12)
    np.testing.assert_allclose(b.alpha, alpha, atol=1e-12)
    # too few photons for the new point (n a = 0.45 n < r_min), or no free slot: unchanged
    b2 = O.birth_points(st, z, np.array([2]), hhat, O.Params(T, m, 2, r_min=1.0))
    np.testing.assert_array_equal(b2.active, st.active)
    full = O.State(np.array([[60.0, 120.0]]), np.array([[0.25, 0.1]]), np.array([[True, True]]))
    b3 = O.birth_points(full, z, np.array([50]), hhat, p)
    np.testing.assert_array_equal(b3.t, full.t)


def test_birth_respects_the_exclusion_distance():
    """A residual peaked at an active point (its amplitude underestimated) cannot spawn a point
    closer than T/m to it."""
    T, m = 1024, 8
    p = O.Params(T, m, 3, r_min=0.0)
    h, o = _gauss_irf(3.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    rng = np.random.default_rng(7)
    P = 40
    t = rng.uniform(0, T, (P, 1))
    z = _noiseless(t, np.full((P, 1), 0.8), np.ones((P, 1), bool), hhat, T)
    st = O.State(np.concatenate([t, np.zeros((P, 2))], 1), np.concatenate([np.full((P, 1), 0.3), np.zeros((P, 2))], 1),
                 np.array([[True, False, False]] * P))
    b = O.birth_points(st, z, np.full(P, 100), hhat, p)
    born = b.active[:, 1]
    d = np.abs(O.circ_diff(b.t[:, 1] - t[:, 0], T))
    assert np.all(d[born] * m >= T)
    assert not b.active[:, 2].any()          # one birth per stage


def test_merge_weighted_circular_mean():
    T, m = 1000, 10                          # merge below T/(2m) = 50 bins
    p = O.Params(T, m, 3)
    st = O.State(np.array([[100.0, 130.0, 700.0], [990.0, 20.0, 500.0], [100.0, 160.0, 300.0]]),
                 np.array([[0.2, 0.3, 0.1], [0.1, 0.3, 0.2], [0.2, 0.3, 0.1]]),
                 np.array([[True, True, True], [True, True, True], [True, True, False]]))
    r = O.merge_points(st, p)
    np.testing.assert_allclose(r.t[0, :1], [100.0 + 0.6 * 30.0])
    np.testing.assert_allclose(r.alpha[0], [0.5, 0.0, 0.1])
    np.testing.assert_array_equal(r.active[0], [True, False, True])
    np.testing.assert_allclose(r.t[1, 0], 990.0 + 0.75 * 30.0 - 1000.0)     # across the wrap
    np.testing.assert_allclose(r.alpha[1], [0.4, 0.0, 0.2])
    np.testing.assert_array_equal(r.active[2], [True, True, False])         # 60 bins apart: kept
    np.testing.assert_array_equal(r.t[2], st.t[2])


def test_iterations_with_births_find_a_surface_the_start_lacks():
    """Noiseless two-surface pixels started from one surface only: with merge/birth stages
    every 5 iterations the second surface is found; without them it is not."""
    T, m, rows, cols = 1024, 8, 6, 6
    P = rows * cols
    h, o = _gauss_irf(2.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    t = np.stack([np.full(P, 200.0), np.full(P, 600.0)], 1)
    alpha = np.stack([np.full(P, 0.3), np.full(P, 0.4)], 1)
    z = _noiseless(t, alpha, np.ones((P, 2), bool), hhat, T)
    n = np.full(P, 500)
    st0 = O.State(np.stack([t[:, 0], np.zeros(P)], 1), np.stack([alpha[:, 0], np.zeros(P)], 1),
                  np.stack([np.ones(P, bool), np.zeros(P, bool)], 1))
    tau_z = 6.0
    with_b = O.iterate(st0, z, n, hhat, rows, cols, O.Params(T, m, 2, birth_every=5), tau_z, 40)
    without = O.iterate(st0, z, n, hhat, rows, cols, O.Params(T, m, 2), tau_z, 40)
    assert with_b.active.all() and not without.active[:, 1].any()
    d = np.abs(O.circ_diff(np.sort(with_b.t, 1) - t, T))
    assert np.max(d) < 0.5
