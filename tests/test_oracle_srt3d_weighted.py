"""Pins of SRT3D with the precision weighting in its data step (oracle/srt3d_weighted.py): the
weights invert the ridged covariance, W = c I gives exactly SRT3D's W = I step and iteration,
the weighted gradient against central differences and against the independent W = I formula,
and the noiseless fixed point."""
import numpy as np
import pytest

import synth
from oracle import model as OM
from oracle import sketch as OS
from oracle import srt3d as O
from oracle import srt3d_weighted as OW
from oracle import weighted as OWP


def _problem(seed, P=40, K=2, T=512, m=6):
    rng = np.random.default_rng(seed)
    h, o = synth.binned_gaussian_irf(3.0)
    hhat = OM.irf_spectrum(h, o, T, m)
    hhat2 = OM.irf_spectrum(h, o, T, 2 * m)
    t = rng.uniform(0, T, (P, K))
    a = rng.uniform(0.05, 0.4, (P, K))
    act = rng.uniform(size=(P, K)) < 0.8
    act[:, 0] = True
    z = OM.model_sketch(t + rng.normal(0, 2, (P, K)), a * rng.uniform(0.8, 1.2, (P, K)), act, hhat, T)
    z = z + (rng.normal(0, 0.03, z.shape) + 1j * rng.normal(0, 0.03, z.shape))
    n = rng.integers(20, 2000, P)
    st = O.State(t, np.where(act, a, 0.0), act)
    return T, m, hhat, hhat2, z, n, st


def test_weights_invert_the_ridged_covariance():
    T, m, hhat, hhat2, z, n, st = _problem(0)
    p = O.Params(T, m, 2)
    W = OW.weight_matrices(st, hhat2, p)
    S = OWP.covariance(st.t, st.alpha, st.active, hhat2, T, m)
    d = 2 * m
    tr = np.trace(S, axis1=1, axis2=2)
    Sr = S + (OWP.RIDGE * tr / d)[:, None, None] * np.eye(d)
    np.testing.assert_allclose(np.einsum("pij,pjk->pik", W, Sr), np.broadcast_to(np.eye(d), W.shape), atol=1e-8)
    np.testing.assert_allclose(W, np.swapaxes(W, 1, 2), atol=1e-9)
    lam = np.linalg.eigvalsh(W).max(1)
    assert np.all(OW.gershgorin(W) >= lam * (1 - 1e-12))
    assert np.allclose(OW.gershgorin(np.broadcast_to(3.0 * np.eye(d), W.shape)), 3.0)


def test_identity_weights_give_the_srt3d_step_and_iteration():
    """W_p = c I for every pixel: the weighted steps are the W = I steps divided by c and the
    gradient is c times the W = I gradient, so data step and whole iterations equal SRT3D's.  The
    covariance of a pixel without signal is I / 2 exactly, which gives such weights."""
    T, m, hhat, hhat2, z, n, st = _problem(1)
    p = O.Params(T, m, 2)
    P = z.shape[0]
    bg = O.State(st.t, np.zeros_like(st.alpha), st.active)             # no signal: Sigma = I / 2
    W = OW.weight_matrices(bg, hhat2, p)
    c = 1.0 / (0.5 + OWP.RIDGE * 0.5)
    np.testing.assert_allclose(W, np.broadcast_to(c * np.eye(2 * m), W.shape), rtol=1e-12)
    gw = OW.weighted_step_sizes(n, hhat, W, p)
    gi = O.step_sizes(n, hhat, p)
    np.testing.assert_allclose(np.array(gw) * c, gi, rtol=1e-12)
    a = OW.data_step_weighted(st, z, n, hhat, W, p, *gw)
    b = O.data_step(st, z, n, hhat, p, *gi)
    np.testing.assert_allclose(a.t, b.t, atol=1e-9)
    np.testing.assert_allclose(a.alpha, b.alpha, atol=1e-12)
    # whole iterations on a small frame
    spec = synth.FrameSpec(12, 10, 256, 2.0, 300.0, 2.0, 1, seed=4)
    f = synth.make_frame(spec)
    zz, nn = OS.sketch(f.stamps.numpy(), f.offsets.numpy(), spec.T, 5)
    pp = O.Params(spec.T, 5, 1, iters=5)
    hh = OM.irf_spectrum(f.irf, f.irf_origin, spec.T, 5)
    tau = O.default_tau_z(f.irf, f.irf_origin, pp)
    st0 = O.init_points(zz, nn, hh, pp)
    Wc = np.broadcast_to(4.0 * np.eye(10), (spec.P, 10, 10))
    r1 = OW.iterate_weighted(st0, zz, nn, hh, Wc, spec.rows, spec.cols, pp, tau, 5)
    r2 = O.iterate(st0, zz, nn, hh, spec.rows, spec.cols, pp, tau, 5)
    np.testing.assert_allclose(r1.t, r2.t, atol=1e-9)
    np.testing.assert_allclose(r1.alpha, r2.alpha, atol=1e-12)
    np.testing.assert_array_equal(r1.active, r2.active)


def test_identity_weight_gradient_is_the_model_gradient():
    """W = I: 2 n J^T e equals the complex-form gradient of the W = I loss (oracle.model)."""
    T, m, hhat, hhat2, z, n, st = _problem(2)
    I = np.broadcast_to(np.eye(2 * m), (z.shape[0], 2 * m, 2 * m))
    gw = OW.weighted_gradients(z, n, st.t, st.alpha, st.active, hhat, I, T)
    gm = OM.gradients(z, n, st.t, st.alpha, st.active, hhat, T)
    for x, y in zip(gw, gm):
        np.testing.assert_allclose(x, y, rtol=1e-10, atol=1e-9)


def test_weighted_gradient_matches_central_differences():
    T, m, hhat, hhat2, z, n, st = _problem(3, P=12)
    p = O.Params(T, m, 2)
    W = OW.weight_matrices(st, hhat2, p)
    gt, ga = OW.weighted_gradients(z, n, st.t, st.alpha, st.active, hhat, W, T)
    eps = 1e-6
    for k in range(2):
        d = np.zeros_like(st.t)
        d[:, k] = eps
        L = lambda t, a: OW.weighted_loss(z, n, t, a, st.active, hhat, W, T)     # noqa: E731
        ft = (L(st.t + d, st.alpha) - L(st.t - d, st.alpha)) / (2 * eps)
        fa = (L(st.t, st.alpha + d) - L(st.t, st.alpha - d)) / (2 * eps)
        act = st.active[:, k]
        np.testing.assert_allclose(gt[act, k], ft[act], rtol=1e-5, atol=1e-4)
        np.testing.assert_allclose(ga[act, k], fa[act], rtol=1e-5, atol=1e-4)


def test_noiseless_sketch_is_a_fixed_point():
    T, m, hhat, hhat2, z, n, st = _problem(5)
    p = O.Params(T, m, 2)
    z0 = OM.model_sketch(st.t, st.alpha, st.active, hhat, T)
    W = OW.weight_matrices(st, hhat2, p)
    gt, ga = OW.weighted_gradients(z0, n, st.t, st.alpha, st.active, hhat, W, T)
    assert np.abs(gt).max() < 1e-8 and np.abs(ga).max() < 1e-8
    s1 = OW.data_step_weighted(st, z0, n, hhat, W, p, *OW.weighted_step_sizes(n, hhat, W, p))
    np.testing.assert_allclose(s1.t, st.t, atol=1e-9)
    np.testing.assert_allclose(s1.alpha, st.alpha, atol=1e-12)


@pytest.mark.parametrize("sbr", [1.0, 10.0])
def test_weighted_reconstruction_finds_the_surfaces(sbr):
    """The weighted iteration reconstructs a throughput-like frame as well as SRT3D: depths
    within 3 sigma of the synthetic truth on >= 99% of pixels for both."""
    spec = synth.FrameSpec(24, 24, 1024, 4.0, 300.0, sbr, 1, seed=7)
    f = synth.make_frame(spec)
    m = 8
    z, n = OS.sketch(f.stamps.numpy(), f.offsets.numpy(), spec.T, m)
    p = O.Params(spec.T, m, 1, iters=30)
    rw = OW.reconstruct_weighted(z, n, f.irf, f.irf_origin, spec.rows, spec.cols, p)
    r1 = O.reconstruct(z, n, f.irf, f.irf_origin, spec.rows, spec.cols, p)
    tol = 3 * spec.sigma
    hit = lambda r: (r["active"][:, 0] & (np.abs(O.circ_diff(r["depth"][:, 0] - f.scene.depth[:, 0], spec.T)) <= tol)).mean()  # noqa: E731
    print(f"sbr {sbr}: within 3 sigma, weighted {hit(rw):.4f}, W = I {hit(r1):.4f}")
    assert hit(rw) >= 0.99 and hit(r1) >= 0.99
