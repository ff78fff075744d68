"""GPU parity of the pixelwise sketched estimator (srt3d_smle: SRT3D's data steps alone, per-pixel
steps, several starts, the lowest loss kept) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import model as OM
from oracle import smle as OSM
from oracle import srt3d as O
from tests.gpu_common import circ_abs, device, to_complex

pytestmark = pytest.mark.gpu


def _case(**kw):
    print("case smle", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _frame(spec, m, K, dev, **pk):
    f = synth.make_frame(spec, device=dev)
    z, n = srt.sketch(f.stamps, f.offsets, spec.T, m)
    torch.cuda.synchronize()
    params = srt.Params.default(spec.rows, spec.cols, spec.T, m, K, **pk)
    op = O.Params(spec.T, m, K, iters=params.iters, R=params.R, Rb=params.Rb, r_min=params.r_min,
                  tau_z=params.tau_z)
    return f, z, n, params, op


def _run(f, z, n, params, op, starts, dev):
    rec = srt.Reconstructor(params, dev)
    irf = torch.from_numpy(f.irf).to(dev)
    loss = rec.smle(z, n, irf, f.irf_origin, starts)
    t, a, act = (x.cpu().numpy() for x in rec.state())
    torch.cuda.synchronize()
    zc = to_complex(z)
    nn = n.cpu().numpy().astype(np.int64)
    r = OSM.smle(zc, nn, f.irf, f.irf_origin, op, starts)
    return rec, loss.cpu().numpy(), O.State(t.astype(np.float64), a.astype(np.float64), act.astype(bool)), r, zc, nn


CASES = [
    ("tiny", dict(spec=synth.preset("tiny").frame, m=4, K=1), 1),
    ("tiny", dict(spec=synth.preset("tiny").frame, m=4, K=1), 4),
    ("mid", dict(spec=synth.FrameSpec(48, 40, 4096, 8.0, 200.0, 1.0, 1, seed=7), m=16, K=1), 5),
    ("layered", dict(spec=synth.FrameSpec(36, 28, 8192, 8.0, 2000.0, 0.5, 3, seed=5), m=32, K=3), 3),
    ("wide_m", dict(spec=synth.FrameSpec(20, 24, 4096, 6.0, 300.0, 1.0, 1, seed=9), m=48, K=2), 2),
    ("max_starts", dict(spec=synth.FrameSpec(12, 10, 512, 3.0, 60.0, 1.0, 1, seed=13), m=6, K=1), 64),
]


@pytest.mark.parametrize("name,cfg,starts", CASES)
def test_smle_matches_oracle(name, cfg, starts):
    dev = device()
    spec, m, K = cfg["spec"], cfg["m"], cfg["K"]
    _case(test="parity", frame=name, P=spec.P, m=m, K=K, starts=starts)
    f, z, n, params, op = _frame(spec, m, K, dev)
    _, loss, g, r, zc, nn = _run(f, z, n, params, op, starts, dev)
    st = r["state"]
    T = spec.T
    # the GPU's chosen points are as good as the oracle's: their FP64 loss is not above the
    # oracle's minimum by more than FP32 rounding
    Lg = OM.loss(zc, nn, g.t, g.alpha, g.active, r["hhat"], T)
    Lr = r["loss"]
    slack = 2e-3 * Lr + 1e-3
    worst = float(np.max((Lg - Lr) / slack))
    print("max (L_gpu - L_oracle) / slack:", worst)
    assert np.all(Lg <= Lr + slack)
    # the reported loss is the chosen points' loss
    np.testing.assert_allclose(loss, Lg, rtol=2e-3, atol=1e-3)
    # and, but for near-ties between starts, the same points
    same_act = (g.active == st.active).all(1)
    close = ((circ_abs(g.t - st.t, T) <= 0.5) | ~st.active).all(1)
    ok = same_act & close
    print("pixels with the oracle's points (0.5 bin):", ok.mean(), "failing:", int((~ok).sum()))
    assert ok.mean() >= 0.99


def test_smle_recovers_a_noiseless_surface():
    """z = Phi(theta*) uploaded as the sketch: every pixel returns theta*."""
    dev = device()
    T, m, rows, cols = 2048, 8, 16, 16
    P = rows * cols
    rng = np.random.default_rng(3)
    sig = 3.0
    o = int(np.ceil(6 * sig))
    irf = np.exp(-0.5 * (np.arange(-o, o + 1) / sig) ** 2)
    hhat = OM.irf_spectrum(irf, o, T, m)
    t = rng.uniform(0, T, (P, 1))
    alpha = rng.uniform(0.3, 0.9, (P, 1))
    zc = OM.model_sketch(t, alpha, np.ones((P, 1), bool), hhat, T)
    z = torch.from_numpy(np.stack([zc.real, zc.imag], -1).astype(np.float32)).to(dev)
    n = torch.full((P,), 800, dtype=torch.int32, device=dev)
    params = srt.Params.default(rows, cols, T, m, 1, iters=400)
    rec = srt.Reconstructor(params, dev)
    _case(test="noiseless", P=P)
    loss = rec.smle(z, n, torch.from_numpy(irf).to(dev), o, 4)
    tg, ag, actg = (x.cpu().numpy() for x in rec.state())
    torch.cuda.synchronize()
    assert actg.all()
    assert np.max(circ_abs(tg - t, T)) < 0.02
    np.testing.assert_allclose(ag, alpha, atol=2e-4)
    assert float(loss.max()) < 1e-2


def test_smle_outputs_through_finalize_and_repeat_calls():
    """finalize reads the chosen points; a second call on the same state gives the same bits."""
    dev = device()
    w = synth.preset("tiny")
    f, z, n, params, op = _frame(w.frame, w.m, w.K_max, dev)
    rec = srt.Reconstructor(params, dev)
    irf = torch.from_numpy(f.irf).to(dev)
    _case(test="repeat")
    l1 = rec.smle(z, n, irf, f.irf_origin, 3).clone()
    s1 = [x.clone() for x in rec.state()]
    out = rec.finalize(n)
    l2 = rec.smle(z, n, irf, f.irf_origin, 3)
    s2 = rec.state()
    torch.cuda.synchronize()
    assert torch.equal(l1, l2)
    for a, b in zip(s1, s2):
        assert torch.equal(a, b)
    assert rec.cur == 1
    d = out["depth"].cpu().numpy()
    act = out["active"].cpu().numpy().astype(bool)
    t = s1[0].cpu().numpy()
    np.testing.assert_array_equal(np.sort(np.where(act, d, np.inf), 1)[act.any(1)],
                                  np.sort(np.where(s1[2].cpu().numpy().astype(bool), t, np.inf), 1)[act.any(1)])
