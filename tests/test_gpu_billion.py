"""Full-size layered frame: 512x512 px, T = 8192, up to 3 surfaces per pixel, ~4000 photons per
pixel (~1.05e9 stamps), m = 32.  Sketch parity on sampled pixels; SRT3D parity for each stage
and for 5 whole iterations from a shared initialisation on the full frame (the oracle's full
50-iteration run at this size takes too long for a test)."""
import numpy as np
import pytest
import torch

import paper_2203_00952_amd as srt
import synth
from oracle import model as OM
from oracle import sketch as OS
from oracle import srt3d as O
from tests.gpu_common import circ_abs, device, sketch_violations, to_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def billion():
    dev = device()
    w = synth.preset("billion")
    print("case billion: generating frame", flush=True)
    f = synth.make_frame(w.frame, device=dev)
    z, n = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m)
    torch.cuda.synchronize()
    return w, f, z, n


def test_billion_sketch_sampled_pixels(billion):
    w, f, z, n = billion
    print("case billion sketch, photons", f.stamps.numel(), flush=True)
    assert f.stamps.numel() > 1.0e9
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(w.frame.P, 600, replace=False))
    st_np = f.stamps.cpu().numpy()
    zr, nr = OS.sketch(st_np, f.offsets.cpu().numpy(), w.frame.T, w.m, pixels=sel)
    np.testing.assert_array_equal(n.cpu().numpy()[sel], nr)
    bad, err, tol = sketch_violations(to_complex(z)[sel], zr, nr)
    print("max err/tol", float(np.max(err / tol)))
    assert not bad.any()


def test_billion_binned_sketch_sampled_pixels(billion):
    """The binned route (the benchmark's sketch) on the same frame: sampled pixels against the
    oracle, every pixel against the photon route within twice the rule."""
    w, f, z, n = billion
    print("case billion binned sketch", flush=True)
    zb, nb = srt.sketch(f.stamps, f.offsets, w.frame.T, w.m, method="binned")
    torch.cuda.synchronize()
    assert torch.equal(nb, n)
    rng = np.random.default_rng(6)
    sel = np.sort(rng.choice(w.frame.P, 600, replace=False))
    st_np = f.stamps.cpu().numpy()
    zr, nr = OS.sketch(st_np, f.offsets.cpu().numpy(), w.frame.T, w.m, pixels=sel)
    bad, err, tol = sketch_violations(to_complex(zb)[sel], zr, nr)
    print("max err/tol", float(np.max(err / tol)))
    assert not bad.any()
    nn = n.cpu().numpy()
    floor = 1.0 / np.sqrt(np.maximum(nn, 1))[:, None]
    zp = to_complex(z)
    d = np.abs(to_complex(zb) - zp) / (2e-5 * np.maximum(np.abs(zp), floor))
    print("binned vs photon, max |dz| / (2 tol) =", float(d.max()))
    assert d.max() <= 1.0


def test_billion_stages_and_iterations(billion):
    w, f, z, n = billion
    dev = z.device
    spec = w.frame
    params = srt.Params.default(spec.rows, spec.cols, spec.T, w.m, w.K_max, r_min=w.r_min)
    op = O.Params(spec.T, w.m, w.K_max, r_min=w.r_min)
    zc, nn = to_complex(z), n.cpu().numpy().astype(np.int64)
    hhat = OM.irf_spectrum(f.irf, f.irf_origin, spec.T, w.m)
    tau_z = O.default_tau_z(f.irf, f.irf_origin, op)
    gam = O.step_sizes(nn, hhat, op)
    rec = srt.Reconstructor(params, dev)
    irf = torch.from_numpy(f.irf).to(dev)
    print("case billion init", flush=True)
    rec.init(z, n, irf, f.irf_origin)
    torch.cuda.synchronize()
    st0 = O.init_points(zc, nn, hhat, op)
    t, a, act = (x.cpu().numpy() for x in rec.state())
    same = (t == st0.t).all(1)
    print("init identical picks", same.mean())
    assert same.mean() >= 0.999

    def upload(st):
        rec.set_state(torch.from_numpy(st.t), torch.from_numpy(st.alpha), torch.from_numpy(st.active))

    def download():
        torch.cuda.synchronize()
        t, a, act = (x.cpu().numpy() for x in rec.state())
        return O.State(t.astype(np.float64), a.astype(np.float64), act.astype(bool))

    st = O.data_step(st0, zc, nn, hhat, op, *gam)
    st = O.depth_denoise(st, spec.rows, spec.cols, op, tau_z)
    refs = {"data": O.data_step(st, zc, nn, hhat, op, *gam),
            "depth": O.depth_denoise(st, spec.rows, spec.cols, op, tau_z),
            "intensity": O.intensity_denoise(st, nn, spec.rows, spec.cols, op, tau_z)}
    for stage, r in refs.items():
        print("case billion stage", stage, flush=True)
        upload(st)
        rec.step(stage, z, n)
        g = download()
        ok = ((g.active == r.active).all(1) & ((circ_abs(g.t - r.t, spec.T) <= 2e-3) | ~r.active).all(1)
              & ((np.abs(g.alpha - r.alpha) <= 1e-4) | ~r.active).all(1))
        print(stage, ok.mean())
        assert ok.mean() >= 0.999
    print("case billion 5 iterations", flush=True)
    upload(st0)
    rec.iterate(z, n, 5)
    out = rec.finalize(n)
    torch.cuda.synchronize()
    r = O.iterate(st0, zc, nn, hhat, spec.rows, spec.cols, op, tau_z, 5)
    d, _, act_r = O.output(r, nn)
    dg, ag = out["depth"].cpu().numpy(), out["active"].cpu().numpy().astype(bool)
    ok = (ag == act_r).all(1) & ((circ_abs(dg - d, spec.T) <= 1.0) | ~act_r).all(1)
    print("5 iterations: pixels within 1 bin", ok.mean())
    assert ok.mean() >= 0.999
