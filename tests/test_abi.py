"""The C ABI library: it loads, exports every declared entry point, and rejects invalid
arguments on the host before touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_2203_00952_amd as srt
from paper_2203_00952_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srt3d.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srt3d_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libsrt3d.so is not built (run __graft_entry__.build())")
    return L._lib()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)


def test_version_and_strerror(lib):
    assert lib.srt3d_version() == 1
    assert lib.srt3d_strerror(0) == b"ok"
    assert lib.srt3d_strerror(-1) == b"invalid argument"
    assert lib.srt3d_strerror(-2) == b"workspace too small"


def test_noalloc_reconstruct_rejects_too_large_problems_on_the_host(lib):
    """srt3d_reconstruct_noalloc refuses a problem whose scratch exceeds its static array before
    any HIP call (the pointers below are never dereferenced), and names the reason."""
    assert lib.srt3d_strerror(L.SRT3D_ESCRATCH).startswith(b"problem needs more scratch")
    p = L._Params()
    lib.srt3d_params_default(ctypes.byref(p), 16, 16, 8192, 64, 1)
    assert lib.srt3d_init_workspace_bytes(ctypes.byref(p)) <= L.STATIC_SCRATCH_BYTES
    p.init_stride = 1                               # 8192 grid points: 4.2 MB of grid table
    assert lib.srt3d_init_workspace_bytes(ctypes.byref(p)) > L.STATIC_SCRATCH_BYTES
    st = L._State()
    fake = 0x1000
    for b in range(2):
        st.t[b] = st.alpha[b] = st.active[b] = fake
    st.hhat = st.scal = fake
    args = [ctypes.c_void_p(fake)] * 3 + [17, 8, ctypes.byref(p), ctypes.byref(st)] + [ctypes.c_void_p(0)] * 4
    assert lib.srt3d_reconstruct_noalloc(*args, None) == L.SRT3D_ESCRATCH
    p.K_max = 4                                     # invalid parameters are still EINVAL
    assert lib.srt3d_reconstruct_noalloc(*args, None) == L.SRT3D_EINVAL


def test_workspace_and_state_size_queries(lib):
    """srt3d_workspace_bytes agrees with the per-call queries; srt3d_state_bytes and
    srt3d_state_carve lay the state out as the header states (host arithmetic only)."""
    p = L._Params()
    lib.srt3d_params_default(ctypes.byref(p), 256, 256, 4096, 16, 1)
    P = 256 * 256
    ws = lambda which, PP=P: lib.srt3d_workspace_bytes(ctypes.byref(p), PP, which)   # noqa: E731
    assert ws(L.CALLS["reconstruct"]) == lib.srt3d_init_workspace_bytes(ctypes.byref(p)) > 0
    assert ws(L.CALLS["smle_weighted"]) == lib.srt3d_smle_weighted_workspace_bytes(ctypes.byref(p)) > 0
    for i, prec in enumerate(("hist_fp32", "hist_fp16x2", "hist_bf16x3")):
        assert ws(L.CALLS[prec]) == lib.srt3d_hist_workspace_bytes(4096, 16, i) > 0
    assert ws(L.CALLS["sketch"]) == 0
    assert ws(L.CALLS["reconstruct"], P + 1) == 0           # P must match rows * cols
    assert ws(99) == 0
    up = lambda b: (b + 255) // 256 * 256                   # noqa: E731
    # weighted SRT3D: n_w, the spectrum to harmonic 2m, then per pixel W's lower triangle by
    # columns, d (d + 1) / 2 floats (d = 2m) rounded up to a multiple of 4
    for m in (16, 5):
        lib.srt3d_params_default(ctypes.byref(p), 256, 256, 4096, m, 1)
        d = 2 * m
        tri = (d * (d + 1) // 2 + 3) // 4 * 4
        assert ws(L.CALLS["weighted_iterate"]) == 256 + up(d * 8) + P * tri * 4
    lib.srt3d_params_default(ctypes.byref(p), 256, 256, 4096, 16, 1)
    for K in (1, 2, 3):
        p.K_max = K
        PK = P * K
        expect = 4 * up(4 * PK) + 2 * up(PK) + up(8 * 16) + up(4 * L.NSCAL)
        n = lib.srt3d_state_bytes(ctypes.byref(p), P)
        assert n == expect
        st = L._State()
        base = 0x7f0000000000
        assert lib.srt3d_state_carve(ctypes.byref(st), ctypes.byref(p), ctypes.c_void_p(base), n) == L.SRT3D_OK
        offs = [st.t[0], st.t[1], st.alpha[0], st.alpha[1], st.active[0], st.active[1], st.hhat, st.scal]
        assert [o - base for o in offs] == [0, up(4 * PK), 2 * up(4 * PK), 3 * up(4 * PK), 4 * up(4 * PK),
                                            4 * up(4 * PK) + up(PK), 4 * up(4 * PK) + 2 * up(PK),
                                            4 * up(4 * PK) + 2 * up(PK) + up(128)]
        assert st.cur == 0
        assert lib.srt3d_state_carve(ctypes.byref(st), ctypes.byref(p), ctypes.c_void_p(base), n - 1) == L.SRT3D_ENOMEM
        assert lib.srt3d_state_carve(ctypes.byref(st), ctypes.byref(p), ctypes.c_void_p(base + 16), n) == L.SRT3D_EINVAL
    assert lib.srt3d_state_bytes(ctypes.byref(p), P - 1) == 0
    p.K_max = 4
    assert lib.srt3d_state_bytes(ctypes.byref(p), P) == 0


def test_params_default(lib):
    p = srt.Params.default(256, 256, 4096, 16)
    assert (p.iters, p.R, p.Rb, p.init_stride) == (50, 2, 1, 0)
    assert (p.eta_t, p.eta_a, p.lambda_z, p.tau_z, p.r_min) == (1.0, 1.0, 1.0, 0.0, 1.0)


def test_workspace_queries(lib):
    # split F planes (16-row column tiles x T), then G: FP64 [chunks of 32 bins, rounded up to a
    # multiple of 4][column tiles x 16], each part rounded up to 256 bytes
    G = 32 * 32 * 8
    assert lib.srt3d_hist_workspace_bytes(1024, 16, 0) == 32 * 1024 * 4 + G
    assert lib.srt3d_hist_workspace_bytes(1024, 16, 1) == 2 * 32 * 1024 * 2 + G
    assert lib.srt3d_hist_workspace_bytes(1024, 16, 2) == 3 * 32 * 1024 * 2 + G
    assert lib.srt3d_hist_workspace_bytes(96, 1, 0) == 16 * 96 * 4 + 4 * 16 * 8   # 3 chunks -> 4
    assert lib.srt3d_hist_workspace_bytes(1024, 33, 0) == 0
    assert lib.srt3d_hist_workspace_bytes(1024, 16, 3) == 0
    assert lib.srt3d_hist_workspace_bytes(16384, 4, 0) == 0
    p = L._Params()
    lib.srt3d_params_default(ctypes.byref(p), 32, 32, 1024, 4, 1)
    # per-workgroup maxima of n and a completion counter (256 bytes), the grid table: T=1024, m=4
    # -> stride 32, 32 grid points (2 column tiles) x 2 k-steps x 64 lanes of FP32 B-operand
    # fragments, then the atom's autocorrelation on 16 lags per column tile (FP32)
    assert lib.srt3d_init_workspace_bytes(ctypes.byref(p)) == 4096 * 4 + 256 + 2 * 2 * 64 * 4 + 2 * 16 * 4
    p.K_max = 4
    assert lib.srt3d_init_workspace_bytes(ctypes.byref(p)) == 0
    # event streams: G = min(ceil(N / 8192), 512) stream chunks, NB buckets of W pixels (W the
    # smaller of 2^ceil(log2(P) / 2) and 2^ceil(log2(ceil(P / 512)))); an int32 [NB][G] table,
    # int64 [NB + 1] bucket slots, int64 [P + 1] offsets and two int32 [N] streams, each rounded
    # up to 256 bytes
    up = lambda b: (b + 255) // 256 * 256
    ws = lambda N, P, G, NB: up(4 * NB * G) + up(8 * (NB + 1)) + up(8 * (P + 1)) + 2 * up(4 * max(N, 1))
    assert lib.srt3d_sketch_events_workspace_bytes(1000, 3000) == ws(1000, 3000, 1, 375)        # W = 8
    assert lib.srt3d_sketch_events_workspace_bytes(0, 1) == ws(0, 1, 1, 1)
    assert lib.srt3d_sketch_events_workspace_bytes(1 << 20, 1000) == ws(1 << 20, 1000, 128, 500)  # W = 2
    assert lib.srt3d_sketch_events_workspace_bytes(65_533_692, 65536) == ws(65_533_692, 65536, 512, 512)
    assert lib.srt3d_sketch_events_workspace_bytes(100, 2**21 + 1) == ws(100, 2**21 + 1, 1, 1025)  # W = 2048
    assert lib.srt3d_sketch_events_workspace_bytes(-1, 10) == 0
    assert lib.srt3d_sketch_events_workspace_bytes(10, 0) == 0
    assert lib.srt3d_sketch_events_workspace_bytes(2**31, 10) == 0
    assert lib.srt3d_sketch_events_workspace_bytes(10, 2**30 + 1) == 0


def test_invalid_arguments_rejected_on_host(lib):
    VP = ctypes.c_void_p
    fake = VP(0x1000)   # never dereferenced: validation fails first
    # P < 1, m > T/2, T too large, NULL table / outputs, acc without nacc, N < 0, misaligned z
    assert lib.srt3d_sketch(fake, 10, fake, 0, 1024, 4, fake, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 1024, 513, fake, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 16384, 4, fake, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 1024, 4, None, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 1024, 4, fake, None, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 1024, 4, fake, fake, fake, fake, None, None, None) == -1
    assert lib.srt3d_sketch(fake, -1, fake, 4, 1024, 4, fake, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch(fake, 10, fake, 4, 1024, 4, fake, VP(0x1004), fake, None, None, None, None) == -1
    for args in ((fake, 10, fake, 0, 1024, 4), (fake, 10, fake, 4, 1024, 33), (fake, 10, fake, 4, 16384, 4),
                 (fake, -1, fake, 4, 1024, 4)):
        assert lib.srt3d_sketch_binned(*args, fake, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch_binned(fake, 10, fake, 4, 1024, 4, None, fake, fake, None, None, None, None) == -1
    assert lib.srt3d_sketch_binned(fake, 10, fake, 4, 1024, 4, fake, fake, fake, fake, None, None, None) == -1
    assert lib.srt3d_phase_table(1, fake, None) == -1
    # fixed lane counts: only 4, 8, 16, 32 and 64, and the sketch's own checks
    for lanes in (0, 3, 5, 12, 128, -4):
        assert lib.srt3d_sketch_lanes(fake, 10, fake, 4, 1024, 4, fake, fake, fake, None, None, None, lanes,
                                      None) == -1
    assert lib.srt3d_sketch_lanes(fake, 10, fake, 4, 1024, 513, fake, fake, fake, None, None, None, 16, None) == -1
    assert lib.srt3d_sketch_lanes(fake, 10, fake, 4, 1024, 4, fake, None, fake, None, None, None, 16, None) == -1
    # phase export: the sketch's checks plus a NULL index buffer with photons
    assert lib.srt3d_sketch_phases(fake, 10, fake, 4, 1024, 4, fake, fake, fake, None, None) == -1
    assert lib.srt3d_sketch_phases(fake, 10, fake, 4, 1024, 513, fake, fake, fake, fake, None) == -1
    assert lib.srt3d_sketch_phases(fake, 10, fake, 0, 1024, 4, fake, fake, fake, fake, None) == -1
    assert lib.srt3d_sketch_phases(fake, 10, fake, 4, 1024, 4, fake, VP(0x1004), fake, fake, None) == -1
    # event streams: P < 1, m > T/2, NULL pixels with events, NULL workspace, misaligned or too
    # small workspace, N or P past the limits
    ws = VP(0x10000)
    assert lib.srt3d_sketch_events(fake, fake, 10, 0, 1024, 4, fake, fake, fake, None, None, None, ws, 1 << 20, None) == -1
    assert lib.srt3d_sketch_events(fake, fake, 10, 4, 1024, 513, fake, fake, fake, None, None, None, ws, 1 << 20,
                                   None) == -1
    assert lib.srt3d_sketch_events(None, fake, 10, 4, 1024, 4, fake, fake, fake, None, None, None, ws, 1 << 20, None) == -1
    assert lib.srt3d_sketch_events(fake, fake, 10, 4, 1024, 4, fake, fake, fake, None, None, None, None, 1 << 20,
                                   None) == -1
    assert lib.srt3d_sketch_events(fake, fake, 10, 4, 1024, 4, fake, fake, fake, None, None, None, VP(0x10010),
                                   1 << 20, None) == -1
    assert lib.srt3d_sketch_events(fake, fake, 10, 4, 1024, 4, fake, fake, fake, None, None, None, ws, 16, None) == -2
    assert lib.srt3d_sketch_events(fake, fake, 2**31, 4, 1024, 4, fake, fake, fake, None, None, None, ws, 1 << 20,
                                   None) == -1
    assert lib.srt3d_sketch_events(fake, fake, 10, 2**30 + 1, 1024, 4, fake, fake, fake, None, None, None, ws,
                                   1 << 20, None) == -1
    # histogram: T not a multiple of 32, m > 32, bad precision, misaligned pointer, small workspace
    assert lib.srt3d_hist_prepare(1000, 4, 0, fake, 1 << 20, None) == -1
    assert lib.srt3d_hist_prepare(1024, 4, 0, fake, 16, None) == -2
    assert lib.srt3d_sketch_from_hist(fake, 4, 1000, 4, 0, fake, 1 << 20, fake, fake, None) == -1
    assert lib.srt3d_sketch_from_hist(fake, 4, 1024, 33, 0, fake, 1 << 20, fake, fake, None) == -1
    assert lib.srt3d_sketch_from_hist(fake, 4, 1024, 4, 7, fake, 1 << 20, fake, fake, None) == -1
    assert lib.srt3d_sketch_from_hist(VP(0x1002), 4, 1024, 4, 0, fake, 1 << 20, fake, fake, None) == -1
    assert lib.srt3d_sketch_from_hist(fake, 4, 1024, 4, 0, fake, 16, fake, fake, None) == -2


def test_invalid_reconstruction_arguments(lib):
    fake = ctypes.c_void_p(0x1000)
    p = L._Params()
    lib.srt3d_params_default(ctypes.byref(p), 8, 8, 1024, 4, 1)
    st = L._State()
    for b in range(2):
        st.t[b] = st.alpha[b] = st.active[b] = 0x1000
    st.hhat = st.scal = 0x1000
    args = (fake, fake, fake, 5, 2, ctypes.byref(p), ctypes.byref(st), fake, 1 << 20, None)
    bad = [dict(K_max=4), dict(m=65), dict(R=4), dict(rows=0), dict(iters=-1), dict(eta_t=-1.0),
           dict(init_stride=1024), dict(T=16384), dict(birth_every=-1)]
    for change in bad:
        q = L._Params()
        ctypes.pointer(q)[0] = p
        for k, v in change.items():
            setattr(q, k, v)
        assert lib.srt3d_init(fake, fake, fake, 5, 2, ctypes.byref(q), ctypes.byref(st), fake, 1 << 20, None) == -1
    assert lib.srt3d_init(fake, fake, fake, 5, 5, *args[5:]) == -1            # origin outside irf
    assert lib.srt3d_init(fake, fake, fake, 0, 0, *args[5:]) == -1            # empty irf
    assert lib.srt3d_init(*args[:7], fake, 16, None) == -2                    # workspace too small
    # pixelwise estimator: starts outside [1, 64], NULL loss, small workspace
    for starts, loss in ((0, fake), (65, fake), (2, None)):
        assert lib.srt3d_smle(fake, fake, fake, 5, 2, ctypes.byref(p), starts, ctypes.byref(st), loss, fake, 1 << 20,
                              None) == -1
    assert lib.srt3d_smle(fake, fake, fake, 5, 2, ctypes.byref(p), 2, ctypes.byref(st), fake, fake, 16, None) == -2
    # precision weighting: m > 32 or 2 m >= T, witers outside [0, 1000], small workspace
    assert lib.srt3d_smle_weighted_workspace_bytes(ctypes.byref(p)) > 0
    for change in (dict(m=33, T=1024), dict(m=4, T=8)):
        q = L._Params()
        ctypes.pointer(q)[0] = p
        for k, v in change.items():
            setattr(q, k, v)
        assert lib.srt3d_smle_weighted_workspace_bytes(ctypes.byref(q)) == 0
        assert lib.srt3d_smle_weighted(fake, fake, fake, 5, 2, ctypes.byref(q), 2, 10, ctypes.byref(st), fake, fake,
                                       1 << 20, None) == -1
        assert lib.srt3d_weighted_fit(ctypes.byref(st), fake, fake, fake, 5, 2, ctypes.byref(q), 10, fake, fake,
                                      1 << 20, None) == -1
    for witers in (-1, 1001):
        assert lib.srt3d_weighted_fit(ctypes.byref(st), fake, fake, fake, 5, 2, ctypes.byref(p), witers, fake, fake,
                                      1 << 20, None) == -1
    assert lib.srt3d_weighted_fit(ctypes.byref(st), fake, fake, fake, 5, 2, ctypes.byref(p), 10, fake, fake, 16,
                                  None) == -2
    st2 = L._State()
    ctypes.pointer(st2)[0] = st
    st2.cur = 2
    assert lib.srt3d_step(ctypes.byref(st2), fake, fake, ctypes.byref(p), 0, None) == -1
    assert lib.srt3d_step(ctypes.byref(st), fake, fake, ctypes.byref(p), 4, None) == -1
    assert lib.srt3d_step(ctypes.byref(st), None, fake, ctypes.byref(p), 3, None) == -1    # birth needs z
    st2.cur = 0
    st2.scal = None
    assert lib.srt3d_iterate(ctypes.byref(st2), fake, fake, ctypes.byref(p), 1, None) == -1
    assert lib.srt3d_phase_table(16384, fake, None) == -1
    assert lib.srt3d_phase_indices(fake, 10, 1024, 0, fake, None) == -1


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(TypeError):
        srt.sketch(torch.zeros(4, dtype=torch.int32), torch.zeros(3, dtype=torch.int64), 64, 4)


def test_auto_sketch_route():
    """"auto" takes the binned pass from 0.04 T photons per pixel (m <= 32), else the photon pass."""
    assert srt.sketch_route(65536 * 1000, 65536, 4096, 16) == "binned"
    assert srt.sketch_route(65536 * 100, 65536, 4096, 16) == "photon"
    assert srt.sketch_route(1639, 10, 4096, 16) == "binned"          # 0.04 T P = 1638.4
    assert srt.sketch_route(1638, 10, 4096, 16) == "photon"
    assert srt.sketch_route(10 ** 9, 10, 4096, 33) == "photon"
