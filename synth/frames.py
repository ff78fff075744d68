"""Synthetic frames that follow the observation model of the paper.

Section 2, eq. (1): each photon of a pixel comes from surface k with
probability alpha_k (its stamp is the surface depth t_k plus a draw from the
impulse response h) or from the background with probability alpha_0 (its stamp
is uniform on {0, ..., T-1}).  Section 4 builds its synthetic frames from a
reference depth map at a range of mean photon counts per pixel and of
signal-to-background ratios; the reference scenes are not available, so
`make_scene` draws piecewise-planar scenes instead (a back wall, three
axis-aligned objects and, for layered frames, a front mesh with partial
coverage).

Scene geometry is drawn with numpy's PCG64 from `seed`; photons are drawn with a
torch generator on the requested device (seed + 1), so large frames are
produced where they will be consumed.  The random streams on CPU and GPU differ:
a test that compares two implementations feeds both the same tensors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

# Photons are drawn in blocks of this many pixels so that the random stream,
# and therefore the frame, does not depend on available memory.
CHUNK_PIXELS = 1 << 14


@dataclass(frozen=True)
class FrameSpec:
    rows: int
    cols: int
    T: int
    sigma: float          # IRF standard deviation in bins
    lam: float            # mean photons per pixel (signal + background)
    sbr: float            # frame-average signal-to-background ratio
    layers: int = 1       # 1: nearest surface per pixel; 2: netting in front; 3: layered scene
    seed: int = 0

    @property
    def P(self) -> int:
        return self.rows * self.cols


@dataclass
class Scene:
    depth: np.ndarray     # [P, L] float64, bins, surface depths (front to back)
    weight: np.ndarray    # [P, L] float64, share of the pixel's signal per surface (0 = absent)
    refl: np.ndarray      # [P, L] float64, reflectivity of each surface


@dataclass
class Frame:
    spec: FrameSpec
    scene: Scene
    stamps: torch.Tensor          # int32 [N], pixel-major
    offsets: torch.Tensor         # int64 [P + 1]
    counts: torch.Tensor          # int64 [P, L + 1] photons per surface, last column background
    sig_mean: np.ndarray          # [P, L] float64 expected signal photons per surface
    bg_mean: np.ndarray           # [P] float64 expected background photons
    irf: np.ndarray = field(default=None)   # float64 binned Gaussian impulse response
    irf_origin: int = 0

    @property
    def n(self) -> torch.Tensor:
        return self.offsets[1:] - self.offsets[:-1]


def binned_gaussian_irf(sigma: float) -> tuple[np.ndarray, int]:
    """Impulse response seen by the detector for a Gaussian pulse of std `sigma`.

    The generator rounds t + sigma*N(0,1) to the nearest bin, so for an integer
    depth the stamp offset d has probability Phi((d+1/2)/sigma) - Phi((d-1/2)/sigma).
    Returned on d = -o..o with o = ceil(6 sigma); the origin index is o.
    """
    o = int(math.ceil(6.0 * sigma))
    d = np.arange(-o, o + 1, dtype=np.float64)
    cdf = lambda u: 0.5 * (1.0 + np.vectorize(math.erf)(u / math.sqrt(2.0)))  # noqa: E731
    h = cdf((d + 0.5) / sigma) - cdf((d - 0.5) / sigma)
    return h, o


def _plane(rng, rows, cols, d0, gmax, ic, jc):
    gi, gj = rng.uniform(-gmax, gmax, size=2)
    ii, jj = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    return d0 + gi * (ii - ic) + gj * (jj - jc)


def _rect(rng, rows, cols):
    # clamped after the draw, so frames of two or more rows and columns draw what they always did
    h = min(rows, int(rng.integers(max(1, rows // 8), max(2, rows // 2) + 1)))
    w = min(cols, int(rng.integers(max(1, cols // 8), max(2, cols // 2) + 1)))
    i0 = int(rng.integers(0, rows - h + 1))
    j0 = int(rng.integers(0, cols - w + 1))
    return i0, j0, h, w


def make_scene(spec: FrameSpec) -> Scene:
    """Piecewise-planar scene: back wall plus three rectangles (plus a mesh if layered: a
    checkerboard mesh over object and wall for 3 layers, a netting with holes in front of the
    nearest surface for 2)."""
    rng = np.random.default_rng(spec.seed)
    R, C, T = spec.rows, spec.cols, spec.T
    lo, hi = 6.0 * spec.sigma, T - 6.0 * spec.sigma

    wall = _plane(rng, R, C, rng.uniform(0.6 * T, 0.8 * T), 0.25, (R - 1) / 2, (C - 1) / 2)
    r_wall = rng.uniform(0.5, 1.5)

    obj_depth = np.full((R, C), np.inf)
    obj_refl = np.zeros((R, C))
    d_range = (0.2 * T, 0.6 * T) if spec.layers == 1 else (0.35 * T, 0.5 * T)
    for _ in range(3):
        i0, j0, h, w = _rect(rng, R, C)
        d0 = rng.uniform(*d_range)
        box = rng.uniform() < 0.5            # a box face has no slope
        plane = _plane(rng, R, C, d0, 0.0 if box else 0.25, i0 + (h - 1) / 2, j0 + (w - 1) / 2)
        r = rng.uniform(0.5, 1.5)
        sub = (slice(i0, i0 + h), slice(j0, j0 + w))
        nearer = plane[sub] < obj_depth[sub]
        obj_depth[sub] = np.where(nearer, plane[sub], obj_depth[sub])
        obj_refl[sub] = np.where(nearer, r, obj_refl[sub])
    has_obj = np.isfinite(obj_depth)

    if spec.layers == 1:
        front = has_obj & (obj_depth < wall)
        depth = np.where(front, obj_depth, wall)[..., None]
        refl = np.where(front, obj_refl, r_wall)[..., None]
        weight = np.ones_like(depth)
    elif spec.layers == 3:
        net = _plane(rng, R, C, rng.uniform(0.15 * T, 0.22 * T), 0.05, (R - 1) / 2, (C - 1) / 2)
        r_net = rng.uniform(0.5, 1.5)
        cell = max(2, R // 16)
        ii, jj = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
        has_net = ((ii // cell + jj // cell) % 2) == 0
        f_net = np.where(has_net, 0.5, 0.0)
        rest = 1.0 - f_net
        f_obj = np.where(has_obj, 0.7 * rest, 0.0)
        f_wall = rest - f_obj
        depth = np.stack([np.where(has_net, net, 0.0), np.where(has_obj, obj_depth, 0.0), wall], -1)
        weight = np.stack([f_net, f_obj, f_wall], -1)
        refl = np.stack([np.full((R, C), r_net), obj_refl, np.full((R, C), r_wall)], -1)
    elif spec.layers == 2:
        # camouflage-like: a netting plane in front of most pixels, the object or the wall behind
        net = _plane(rng, R, C, rng.uniform(0.22 * T, 0.3 * T), 0.05, (R - 1) / 2, (C - 1) / 2)
        r_net = rng.uniform(0.5, 1.5)
        cell = max(2, R // 8)
        ii, jj = np.meshgrid(np.arange(R), np.arange(C), indexing="ij")
        has_net = ((ii % cell) != 0) | ((jj % cell) != 0)      # a grid of holes, one per cell
        front = has_obj & (obj_depth < wall)
        back = np.where(front, obj_depth, wall)
        r_back = np.where(front, obj_refl, r_wall)
        f_net = np.where(has_net, 0.4, 0.0)
        depth = np.stack([np.where(has_net, net, 0.0), back], -1)
        weight = np.stack([f_net, 1.0 - f_net], -1)
        refl = np.stack([np.full((R, C), r_net), r_back], -1)
    else:
        raise ValueError("layers must be 1, 2 or 3")

    depth = np.where(weight > 0, np.clip(depth, lo, hi), 0.0)
    L = depth.shape[-1]
    return Scene(depth.reshape(-1, L), weight.reshape(-1, L), refl.reshape(-1, L))


def expected_counts(spec: FrameSpec, scene: Scene) -> tuple[np.ndarray, np.ndarray]:
    """Mean signal photons per surface and mean background photons per pixel.

    The frame-average signal is lam*sbr/(1+sbr) and the background lam/(1+sbr);
    each surface's share is scaled by its reflectivity relative to the frame mean.
    """
    s = scene.weight * scene.refl
    rbar = s.sum(1).mean()
    sig = spec.lam * spec.sbr / (1.0 + spec.sbr) * s / rbar
    bg = np.full(spec.P, spec.lam / (1.0 + spec.sbr))
    return sig, bg


def draw_photons(spec: FrameSpec, scene: Scene, device="cpu"):
    """Poisson photon counts per surface and per-photon stamps, pixel-major CSR.

    A signal stamp is round(t_k + sigma*N(0,1)) mod T, a background stamp is
    uniform on {0..T-1}.  Within a pixel the stamps are in random order (a
    detector records a pixel's signal and background photons interleaved), by a
    sort on (pixel, random key).
    """
    device = torch.device(device)
    sig_mean, bg_mean = expected_counts(spec, scene)
    P, L, T = spec.P, scene.depth.shape[1], spec.T
    gen = torch.Generator(device=device)
    gen.manual_seed(spec.seed + 1)
    lam = torch.from_numpy(np.concatenate([sig_mean, bg_mean[:, None]], 1)).to(device)
    depth = torch.from_numpy(scene.depth).to(device=device, dtype=torch.float32)

    counts = torch.empty((P, L + 1), dtype=torch.int64, device=device)
    parts = []
    for p0 in range(0, P, CHUNK_PIXELS):
        p1 = min(P, p0 + CHUNK_PIXELS)
        c = torch.poisson(lam[p0:p1], generator=gen).to(torch.int64)
        counts[p0:p1] = c
        src = torch.repeat_interleave(torch.arange(c.numel(), device=device), c.reshape(-1))
        comp = src % (L + 1)
        pix = src // (L + 1)
        is_sig = comp < L
        d = depth[p0:p1].reshape(-1)[(pix * L + torch.clamp(comp, max=L - 1))]
        noise = torch.randn(src.numel(), generator=gen, device=device, dtype=torch.float32)
        bg = torch.randint(0, T, (src.numel(),), generator=gen, device=device, dtype=torch.int64)
        sig = torch.remainder(torch.round(d + spec.sigma * noise).to(torch.int64), T)
        st = torch.where(is_sig, sig, bg).to(torch.int32)
        del src, comp, is_sig, d, noise, bg, sig
        key = torch.randint(0, 1 << 31, (st.numel(),), generator=gen, device=device, dtype=torch.int64)
        order = torch.argsort(pix * (1 << 31) + key)
        parts.append(st[order])
        del pix, key, order, st
    stamps = torch.cat(parts) if parts else torch.empty(0, dtype=torch.int32, device=device)
    n = counts.sum(1)
    offsets = torch.zeros(P + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(n, 0)
    return stamps, offsets, counts, sig_mean, bg_mean


def make_frame(spec: FrameSpec, device="cpu") -> Frame:
    scene = make_scene(spec)
    stamps, offsets, counts, sig_mean, bg_mean = draw_photons(spec, scene, device)
    irf, o = binned_gaussian_irf(spec.sigma)
    return Frame(spec, scene, stamps, offsets, counts, sig_mean, bg_mean, irf, o)


def histogram(stamps: torch.Tensor, offsets: torch.Tensor, T: int) -> torch.Tensor:
    """Per-pixel ToA histogram (eq. 2 with T' = T), returned as int16 holding uint16 bits."""
    P = offsets.numel() - 1
    n = offsets[1:] - offsets[:-1]
    pix = torch.repeat_interleave(torch.arange(P, device=stamps.device), n)
    idx = pix * T + torch.remainder(stamps.to(torch.int64), T)
    h = torch.bincount(idx, minlength=P * T)
    if h.numel() and int(h.max()) > 0xFFFF:
        raise ValueError("histogram count exceeds uint16")
    h = torch.where(h > 0x7FFF, h - 0x10000, h)
    return h.to(torch.int16).reshape(P, T)


def hist_as_uint(h16: torch.Tensor) -> np.ndarray:
    """View an int16 histogram that holds uint16 bits as unsigned counts (host)."""
    return h16.cpu().numpy().view(np.uint16)
