"""Sketch of photon time stamps, Section 2, eq. (3), and of histograms, eq. (2).

z_l = (1/n) * sum_p exp(+i * w_l * x_p),   w_l = 2*pi*l/T,   l = 1..m

The frequencies are those of the sampling scheme of Section 2 (w_l = 2 pi l/T),
and l runs over 1..m as eq. (3) states.  The phase w_l * x_p is reduced exactly:
k = (l * x_p) mod T is an integer and the angle is 2*pi*k/T, so cos/sin are
evaluated on [0, 2*pi) in FP64.  A stamp outside [0, T) is folded by the
mathematical modulus (exp(i w_l x) has period T in x).  A pixel without photons
has n = 0 and z = 0 (eq. (8) gives it zero data weight).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np


def phase_indices(x, T: int, m: int) -> np.ndarray:
    """Exact integer phase indices k[l-1, p] = (l * x_p) mod T, l = 1..m."""
    x = np.mod(np.asarray(x, dtype=np.int64), T)
    ell = np.arange(1, m + 1, dtype=np.int64)
    return np.mod(ell[:, None] * x[None, :], T)


def sketch_loop(x, T: int, m: int):
    """Pure-Python per-photon sketch of one pixel with correctly rounded sums.

    Returns (z, n) with z a list of m complex numbers.
    """
    xs = [int(v) % T for v in x]
    n = len(xs)
    z = []
    for ell in range(1, m + 1):
        ang = [2.0 * math.pi * ((ell * v) % T) / T for v in xs]
        re = math.fsum(math.cos(a) for a in ang)
        im = math.fsum(math.sin(a) for a in ang)
        z.append(complex(re / n, im / n) if n else 0j)
    return z, n


def sketch_sums(stamps, offsets, T: int, m: int, pixels=None):
    """Unnormalised sums S[p, l-1] = sum over the pixel's photons of exp(i w_l x).

    stamps: int [N] pixel-major; offsets: int [P+1].  `pixels` optionally selects
    a subset of pixels (their rows are returned in that order).
    Returns (S complex128 [P', m], n int64 [P']).
    """
    stamps = np.asarray(stamps)
    offsets = np.asarray(offsets, dtype=np.int64)
    P = offsets.size - 1
    pix = np.arange(P) if pixels is None else np.asarray(pixels, dtype=np.int64)
    lo, hi = offsets[pix], offsets[pix + 1]
    n = np.maximum(hi - lo, 0)
    owner = np.repeat(np.arange(pix.size), n)
    if pixels is None:
        x = np.mod(stamps[offsets[0]:offsets[-1]].astype(np.int64), T)
    else:
        idx = (np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
               if pix.size else np.zeros(0, np.int64))
        x = np.mod(stamps[idx].astype(np.int64), T)
    S = np.zeros((pix.size, m), dtype=np.complex128)
    for ell in range(1, m + 1):
        ang = 2.0 * np.pi * np.mod(ell * x, T) / T
        S[:, ell - 1] = (np.bincount(owner, weights=np.cos(ang), minlength=pix.size)
                         + 1j * np.bincount(owner, weights=np.sin(ang), minlength=pix.size))
    return S, n


def normalise(S: np.ndarray, n: np.ndarray) -> np.ndarray:
    """z = S / n, with z = 0 where n = 0."""
    z = np.zeros_like(S)
    nz = n > 0
    z[nz] = S[nz] / n[nz, None]
    return z


def sketch(stamps, offsets, T: int, m: int, pixels=None):
    """Per-pixel sketch z [P', m] complex128 and photon count n [P'] (eq. 3)."""
    S, n = sketch_sums(stamps, offsets, T, m, pixels)
    return normalise(S, n), n


def sketch_event_sums(pix, stamps, P: int, T: int, m: int):
    """Unnormalised sums of an arrival-order event stream (Section 2: the sketch is updated
    online, photon by photon, as each one arrives).

    Event e = (pix[e], stamps[e]) adds exp(i w_l x_e) to pixel pix[e], in stream order.  An event
    whose pixel index lies outside [0, P) belongs to no pixel: it is dropped and counted.  Stamps
    are folded as in sketch_sums.  Returns (S complex128 [P, m], n int64 [P], dropped, folded)
    with `folded` the number of kept events whose stamp lay outside [0, T).
    """
    pix = np.asarray(pix, dtype=np.int64)
    raw = np.asarray(stamps, dtype=np.int64)
    keep = (pix >= 0) & (pix < P)
    dropped = int(np.count_nonzero(~keep))
    pix, raw = pix[keep], raw[keep]
    folded = int(np.count_nonzero((raw < 0) | (raw >= T)))
    x = np.mod(raw, T)
    S = np.zeros((P, m), dtype=np.complex128)
    for ell in range(1, m + 1):
        ang = 2.0 * np.pi * np.mod(ell * x, T) / T
        col = np.zeros(P, dtype=np.complex128)
        np.add.at(col, pix, np.cos(ang) + 1j * np.sin(ang))     # one update per event, in order
        S[:, ell - 1] = col
    n = np.bincount(pix, minlength=P).astype(np.int64)
    return S, n, dropped, folded


def sketch_events(pix, stamps, P: int, T: int, m: int):
    """Per-pixel sketch z [P, m] and photon count n [P] of an event stream (see sketch_event_sums)."""
    S, n, _, _ = sketch_event_sums(pix, stamps, P, T, m)
    return normalise(S, n), n


def dft_columns(T: int, m: int) -> np.ndarray:
    """F[t, l-1] = exp(i w_l t) for t = 0..T-1 with exact phase reduction."""
    t = np.arange(T, dtype=np.int64)
    ell = np.arange(1, m + 1, dtype=np.int64)
    return np.exp(1j * 2.0 * np.pi * np.mod(t[:, None] * ell[None, :], T) / T)


def sketch_hist(H, m: int):
    """Sketch of per-pixel histograms with unit bins [t, t+1), t = 0..T-1 (eq. 2).

    H: counts [P, T].  S = H @ F, n = row sums, z = S / n.
    """
    H = np.asarray(H, dtype=np.float64)
    T = H.shape[1]
    S = H @ dft_columns(T, m)
    n = np.rint(H.sum(1)).astype(np.int64)
    return normalise(S, n), n
