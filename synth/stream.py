"""Seeded stream of reconstruction requests with Poisson arrivals.

Array sizes are drawn from {32^2, 128^2, 256^2, 512^2}, mean photons per pixel
from U[10, 2000], T = 2048 and m uniform on {8..32}; each request asks for a
sketch plus `iters` iterations.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .frames import FrameSpec

SIZES = (32, 128, 256, 512)


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    frame: FrameSpec
    m: int
    iters: int


def request_stream(seed: int, count: int, rate_hz: float, iters: int = 20, T: int = 2048,
                   sigma: float = 8.0, sbr: float = 1.0, sizes=SIZES) -> list[Request]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate_hz)
        side = int(sizes[int(rng.integers(0, len(sizes)))])
        lam = float(rng.uniform(10.0, 2000.0))
        m = int(rng.integers(8, 33))
        spec = FrameSpec(side, side, T, sigma, lam, sbr, 1, seed=int(rng.integers(1, 2**31 - 2)))
        out.append(Request(rid, t, spec, m, iters))
    return out
