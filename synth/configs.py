"""Named workloads: frame shape, photon statistics and sketch size.

Each preset fixes the frame (FrameSpec) plus the sketch size m, the number of
surfaces per pixel the reconstruction allows (K_max) and its iteration count.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

from .frames import FrameSpec


@dataclass(frozen=True)
class Workload:
    name: str
    frame: FrameSpec
    m: int
    K_max: int
    iters: int
    description: str
    r_min: float = 1.0          # photons below which a reconstructed point is removed

    def with_seed(self, seed: int) -> "Workload":
        return replace(self, frame=replace(self.frame, seed=seed))


PRESETS = {
    "tiny": Workload(
        "tiny", FrameSpec(32, 32, 1024, 5.0, 10.0, 1.0, 1, seed=1), m=4, K_max=1, iters=50,
        description="32x32 px, T=1024, sigma=5, ~10 photons/px, SBR=1, m=4"),
    "throughput": Workload(
        "throughput", FrameSpec(256, 256, 4096, 8.0, 1000.0, 1.0, 1, seed=21), m=16, K_max=1,
        iters=50, description="256x256 px, T=4096, sigma=8, ~1000 photons/px, SBR=1, m=16, 50 iterations"),
    "throughput_sbr0.1": Workload(
        "throughput_sbr0.1", FrameSpec(256, 256, 4096, 8.0, 1000.0, 0.1, 1, seed=20), m=16,
        K_max=1, iters=50, description="as throughput, SBR=0.1"),
    "throughput_sbr10": Workload(
        "throughput_sbr10", FrameSpec(256, 256, 4096, 8.0, 1000.0, 10.0, 1, seed=22), m=16,
        K_max=1, iters=50, description="as throughput, SBR=10"),
    "precision": Workload(
        "precision", FrameSpec(256, 256, 1024, 5.0, 4000.0, 1.0, 1, seed=3), m=16, K_max=1,
        iters=0, description="256x256 uint16 histograms, T=1024, ~4000 photons/px, m=16"),
    "billion": Workload(
        "billion", FrameSpec(512, 512, 8192, 8.0, 4000.0, 0.5, 3, seed=5), m=32, K_max=3,
        iters=50, description="512x512 px, T=8192, <=3 surfaces/px, ~4000 photons/px, SBR=0.5, m=32",
        r_min=100.0),
    "camouflage": Workload(
        "camouflage", FrameSpec(32, 32, 153, 2.0, 200.0, 2.0, 2, seed=11), m=10, K_max=2,
        iters=50, description="32x32 px, T=153, two surfaces on most pixels (netting in front), "
                              "~200 photons/px, SBR=2, m=10 (the shape of the camouflage frame of Section 4)",
        r_min=5.0),
}


def preset(name: str) -> Workload:
    return PRESETS[name]
