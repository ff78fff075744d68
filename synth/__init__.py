"""Seeded synthetic single-photon lidar frames.

This package only draws inputs: scenes, photon time stamps, histograms and
request streams. It holds none of the sketching or reconstruction arithmetic,
so both the HIP path and the FP64 oracle can consume what it produces.
"""
from .frames import (  # noqa: F401
    Frame,
    FrameSpec,
    binned_gaussian_irf,
    histogram,
    make_frame,
    make_scene,
    draw_photons,
)
from .configs import PRESETS, preset  # noqa: F401
from .stream import Request, request_stream  # noqa: F401
