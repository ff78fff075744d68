"""Sketched RT3D (SRT3D) on AMD Instinct MI355X.

Photon and histogram sketches (eq. 2-3) and the SRT3D reconstruction (eq. 8 with W = I plus
point-cloud and intensity denoising) run in hand-written HIP kernels of libsrt3d.so; this
package is the thin binding plus the serving loop.
"""
from ._lib import (  # noqa: F401
    EXPORTS,
    HistWorkspace,
    LIB_PATH,
    PRECISIONS,
    Params,
    Reconstructor,
    SRT3DError,
    cached_phase_table,
    events_workspace,
    hist_workspace,
    phase_indices,
    sketch_phases,
    phase_table,
    sketch,
    sketch_events,
    sketch_from_hist,
    sketch_route,
)
