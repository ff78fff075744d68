"""Helpers shared by the GPU parity tests (comparison rules, frame construction)."""
import numpy as np
import torch

SKETCH_REL = 1e-5   # |z_gpu - z_ref| <= SKETCH_REL * max(|z_ref|, n^-1/2) per (pixel, harmonic)


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def to_complex(z: torch.Tensor) -> np.ndarray:
    """[..., m, 2] float32 -> complex128 [..., m]."""
    a = z.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def sketch_violations(z_gpu: np.ndarray, z_ref: np.ndarray, n: np.ndarray):
    """Entries breaking the sketch rule.  The floor n^-1/2 is the spread of the empirical
    characteristic function (eq. 5); a pixel with n = 0 must be exactly zero."""
    n = np.asarray(n, dtype=np.float64)
    floor = np.where(n > 0, 1.0 / np.sqrt(np.maximum(n, 1.0)), 0.0)[:, None]
    tol = SKETCH_REL * np.maximum(np.abs(z_ref), floor)
    err = np.abs(z_gpu - z_ref)
    bad = err > tol
    bad |= (n[:, None] == 0) & (z_gpu != 0)
    return bad, err, tol


def csr(pixels, device):
    stamps = np.concatenate([np.asarray(p, dtype=np.int64) for p in pixels]) if len(pixels) else np.zeros(0)
    offsets = np.zeros(len(pixels) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in pixels])
    return (torch.from_numpy(stamps.astype(np.int32)).to(device), torch.from_numpy(offsets).to(device),
            stamps, offsets)


def circ_abs(d, T):
    d = np.mod(d, T)
    return np.minimum(d, T - d)
