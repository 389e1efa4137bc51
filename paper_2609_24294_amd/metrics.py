"""Host-side accuracy and size reporting (not timed, not on the GPU path).

Relative error as the paper defines it (Section IV-F): eps = ||x - xhat|| /
||x|| with x the original and xhat the reconstructed values; the paper
reports its distribution over all 4x4x4 blocks and the mean (Section V-C).
Here the norm is the Euclidean one, taken per block over the block's real
(unpadded) values; blocks with ||x|| = 0 are skipped.  The global error over
the whole field and pointwise |x - xhat| / |x| statistics are reported too.
"""
from __future__ import annotations

import numpy as np


def _pad_to_blocks(a: np.ndarray, fill=0.0):
    nz, ny, nx = a.shape
    pz, py, px = (-nz) % 4, (-ny) % 4, (-nx) % 4
    return np.pad(a, ((0, pz), (0, py), (0, px)), constant_values=fill)


def _block_sums(a: np.ndarray) -> np.ndarray:
    """Sum over each 4x4x4 block of a padded (4A, 4B, 4C) array -> (A, B, C)."""
    z, y, x = a.shape
    return a.reshape(z // 4, 4, y // 4, 4, x // 4, 4).sum(axis=(1, 3, 5))


def block_relative_errors(x: np.ndarray, xhat: np.ndarray) -> np.ndarray:
    """Per-block ||x_b - xhat_b||_2 / ||x_b||_2 of a (nz, ny, nx) field, over real
    values only, for blocks with ||x_b|| > 0 (a flat array, block order)."""
    x = np.asarray(x, np.float64)
    d = x - np.asarray(xhat, np.float64)
    num = _block_sums(_pad_to_blocks(d * d))
    den = _block_sums(_pad_to_blocks(x * x))
    ok = den > 0
    return np.sqrt(num[ok] / den[ok])


def error_report(x: np.ndarray, xhat: np.ndarray, pointwise: bool = True) -> dict:
    """Mean/max per-block relative error, global error and (optionally)
    pointwise relative error statistics of a 3-D field."""
    x64 = np.asarray(x, np.float64)
    eb = block_relative_errors(x64, xhat)
    d = x64 - np.asarray(xhat, np.float64)
    out = {
        "block_mean": float(eb.mean()) if eb.size else 0.0,
        "block_max": float(eb.max()) if eb.size else 0.0,
        "global": float(np.sqrt((d * d).sum() / max((x64 * x64).sum(), 1e-300))),
    }
    if pointwise:
        nz = x64 != 0
        r = np.abs(d[nz]) / np.abs(x64[nz])
        out["point_mean"] = float(r.mean()) if r.size else 0.0
        out["point_max"] = float(r.max()) if r.size else 0.0
    return out


def bytes_reduction(float32_values: int, coded_bytes: int) -> float:
    """float32 bytes divided by the coded bytes (padding included)."""
    return 4.0 * float32_values / float(coded_bytes)
