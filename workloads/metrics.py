"""Reporting helpers: error against a reference frame, photocentres, px -> cm/s.

Used by the tests and the benchmark to state every result the way the paper
states its requirement (Sec. 1 and Sec. 2.2): a photocentre residual in
pixels and in radial-velocity units.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0


def px_to_mps(dx_px: float, lam_nm: float, dxdlam_px_per_nm: float) -> float:
    """Velocity that moves a line by dx_px: dv = c dx / (lambda dx/dlambda)."""
    return C_LIGHT * dx_px / (lam_nm * dxdlam_px_per_nm)


def px_to_cms_sampling(dx_px: float, R: float, px_per_resel: float) -> float:
    """Same conversion when the dispersion is given as R and px per resolution
    element: dx/dlambda = px_per_resel / (lambda / R)."""
    return 100.0 * C_LIGHT * dx_px / (R * px_per_resel)


def max_rel_err(test: np.ndarray, ref: np.ndarray) -> float:
    """max |test - ref| / max |ref| over the frame."""
    peak = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(np.asarray(test, np.float64) - ref)) / peak) if peak > 0 else 0.0


def centroid(img: np.ndarray, i0: int = 0, j0: int = 0):
    """(x, y) intensity-weighted centroid of a cut-out whose [0, 0] is pixel (i0, j0)."""
    img = np.asarray(img, np.float64)
    tot = img.sum()
    jj, ii = np.indices(img.shape)
    return (float((img * (ii + i0)).sum() / tot), float((img * (jj + j0)).sum() / tot))


def aliasing_level(frame: np.ndarray, scene, margin_px: int = 12) -> dict:
    """Aliasing of a flat field rendered from discrete SFIs (Fig. 4): the
    flux of a straight trace with a constant spectrum and uniform dispersion
    is constant along x, so its relative RMS along the central row and along
    the column sums, away from the trace ends, is the aliasing ripple.  The
    photon-noise level is 1 / sqrt(mean count) of the same quantity."""
    tr = scene.traces[0]
    xs, xe = tr.cx[0] - tr.cx[1], tr.cx[0] + tr.cx[1]
    cols = np.arange(int(np.ceil(xs)) + margin_px, int(np.floor(xe)) - margin_px)
    yc = int(np.floor(tr.cy[0] + 0.5))
    row = np.asarray(frame[yc, cols], np.float64)
    col = np.asarray(frame[:, cols], np.float64).sum(0)
    return {"row_ripple": float(np.std(row) / row.mean()),
            "row_photon": float(1.0 / np.sqrt(row.mean())),
            "col_ripple": float(np.std(col) / col.mean()),
            "col_photon": float(1.0 / np.sqrt(col.mean())),
            "row_mean": float(row.mean()), "columns": int(cols.size)}
