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


def stratified_pixels(frame: np.ndarray, tw: int, th: int, *, node_x=(), node_y=(),
                      n_each: int = 40, seed: int = 0, carry_rows: int = 16):
    """Pixels to check a rendered frame at, drawn from the places where a tiled
    renderer's case logic lives (all among lit pixels, >= 1e-3 of the peak,
    except the last group): rows at tile boundaries (multiples of th, +-1);
    rows where a tile's carried rows end (th k + carry_rows, +-1); columns at
    tile-column edges (multiples of tw, +-1); lines within one pixel of the
    given PSF node-cell boundaries (node_x columns, node_y rows); the
    brightest pixels; the two ends of every lit row band's extent in x (trace
    ends); and pixels anywhere.  Returns (px, py) int arrays without repeats."""
    rng = np.random.default_rng(seed)
    f = np.asarray(frame)
    ny, nx = f.shape
    peak = float(f.max())
    lit = f > 1e-3 * peak
    jj, ii = np.nonzero(lit)
    groups = []

    def take(mask_idx):
        if mask_idx.size == 0:
            return
        sel = rng.choice(mask_idx.size, size=min(n_each, mask_idx.size), replace=False)
        groups.append(mask_idx[sel])

    near = lambda v, m: (np.abs(((v + 1) % m) - 1) <= 1)  # v mod m in {m-1, 0, 1}
    take(np.nonzero(near(jj, th))[0])
    take(np.nonzero(np.abs(((jj - carry_rows) % th + 1) % th - 1) <= 1)[0])
    take(np.nonzero(near(ii, tw))[0])
    if len(node_x):
        nxl = np.asarray(node_x, float)
        take(np.nonzero(np.min(np.abs(ii[:, None] - nxl[None, :]), axis=1) <= 1.0)[0])
    if len(node_y):
        nyl = np.asarray(node_y, float)
        take(np.nonzero(np.min(np.abs(jj[:, None] - nyl[None, :]), axis=1) <= 1.0)[0])
    bright = np.nonzero(f[jj, ii] > 0.3 * peak)[0]
    take(bright)
    # trace ends: the outermost lit columns of lit rows
    ends = []
    for j in np.unique(jj)[:: max(1, np.unique(jj).size // n_each)]:
        cols = ii[jj == j]
        ends += [np.nonzero((jj == j) & (ii == cols.min()))[0][0],
                 np.nonzero((jj == j) & (ii == cols.max()))[0][0]]
    if ends:
        groups.append(np.asarray(ends[: 2 * n_each]))
    idx = np.unique(np.concatenate(groups)) if groups else np.zeros(0, int)
    px, py = ii[idx], jj[idx]
    rx, ry = rng.integers(0, nx, n_each), rng.integers(0, ny, n_each)
    key = np.unique(np.concatenate([py, ry]).astype(np.int64) * nx + np.concatenate([px, rx]))
    return (key % nx).astype(np.int64), (key // nx).astype(np.int64)


def line_windows(frame: np.ndarray, n: int = 6, half: int = 2, seed: int = 0):
    """Corners (i0, j0) of n (2 half + 1)^2 windows centred on local maxima of
    the frame (a pixel brighter than its 8 neighbours, above 0.2 of the peak),
    away from the edges: isolated line images for photocentre checks."""
    f = np.asarray(frame, np.float64)
    c = f[1:-1, 1:-1]
    is_max = np.ones_like(c, bool)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if dj or di:
                is_max &= c > f[1 + dj:f.shape[0] - 1 + dj, 1 + di:f.shape[1] - 1 + di]
    is_max &= c > 0.2 * f.max()
    jj, ii = np.nonzero(is_max)
    jj, ii = jj + 1, ii + 1
    ok = (jj >= half + 1) & (jj < f.shape[0] - half - 1) & (ii >= half + 1) & (ii < f.shape[1] - half - 1)
    jj, ii = jj[ok], ii[ok]
    rng = np.random.default_rng(seed)
    sel = rng.choice(jj.size, size=min(n, jj.size), replace=False) if jj.size else []
    return [(int(ii[s]) - half, int(jj[s]) - half) for s in sel]


def dispersion_at(scene, x: float, y: float):
    """(lambda nm, dx/dlambda px/nm) of the trace passing nearest to (x, y):
    t solving x(t) = x by Newton steps on the format polynomial."""
    best = None
    P = np.polynomial.polynomial
    for tr in scene.traces:
        cx, cy = np.asarray(tr.cx, float), np.asarray(tr.cy, float)
        x_lo, x_hi = P.polyval(-1.0, cx), P.polyval(1.0, cx)
        if not (min(x_lo, x_hi) <= x <= max(x_lo, x_hi)):
            continue
        t = 2.0 * (x - x_lo) / (x_hi - x_lo) - 1.0
        dcx = P.polyder(cx)
        for _ in range(30):
            t -= (P.polyval(t, cx) - x) / P.polyval(t, dcx)
        d = abs(P.polyval(t, cy) - y)
        if best is None or d < best[0]:
            lam = 0.5 * (t * (tr.lmax - tr.lmin) + tr.lmin + tr.lmax)
            best = (d, lam, P.polyval(t, dcx) * 2.0 / (tr.lmax - tr.lmin))
    if best is None:
        return float("nan"), float("nan")
    return float(best[1]), float(best[2])
