"""Post-processing of density fields: contour extraction and contact angle.

The paper does not say how it measured the contact angle (Fig. 3).  The reading
used here: take the rho = level contour by linear interpolation along grid
edges, drop points within ``skip`` rows of the wall plane, fit a circle by
algebraic least squares (Kasa fit) and take cos(theta) = (y_w - y_c) / R, with
the wall plane at y_w = 0.5 (halfway bounce-back next to solid row 0).
"""
from __future__ import annotations

import numpy as np


def contour_points(rho: np.ndarray, level: float, fluid: np.ndarray | None = None):
    """Points where rho crosses ``level`` on horizontal and vertical grid edges."""
    ny, nx = rho.shape
    ok = np.ones_like(rho, bool) if fluid is None else fluid.astype(bool)
    d = rho - level
    pts = []
    # horizontal edges (x, y) - (x+1, y), not wrapping
    a, b = d[:, :-1], d[:, 1:]
    m = (a * b < 0) & ok[:, :-1] & ok[:, 1:]
    yy, xx = np.nonzero(m)
    t = a[yy, xx] / (a[yy, xx] - b[yy, xx])
    pts.append(np.stack([xx + t, yy.astype(float)], 1))
    # vertical edges (x, y) - (x, y+1)
    a, b = d[:-1, :], d[1:, :]
    m = (a * b < 0) & ok[:-1, :] & ok[1:, :]
    yy, xx = np.nonzero(m)
    t = a[yy, xx] / (a[yy, xx] - b[yy, xx])
    pts.append(np.stack([xx.astype(float), yy + t], 1))
    return np.concatenate(pts, 0)


def fit_circle(pts: np.ndarray):
    """Kasa algebraic circle fit: returns (xc, yc, R).  Raises ValueError when
    the points do not determine a circle (fewer than 5, or a fit whose R^2 is
    not positive and finite)."""
    if len(pts) < 5:
        raise ValueError(f"circle fit needs at least 5 contour points, got {len(pts)}")
    x, y = pts[:, 0], pts[:, 1]
    A = np.stack([x, y, np.ones_like(x)], 1)
    rhs = -(x * x + y * y)
    (D, E, F), *_ = np.linalg.lstsq(A, rhs, rcond=None)
    xc, yc = -D / 2, -E / 2
    r2 = xc * xc + yc * yc - F
    if not (np.isfinite(r2) and r2 > 0):
        raise ValueError(f"degenerate circle fit (R^2 = {r2})")
    return xc, yc, float(np.sqrt(r2))


def contact_angle(rho: np.ndarray, fluid: np.ndarray, level: float = 1.0,
                  y_wall: float = 0.5, skip: float = 3.0, y_max: float | None = None):
    """Contact angle (radians) of a droplet sitting on the bottom wall.

    Returns (theta, (xc, yc, R)).  ``y_max`` bounds the contour points from
    above (to exclude a film on the top wall).  Raises ValueError if the
    contour left after dropping the near-wall points does not determine a
    circle (e.g. a droplet that has spread or fallen apart).
    """
    pts = contour_points(rho, level, fluid)
    keep = pts[:, 1] >= y_wall + skip
    if y_max is not None:
        keep &= pts[:, 1] <= y_max
    xc, yc, R = fit_circle(pts[keep])
    c = np.clip((y_wall - yc) / R, -1.0, 1.0)
    return float(np.arccos(c)), (xc, yc, R)


def base_angle(rho: np.ndarray, level: float = 1.0, row: int = 1):
    """Cross-check: base width from the first fluid row and apex height."""
    line = rho[row] - level
    idx = np.nonzero(line >= 0)[0]
    if len(idx) == 0:
        return float("nan")
    x1, x2 = idx.min(), idx.max()
    col = rho[:, (x1 + x2) // 2] - level
    ys = np.nonzero(col >= 0)[0]
    h = ys.max() + 0.5
    return 2.0 * np.arctan2(2.0 * h, (x2 - x1 + 1))
