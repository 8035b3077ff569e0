"""Diagnostics of the oracle (test infrastructure only): contact angle, cap
shape and steady-state residual.

The paper measures equilibrium contact angles against analytic circles (Sec. 3.1
after Eq. initialphi; Sec. 3.3 Eq. initialphi_cirref) but prints no estimator.
READING (used identically, in separate code, by the GPU library):
  * interface points are the sub-cell phi = 1/2 crossings on lattice edges along
    each axis between two zeta = 1 nodes: an edge (a, b) crosses when exactly one
    of phi_a, phi_b is below 1/2, at a + (1/2 - phi_a)/(phi_b - phi_a) (b - a);
  * only points at least W away from the wall surface are kept;
  * a Kasa least-squares circle (2D) or sphere (3D) is fitted to them;
  * flat or inclined wall: cos(theta) = -h / R with h the signed distance of the
    centre from the wall plane along the normal pointing into the fluid;
  * curved wall of radius R_s: cos(theta) = (R^2 + R_s^2 - d^2) / (2 R R_s), with d
    the centre distance; this is Eq. (initialphi_cirref) solved for theta.
"""
import math

import numpy as np


def interface_points(phi, zeta, level=0.5):
    """phi, zeta: domain arrays of numpy shape (ny, nx) or (nz, ny, nx).
    Returns an (n, D) array of (x, y[, z]) crossing positions."""
    phi = np.asarray(phi, dtype=np.float64)
    zeta = np.asarray(zeta, dtype=bool)
    D = phi.ndim
    pts = []
    idx = np.indices(phi.shape).astype(np.float64)      # numpy-axis order (z, y, x)
    for ax in range(D):
        lo = [slice(None)] * D
        hi = [slice(None)] * D
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        a, b = phi[lo], phi[hi]
        cross = zeta[lo] & zeta[hi] & ((a < level) != (b < level))
        t = (level - a[cross]) / (b[cross] - a[cross])
        coord = [idx[k][lo][cross] for k in range(D)]
        coord[ax] = coord[ax] + t
        pts.append(np.stack(coord[::-1], axis=1))       # -> (x, y[, z])
    return np.concatenate(pts, axis=0)


def wall_distance(points, wall):
    if wall["kind"] == "plane":
        p0 = np.asarray(wall["point"], dtype=np.float64)
        n = np.asarray(wall["normal"], dtype=np.float64)
        n = n / np.linalg.norm(n)
        return (points - p0) @ n
    c = np.asarray(wall["center"], dtype=np.float64)
    return np.linalg.norm(points - c, axis=1) - wall["radius"]


def kasa_fit(points):
    """Least-squares circle/sphere |x|^2 + a.x + b = 0 -> (centre, radius)."""
    n, D = points.shape
    A = np.concatenate([points, np.ones((n, 1))], axis=1)
    rhs = -(points ** 2).sum(axis=1)
    sol, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    centre = -0.5 * sol[:D]
    radius = math.sqrt(float(centre @ centre - sol[D]))
    return centre, radius


def contact_angle(phi, zeta, wall, width):
    """Contact angle in degrees, fitted centre and radius, point count."""
    pts = interface_points(phi, zeta)
    pts = pts[wall_distance(pts, wall) >= width]
    if len(pts) < 2 * pts.shape[1] + 2:
        return float("nan"), None, float("nan"), len(pts)
    centre, R = kasa_fit(pts)
    if wall["kind"] == "plane":
        n = np.asarray(wall["normal"], dtype=np.float64)
        n = n / np.linalg.norm(n)
        h = float((centre - np.asarray(wall["point"], dtype=np.float64)) @ n)
        cos_t = -h / R
    else:
        Rs = float(wall["radius"])
        d = float(np.linalg.norm(centre - np.asarray(wall["center"], dtype=np.float64)))
        cos_t = (R * R + Rs * Rs - d * d) / (2.0 * R * Rs)
    cos_t = min(1.0, max(-1.0, cos_t))
    return math.degrees(math.acos(cos_t)), centre, R, len(pts)


def cap_radius_2d(r0, theta_deg):
    """Equal-area circular cap on a flat wall from a semicircle of radius r0:
    area R^2 (theta - sin theta cos theta) = pi r0^2 / 2."""
    t = math.radians(theta_deg)
    return r0 * math.sqrt(math.pi / (2.0 * (t - math.sin(t) * math.cos(t))))


def cap_radius_3d(r0, theta_deg):
    """Equal-volume spherical cap from a hemisphere of radius r0:
    pi R^3 (1 - cos)^2 (2 + cos) / 3 = 2 pi r0^3 / 3."""
    c = math.cos(math.radians(theta_deg))
    return r0 * (2.0 / ((1.0 - c) ** 2 * (2.0 + c))) ** (1.0 / 3.0)


def steady_residual(phi_now, phi_then, zeta):
    return float(np.abs(np.asarray(phi_now) - np.asarray(phi_then))[np.asarray(zeta, bool)].max())
