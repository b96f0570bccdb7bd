"""Independent geometric references for pinning the oracle (test-only helpers).

These are written from elementary geometry, not from the paper's construction:
polygon clipping by a half-plane, the shoelace area, and exact piecewise-Gauss
time integration of a clipped area.  They share nothing with the oracle's C code.
"""
import numpy as np


def clip_polygon_halfspace(poly, n, c):
    """Part of a planar polygon (k,3) with n.x <= c (Sutherland-Hodgman, one plane)."""
    out = []
    k = len(poly)
    for i in range(k):
        p, q = poly[i], poly[(i + 1) % k]
        dp, dq = np.dot(n, p) - c, np.dot(n, q) - c
        if dp <= 0:
            out.append(p)
        if (dp <= 0) != (dq <= 0):
            t = dp / (dp - dq)
            out.append(p + t * (q - p))
    return np.array(out) if out else np.zeros((0, 3))


def polygon_area(poly):
    if len(poly) < 3:
        return 0.0
    s = np.zeros(3)
    for i in range(1, len(poly) - 1):
        s += np.cross(poly[i] - poly[0], poly[i + 1] - poly[0])
    return 0.5 * np.linalg.norm(s)


def wet_fraction_exact(tri, xS, nS, un, s):
    """Area fraction of triangle tri (3,3) with (x - xS).nS <= un*s (the moving plane)."""
    A = polygon_area(tri)
    part = clip_polygon_halfspace(tri, nS, np.dot(nS, xS) + un * s)
    return polygon_area(part) / A


def wet_integral_exact(tri, xS, nS, un, dt, gauss=3):
    """int_0^dt wet fraction ds: Gauss-Legendre on the pieces between vertex arrival times.

    Between arrival times the clipped area is a quadratic in s, so a 3-point rule
    on every piece is exact up to round-off.
    """
    d = (tri - xS) @ nS
    br = [0.0, dt]
    if un != 0.0:
        for dk in d:
            sk = dk / un
            if 0.0 < sk < dt:
                br.append(sk)
    br = np.sort(np.array(br))
    gx, gw = np.polynomial.legendre.leggauss(gauss)
    total = 0.0
    for a, b in zip(br[:-1], br[1:]):
        if b <= a:
            continue
        for x, w in zip(gx, gw):
            s = 0.5 * (a + b) + 0.5 * (b - a) * x
            total += 0.5 * (b - a) * w * wet_fraction_exact(tri, xS, nS, un, s)
    return total


def box_below_plane_volume(lo, hi, g, c):
    """Volume of the box [lo,hi] with g.x < c, all g components non-zero.

    Inclusion-exclusion over the box corners of the simplex {g.x < c}:
    V = sum_corners (-1)^{#hi} max(0, c - g.corner)^3 / (6 |g1 g2 g3|),
    with the box mapped so that every g component is positive.
    """
    lo = np.array(lo, float)
    hi = np.array(hi, float)
    g = np.array(g, float)
    # flip axes with negative g so that g > 0 (reflect the box)
    lo2, hi2, g2 = lo.copy(), hi.copy(), g.copy()
    for i in range(3):
        if g2[i] < 0:
            lo2[i], hi2[i] = -hi[i], -lo[i]
            g2[i] = -g2[i]
    tot = 0.0
    for bits in range(8):
        corner = np.array([hi2[i] if (bits >> i) & 1 else lo2[i] for i in range(3)])
        sgn = (-1) ** bin(bits).count("1")
        tot += sgn * max(0.0, c - np.dot(g2, corner)) ** 3
    return tot / (6.0 * g2[0] * g2[1] * g2[2])


def clipped_hull_volume_and_section(verts, edges, g, c):
    """Convex cell (verts, edge list) cut by g.x < c: volume (scipy hull) and the section polygon."""
    from scipy.spatial import ConvexHull
    keep = [v for v in verts if np.dot(g, v) < c]
    sec = []
    for a, b in edges:
        da, db = np.dot(g, verts[a]) - c, np.dot(g, verts[b]) - c
        if (da < 0) != (db < 0):
            t = da / (da - db)
            sec.append(verts[a] + t * (verts[b] - verts[a]))
    pts = np.array(keep + sec)
    vol = ConvexHull(pts).volume if len(pts) >= 4 else 0.0
    return vol, np.array(sec)


def section_centroid(sec, normal):
    """Area centroid of a planar convex polygon given as an unordered point set."""
    n = normal / np.linalg.norm(normal)
    o = sec.mean(axis=0)
    u = sec[0] - o
    u -= np.dot(u, n) * n
    u /= np.linalg.norm(u)
    v = np.cross(n, u)
    ang = np.arctan2((sec - o) @ v, (sec - o) @ u)
    P = sec[np.argsort(ang)]
    A = 0.0
    C = np.zeros(3)
    for i in range(1, len(P) - 1):
        a = 0.5 * np.dot(np.cross(P[i] - P[0], P[i + 1] - P[0]), n)
        A += a
        C += a * (P[0] + P[i] + P[i + 1]) / 3.0
    return C / A, A
