"""Exact-geometry helpers for pinning the oracle: convex polygon clipping and
areas in float64, and small synthetic scenes.  Independent of both the oracle's
and the GPU path's arithmetic."""
import numpy as np


def clip_poly(poly, a, b, c):
    """Keep the part of polygon `poly` ([n,2]) where a*x + b*y + c >= 0."""
    out = []
    n = len(poly)
    for i in range(n):
        p, q = poly[i], poly[(i + 1) % n]
        fp = a * p[0] + b * p[1] + c
        fq = a * q[0] + b * q[1] + c
        if fp >= 0:
            out.append(p)
        if (fp >= 0) != (fq >= 0):
            t = fp / (fp - fq)
            out.append(p + t * (q - p))
    return np.array(out) if out else np.zeros((0, 2))


def poly_area(poly):
    if len(poly) < 3:
        return 0.0
    x, y = poly[:, 0], poly[:, 1]
    return 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))


def clip_to_box(poly, x0, y0, x1, y1):
    poly = clip_poly(poly, 1, 0, -x0)
    poly = clip_poly(poly, -1, 0, x1)
    poly = clip_poly(poly, 0, 1, -y0)
    poly = clip_poly(poly, 0, -1, y1)
    return poly


def clip_to_triangle(poly, tri):
    """Intersect a convex polygon with a triangle (either winding)."""
    s = np.sign((tri[1, 0] - tri[0, 0]) * (tri[2, 1] - tri[0, 1])
                - (tri[1, 1] - tri[0, 1]) * (tri[2, 0] - tri[0, 0]))
    for i in range(3):
        p, q = tri[i], tri[(i + 1) % 3]
        # left of p->q (for counter-clockwise) is inside
        a, b = -(q[1] - p[1]) * s, (q[0] - p[0]) * s
        c = -(a * p[0] + b * p[1])
        poly = clip_poly(poly, a, b, c)
        if len(poly) == 0:
            break
    return poly


def pixel_areas(tri, W, H):
    """Exact area of triangle ∩ pixel for every pixel: [H,W]."""
    A = np.zeros((H, W))
    lo = np.floor(tri.min(0)).astype(int)
    hi = np.ceil(tri.max(0)).astype(int)
    for y in range(max(lo[1], 0), min(hi[1], H)):
        for x in range(max(lo[0], 0), min(hi[0], W)):
            A[y, x] = poly_area(clip_to_box(tri, x, y, x + 1, y + 1))
    return A


def pixel_areas_overlap(t1, t2, W, H):
    """Exact area of (t1 ∩ t2) ∩ pixel: [H,W]."""
    inter = clip_to_triangle(t2.copy(), t1)
    A = np.zeros((H, W))
    if len(inter) < 3:
        return A
    for y in range(H):
        for x in range(W):
            A[y, x] = poly_area(clip_to_box(inter, x, y, x + 1, y + 1))
    return A


def identity_camera(W, H, f):
    """A camera at the origin looking down +z (float32 tables, one view)."""
    return dict(R=np.eye(3, dtype=np.float32).reshape(1, 9), o=np.zeros((1, 3), np.float32),
                intr=np.array([[f, f, W / 2, H / 2]], np.float32),
                wh=np.array([[W, H]], np.int32), hand=np.zeros(1, np.int32),
                pix_off=np.array([0, W * H], np.int64))


def unproject(px, py, z, W, H, f):
    """World point at depth z under `identity_camera` that projects to (px,py)."""
    return np.array([(px - W / 2) / f * z, (py - H / 2) / f * z, z])


def camera_sample_offsets(philox, seed, it, view, pix, spp):
    """(u,v) of every camera sample from the counter layout of the estimator."""
    ctr = np.zeros((len(pix) * ((spp + 3) // 4), 4), dtype=np.uint64)
    q = np.arange((spp + 3) // 4)
    ctr[:, 0] = np.repeat(np.asarray(pix, np.uint64), len(q))
    ctr[:, 1] = np.tile(q.astype(np.uint64), len(pix))
    ctr[:, 2] = np.uint64(view)
    ctr[:, 3] = np.uint64(it)
    r = philox(ctr, np.array([seed, 0], dtype=np.uint64)).reshape(len(pix), -1)[:, :spp]
    u = ((r & np.uint64(0xFFFFFFFF)) >> np.uint64(8)).astype(np.float64) / 2 ** 24
    v = (r >> np.uint64(40)).astype(np.float64) / 2 ** 24
    return u, v
