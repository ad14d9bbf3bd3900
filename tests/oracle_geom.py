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


def convex_hull(pts):
    """Counter-clockwise convex hull of 2-D points (monotone chain)."""
    pts = sorted(map(tuple, np.asarray(pts, np.float64)))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return np.array(lower[:-1] + upper[:-1])


def clip_to_convex(poly, hull):
    """Intersect a convex polygon with a counter-clockwise convex polygon."""
    n = len(hull)
    for i in range(n):
        p, q = hull[i], hull[(i + 1) % n]
        a, b = -(q[1] - p[1]), (q[0] - p[0])
        c = -(a * p[0] + b * p[1])
        poly = clip_poly(poly, a, b, c)
        if len(poly) == 0:
            break
    return poly


def polygon_pixel_areas(poly, W, H):
    """Exact area of (convex polygon) ∩ pixel for every pixel: [H,W]."""
    A = np.zeros((H, W))
    if len(poly) < 3:
        return A
    lo = np.floor(poly.min(0)).astype(int)
    hi = np.ceil(poly.max(0)).astype(int)
    for y in range(max(lo[1], 0), min(hi[1], H)):
        for x in range(max(lo[0], 0), min(hi[0], W)):
            A[y, x] = poly_area(clip_to_box(poly, x, y, x + 1, y + 1))
    return A


def triangulated_cube(half, rot, centre):
    """Closed cube of half-size `half`, rotated by `rot` [3,3] about its centre
    and moved to `centre`: 8 vertices, 12 triangles wound counter-clockwise
    seen from outside (two per square face, split along a diagonal)."""
    corners = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float64)
    quads = []
    for axis in range(3):
        for sgn in (-1, 1):
            q = [i for i, c in enumerate(corners) if c[axis] == sgn]
            # order the face's corners around its normal
            u, v = [a for a in range(3) if a != axis]
            ctr = corners[q].mean(0)
            ang = [np.arctan2(corners[i][v] - ctr[v], corners[i][u] - ctr[u]) for i in q]
            q = [q[k] for k in np.argsort(ang)]
            n = np.zeros(3)
            n[axis] = sgn
            tri = (q[0], q[1], q[2])
            e = np.cross(corners[tri[1]] - corners[tri[0]], corners[tri[2]] - corners[tri[0]])
            if np.dot(e, n) < 0:
                q = q[::-1]
            quads.append(q)
    faces = []
    for q in quads:
        faces.append((q[0], q[1], q[2]))
        faces.append((q[0], q[2], q[3]))
    verts = (corners * half) @ np.asarray(rot).T + np.asarray(centre)
    return verts, np.array(faces, np.int32)
