"""Pins of the oracle's forward renderer: exact pixel coverage of a triangle
over a constant background (closed form, within the binomial band of the
estimator), a linear texture reproduced exactly through the ray / texel-centre
conventions, background-only images, float32 hit decisions against exact
geometry, watertightness and the tie rule."""
import numpy as np

import oracle
from oracle_geom import (camera_sample_offsets, identity_camera, pixel_areas, unproject)

W, H, F_ = 16, 12, 20.0
Z0 = 1.0


def _tri_scene(screen_tri, ka=1.0, kd=0.0, light=(0.0, 0.0, -1.0)):
    verts = np.array([unproject(x, y, Z0, W, H, F_) for x, y in screen_tri])
    faces = np.array([[0, 1, 2]], np.int32)
    uv = np.array([[0.5, 0.5]] * 3)
    sc = oracle.Scene(faces, uv, identity_camera(W, H, F_), [ka, kd, *light])
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    return sc, verts, normals


def test_background_only():
    sc, verts, normals = _tri_scene([[100, 100], [101, 100], [100, 101]])  # off screen
    rng = np.random.default_rng(0)
    bg = rng.uniform(0, 1, (W * H, 3)).astype(np.float32).astype(np.float64)
    img, hits = oracle.render(sc, verts, normals, np.full((2, 2, 3), 0.3), bg, 8, 1, 0, want_hits=True)
    assert (hits == -1).all()
    assert np.array_equal(img, bg)


def test_coverage_closed_form():
    tri = np.array([[2.3, 1.7], [13.6, 4.2], [5.1, 10.4]])
    sc, verts, normals = _tri_scene(tri)
    # float32-representable colours (all inputs of the estimator are float32)
    c0 = np.array([0.9, 0.5, 0.2], np.float32).astype(np.float64)
    b = np.array([0.1, 0.2, 0.3], np.float32).astype(np.float64)
    spp = 256
    img = oracle.render(sc, verts, normals, np.tile(c0, (2, 2, 1)), np.tile(b, (W * H, 1)), spp, 7, 3)
    A = pixel_areas(tri, W, H).reshape(-1)
    exp = b + (c0 - b) * A[:, None]
    sig = np.abs(c0 - b) * np.sqrt(A * (1 - A) / spp)[:, None]
    assert (np.abs(img - exp) <= 5 * sig + 1e-12).all()
    # whole-image coverage
    cov = ((img - b) / (c0 - b))[:, 0].sum()
    assert abs(cov - A.sum()) < 5 * np.sqrt((A * (1 - A)).sum() / spp)
    # pixels fully inside / outside are exact
    assert np.array_equal(img[A == 0], np.tile(b, ((A == 0).sum(), 1)))


def test_linear_texture_and_sample_positions():
    # a fronto-parallel triangle covering the image, with texture coordinates
    # affine in screen position and a texture that is linear in its coordinates:
    # the colour of every sample is known exactly from its screen position
    tri = np.array([[-20.0, -20.0], [60.0, -20.0], [-20.0, 60.0]])
    verts = np.array([unproject(x, y, Z0, W, H, F_) for x, y in tri])
    uvs = np.array([[0.1 + 0.8 * (x + 20) / 80 * 0.25, 0.2 + 0.6 * (y + 20) / 80 * 0.25] for x, y in tri])
    th, tw = 8, 10
    tex = np.zeros((th, tw, 3))
    tex[..., 0] = ((np.arange(tw) + 0.5) / tw)[None, :]
    tex[..., 1] = ((np.arange(th) + 0.5) / th)[:, None]
    tex[..., 2] = 0.25
    sc = oracle.Scene(np.array([[0, 1, 2]], np.int32), uvs, identity_camera(W, H, F_),
                      [1.0, 0.0, 0.0, 0.0, -1.0])
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    spp, seed, it = 4, 11, 5
    img = oracle.render(sc, verts, normals, tex, np.zeros((W * H, 3)), spp, seed, it)
    pix = np.arange(W * H)
    u, v = camera_sample_offsets(oracle.philox4x64, seed, it, 0, pix, spp)
    sx = (pix % W)[:, None] + u
    sy = (pix // W)[:, None] + v
    eu = 0.1 + 0.8 * (sx + 20) / 80 * 0.25
    ev = 0.2 + 0.6 * (sy + 20) / 80 * 0.25
    assert np.abs(img[:, 0] - eu.mean(1)).max() < 1e-12
    assert np.abs(img[:, 1] - ev.mean(1)).max() < 1e-12
    assert np.abs(img[:, 2] - 0.25).max() < 1e-15


def test_shading_closed_form():
    # constant albedo, flat normal: colour = albedo * (ka + kd * max(0, n.l))
    tri = np.array([[-20.0, -20.0], [60.0, -20.0], [-20.0, 60.0]])
    l = np.array([0.3, -0.4, -0.866])
    l /= np.linalg.norm(l)
    sc, verts, normals = _tri_scene(tri, ka=0.25, kd=0.5, light=tuple(l))
    alb = np.array([0.8, 0.4, 0.6])
    img = oracle.render(sc, verts, normals, np.tile(alb, (2, 2, 1)), np.zeros((W * H, 3)), 2, 1, 0)
    exp = alb * (0.25 + 0.5 * max(0.0, float(np.dot([0, 0, -1], l))))
    assert np.abs(img - exp).max() < 1e-15


def _moller(o, d, v0, v1, v2):
    e1, e2 = v1 - v0, v2 - v0
    p = np.cross(d, e2)
    det = e1 @ p
    s = o - v0
    u = (s @ p) / det
    q = np.cross(s, e1)
    v = (d @ q) / det
    t = (e2 @ q) / det
    return u, v, t


def test_float32_decision_agrees_with_exact_geometry():
    rng = np.random.default_rng(5)
    n = 4000
    tris = rng.normal(0, 1, (n, 3, 3)) + np.array([0, 0, 5.0])
    org = rng.normal(0, 0.2, (n, 3))
    tgt = tris.mean(1) + rng.normal(0, 0.8, (n, 3))
    dirs = tgt - org
    t32 = tris.astype(np.float32)
    o32 = org.astype(np.float32)
    d32 = dirs.astype(np.float32)
    faces = np.array([[0, 1, 2]], np.int32)
    checked = 0
    for i in range(n):
        fo, to = oracle.trace_rays32(o32[i], d32[i], t32[i], faces)
        u, v, t = _moller(o32[i].astype(np.float64), d32[i].astype(np.float64), *t32[i].astype(np.float64))
        m = min(u, v, 1 - u - v)
        if abs(m) < 1e-4 or abs(t) < 1e-4:
            continue  # near an edge or the origin: either answer is acceptable
        checked += 1
        inside = m > 0 and t > 0
        assert (fo[0] == 0) == inside, i
        if inside:
            assert abs(to[0] - t) <= 1e-5 * abs(t)
    assert checked > 3500


def _icosphere():
    t = (1 + 5 ** 0.5) / 2
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t],
                  [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
                  [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
                  [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]])
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def test_watertight_no_leaks_through_edges_and_vertices():
    # from inside a closed mesh every ray must hit, including rays aimed
    # exactly at shared edges and vertices
    v, f = _icosphere()
    c = np.array([0.1, -0.2, 1.0], np.float32)
    v32 = (v * 0.3 + c).astype(np.float32)
    rng = np.random.default_rng(6)
    targets = []
    for a, b, cc in f:
        for (p, q) in ((a, b), (b, cc), (cc, a)):
            for s in rng.uniform(0, 1, 16):
                targets.append(v32[p] + np.float32(s) * (v32[q] - v32[p]))
        targets.append(v32[a])
    targets = np.array(targets, np.float32)
    org = np.tile(c, (len(targets), 1)) + rng.normal(0, 0.02, (len(targets), 3)).astype(np.float32)
    fo, _ = oracle.trace_rays32(org, targets - org, v32, f.astype(np.int32))
    assert (fo >= 0).all()
    # rays from the centre through every vertex, exactly
    fo, _ = oracle.trace_rays32(np.tile(c, (12, 1)), v32 - c, v32, f.astype(np.int32))
    assert (fo >= 0).all()


def test_tie_goes_to_smaller_face_id():
    v32 = np.array([[-1, -1, 2], [1, -1, 2], [0, 1, 2]], np.float32)
    faces = np.array([[0, 1, 2], [0, 2, 1], [0, 1, 2]], np.int32)  # same triangle three times
    fo, to = oracle.trace_rays32(np.zeros((1, 3), np.float32), np.array([[0.0, 0.0, 1.0]], np.float32),
                                 v32, faces)
    assert fo[0] == 0 and to[0] == 2.0
    fo, _ = oracle.trace_rays32(np.zeros((1, 3), np.float32), np.array([[0.0, 0.0, 1.0]], np.float32),
                                v32, faces[::-1].copy())
    assert fo[0] == 0
