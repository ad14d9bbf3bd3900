"""Pins of the oracle's silhouette-edge boundary term (visibility gradients,
Section 4.2.2; edge sampling as in Li et al. 2018).  For flat-coloured triangles
over a constant background the expected image is known exactly from pixel
coverage areas (convex polygon clipping), so the gradient of any weighted sum of
pixels is known exactly; the edge-sampled estimate must match it within its
statistical error, and the interior term must vanish."""
import numpy as np

import oracle
from oracle_geom import (clip_to_box, identity_camera, pixel_areas, pixel_areas_overlap, poly_area,
                         unproject)

W, H, F_ = 16, 12, 20.0


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _project(v):
    return np.array([F_ * v[0] / v[2] + W / 2, F_ * v[1] / v[2] + H / 2])


def _scene(verts_list, faces):
    faces = np.asarray(faces, np.int32)
    # edge tables
    directed = {}
    for f, t in enumerate(faces):
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(a, b)] = f
    edges, ef = [], []
    for (a, b), f in directed.items():
        if (b, a) in directed and a > b:
            continue
        edges.append((a, b))
        ef.append((f, directed.get((b, a), -1)))
    uv = np.full((len(verts_list), 2), 0.5)
    sc = oracle.Scene(faces, uv, identity_camera(W, H, F_), [1.0, 0.0, 0.0, 0.0, -1.0],
                      np.array(edges, np.int32), np.array(ef, np.int32))
    return sc


def _estimate(sc, verts, colour, b, g, n_seeds=12, budget=40000):
    normals = np.tile([0.0, 0.0, -1.0], (len(verts), 1))
    alb = np.tile(colour, (2, 2, 1))
    bg = np.tile(b, (W * H, 1))
    ests = []
    for s in range(n_seeds):
        ests.append(oracle.backward_edges(sc, verts, normals, alb, bg, g, 100 + s, 0, 1e-3,
                                          budget=budget)[0])
    ests = np.array(ests)
    return ests.mean(0), ests.std(0, ddof=1) / np.sqrt(n_seeds)


def _check(est, se, exact):
    scale = np.abs(exact).max()
    assert (np.abs(est - exact) <= 5 * se + 2e-3 * scale).all(), (est, exact, se)


def test_single_triangle_matches_exact_coverage_gradient():
    tri_s = np.array([[2.3, 1.7], [13.6, 4.2], [5.1, 10.4]])
    zs = [1.0, 1.2, 0.9]
    verts = _f32([unproject(x, y, z, W, H, F_) for (x, y), z in zip(tri_s, zs)])
    sc = _scene(verts, [[0, 1, 2]])
    c0, b = _f32([0.9, 0.5, 0.2]), _f32([0.1, 0.2, 0.3])
    rng = np.random.default_rng(0)
    g = rng.normal(0, 1, (W * H, 3))
    est, se = _estimate(sc, verts, c0, b, g)
    # exact: d/dv sum_p g_p (b + (c0-b) A_p(v))
    gw = (g * (c0 - b)).sum(1).reshape(H, W)
    exact = np.zeros_like(verts)
    h = 1e-7
    for i in range(3):
        for k in range(3):
            vp = verts.copy(); vp[i, k] += h
            vm = verts.copy(); vm[i, k] -= h
            Ap = pixel_areas(np.array([_project(x) for x in vp]), W, H)
            Am = pixel_areas(np.array([_project(x) for x in vm]), W, H)
            exact[i, k] = (gw * (Ap - Am)).sum() / (2 * h)
    _check(est, se, exact)
    # the interior term vanishes for a flat colour
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    ga, gv, gn = oracle.backward_interior(sc, verts, normals, np.tile(c0, (2, 2, 1)), g, 4, 1, 0)
    assert np.abs(gv).max() == 0.0 and np.abs(gn).max() == 0.0


def test_triangle_crossing_the_image_border():
    tri_s = np.array([[-3.0, 2.0], [10.0, -4.0], [12.5, 15.0]])
    verts = _f32([unproject(x, y, 1.1, W, H, F_) for x, y in tri_s])
    sc = _scene(verts, [[0, 1, 2]])
    c0, b = _f32([0.2, 0.8, 0.6]), _f32([0.7, 0.1, 0.4])
    g = np.ones((W * H, 3))
    est, se = _estimate(sc, verts, c0, b, g)
    gw = (g * (c0 - b)).sum(1).reshape(H, W)
    exact = np.zeros_like(verts)
    h = 1e-7
    for i in range(3):
        for k in range(3):
            vp = verts.copy(); vp[i, k] += h
            vm = verts.copy(); vm[i, k] -= h
            Ap = pixel_areas(np.array([_project(x) for x in vp]), W, H)
            Am = pixel_areas(np.array([_project(x) for x in vm]), W, H)
            exact[i, k] = (gw * (Ap - Am)).sum() / (2 * h)
    _check(est, se, exact)


def test_occluding_triangles():
    # triangle 0 in front (z = 1), triangle 1 behind (z = 2); colours via two
    # texels of a 1x2 texture selected by uv
    t1 = np.array([[3.0, 2.0], [12.0, 3.5], [6.0, 9.5]])
    t2 = np.array([[1.5, 6.0], [14.0, 1.0], [11.0, 11.0]])
    verts = _f32([unproject(x, y, 1.0, W, H, F_) for x, y in t1]
                 + [unproject(x, y, 2.0, W, H, F_) for x, y in t2])
    faces = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    sc = _scene(verts, faces)
    sc.uv = np.array([[0.25, 0.5]] * 3 + [[0.75, 0.5]] * 3)
    c1, c2, b = _f32([0.9, 0.1, 0.5]), _f32([0.2, 0.6, 0.9]), _f32([0.5, 0.5, 0.0])
    tex = np.stack([c1, c2])[None]  # [1,2,3]
    rng = np.random.default_rng(1)
    g = rng.normal(0, 1, (W * H, 3))
    normals = np.tile([0.0, 0.0, -1.0], (6, 1))
    bg = np.tile(b, (W * H, 1))
    ests = np.array([oracle.backward_edges(sc, verts, normals, tex, bg, g, 300 + s, 0, 1e-3,
                                           budget=40000)[0] for s in range(12)])
    est, se = ests.mean(0), ests.std(0, ddof=1) / np.sqrt(12)

    def expected_L(v):
        p1 = np.array([_project(x) for x in v[:3]])
        p2 = np.array([_project(x) for x in v[3:]])
        A1 = pixel_areas(p1, W, H)
        A2 = pixel_areas(p2, W, H)
        A12 = pixel_areas_overlap(p1, p2, W, H)
        # E[I] = b + (c1-b) A1 + (c2-b) (A2 - A12)
        return ((g.reshape(H, W, 3) * ((c1 - b) * A1[..., None] + (c2 - b) * (A2 - A12)[..., None])).sum())

    exact = np.zeros_like(verts)
    h = 1e-7
    for i in range(6):
        for k in range(3):
            vp = verts.copy(); vp[i, k] += h
            vm = verts.copy(); vm[i, k] -= h
            exact[i, k] = (expected_L(vp) - expected_L(vm)) / (2 * h)
    _check(est, se, exact)


def test_budget_is_one_sample_per_silhouette_pixel():
    tri_s = np.array([[2.0, 2.0], [10.0, 2.0], [2.0, 8.0]])
    verts = _f32([unproject(x, y, 1.0, W, H, F_) for x, y in tri_s])
    sc = _scene(verts, [[0, 1, 2]])
    w, cdf, tot, bud = oracle.edge_weights(sc, verts)
    per = 8 + 6 + 10  # screen lengths of the three edges
    assert abs(int(tot[0]) / 256 - per) < 3 / 256 + 1e-3
    assert bud[0] == int(np.ceil(int(tot[0]) / 256))
    assert np.array_equal(np.cumsum(w[0].astype(np.uint64)), cdf[0])
