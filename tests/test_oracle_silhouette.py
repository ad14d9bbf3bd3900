"""Pins of the oracle's silhouette test on closed meshes (visibility
gradients, Section 4.2.2; edge sampling as in Li et al. 2018).  Every edge of
a closed solid is shared by two triangles, so its outline is made of edges
between a triangle facing the camera and one facing away, and the split
diagonals of its square faces join two triangles facing the same way: they
lie inside the outline or behind it and carry no visibility boundary.

For a flat-coloured convex solid over a constant background the expected
image is b + (c - b) A_p, A_p the exact area of the projected outline (the
convex hull of the projected vertices) inside pixel p, so the gradient of any
weighted sum of pixels follows from central differences of exact polygon
areas.  The tests fail if the classification takes boundary edges only (a
closed mesh has none), or edges between two front-facing triangles, or
drops the outline."""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from oracle_geom import clip_to_convex, convex_hull, identity_camera, polygon_pixel_areas, triangulated_cube

W, H, FOC = 24, 20, 24.0


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _project(v):
    v = np.atleast_2d(v)
    return np.stack([FOC * v[:, 0] / v[:, 2] + W / 2, FOC * v[:, 1] / v[:, 2] + H / 2], 1)


def _edge_tables(faces):
    directed = {}
    for f, t in enumerate(faces):
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            directed[(int(a), int(b))] = f
    edges, ef = [], []
    for (a, b), f in directed.items():
        if a > b and (b, a) in directed:
            continue
        edges.append((a, b))
        ef.append((f, directed.get((b, a), -1)))
    return np.array(edges, np.int32), np.array(ef, np.int32)


def _scene(faces, uv):
    edges, ef = _edge_tables(faces)
    return oracle.Scene(faces, uv, identity_camera(W, H, FOC), [1.0, 0.0, 0.0, 0.0, -1.0], edges, ef)


def _cube(seed, half, centre):
    # tilted so that all three face directions are seen obliquely (a hexagonal
    # outline), with a seeded jitter
    rv = np.array([0.62, 0.78, 0.1]) + np.random.default_rng(seed).normal(0, 0.15, 3)
    rot = Rotation.from_rotvec(rv).as_matrix()
    v, f = triangulated_cube(half, rot, centre)
    return _f32(v), f


def _hull_edges(v):
    """Vertex pairs that are consecutive corners of the projected outline."""
    p = _project(v)
    hull = convex_hull(p)
    idx = [int(np.argmin(np.abs(p - q).sum(1))) for q in hull]
    return {tuple(sorted((idx[i], idx[(i + 1) % len(idx)]))) for i in range(len(idx))}, hull


def _estimate(sc, verts, tex, b, g, n_seeds=12, budget=40000):
    normals = np.tile([0.0, 0.0, -1.0], (len(verts), 1))
    bg = np.tile(b, (W * H, 1))
    ests = np.array([oracle.backward_edges(sc, verts, normals, tex, bg, g, 500 + s, 0, 1e-3, budget=budget)[0]
                     for s in range(n_seeds)])
    return ests.mean(0), ests.std(0, ddof=1) / np.sqrt(n_seeds)


def _exact_grad(L, verts, h=1e-7):
    out = np.zeros_like(verts)
    for i in range(len(verts)):
        for k in range(3):
            vp = verts.copy(); vp[i, k] += h
            vm = verts.copy(); vm[i, k] -= h
            out[i, k] = (L(vp) - L(vm)) / (2 * h)
    return out


def _check(est, se, exact):
    scale = np.abs(exact).max()
    assert scale > 0
    assert (np.abs(est - exact) <= 5 * se + 2e-3 * scale).all(), (est, exact, se)


@pytest.mark.parametrize("seed", [0, 1])
def test_closed_cube_silhouette_set_is_its_outline(seed):
    v, f = _cube(seed, 0.25, [0.05, -0.03, 1.4])
    sc = _scene(f, np.full((8, 2), 0.5))
    w, cdf, tot, bud = oracle.edge_weights(sc, v)
    hull_edges, hull = _hull_edges(v)
    assert len(hull) == 6, "a generic view of a cube has a hexagonal outline"
    sampled = {tuple(sorted(map(int, e))) for e, we in zip(sc.edges, w[0]) if we > 0}
    assert sampled == hull_edges
    # the split diagonals join coplanar triangles: never a silhouette
    diag = [k for k, e in enumerate(sc.edges) if abs(np.linalg.norm(v[e[0]] - v[e[1]]) - 0.5 * np.sqrt(2)) < 1e-5]
    assert len(diag) == 6 and all(w[0, k] == 0 for k in diag)
    # one sample per silhouette pixel: total quantised length = outline perimeter
    per = sum(np.linalg.norm(hull[i] - hull[(i + 1) % 6]) for i in range(6))
    assert 256 * per - 6 <= int(tot[0]) <= 256 * per + 1e-6
    assert bud[0] == int(np.ceil(int(tot[0]) / 256))


@pytest.mark.parametrize("seed", [0, 1])
def test_closed_cube_matches_exact_outline_gradient(seed):
    v, f = _cube(seed, 0.25, [0.05, -0.03, 1.4])
    sc = _scene(f, np.full((8, 2), 0.5))
    c, b = _f32([0.85, 0.3, 0.15]), _f32([0.1, 0.25, 0.6])
    g = np.random.default_rng(10 + seed).normal(0, 1, (W * H, 3))
    est, se = _estimate(sc, v, np.tile(c, (2, 2, 1)), b, g)
    gw = (g * (c - b)).sum(1).reshape(H, W)
    exact = _exact_grad(lambda x: (gw * polygon_pixel_areas(convex_hull(_project(x)), W, H)).sum(), v)
    _check(est, se, exact)
    # corners inside the outline do not move it
    inner = sorted(set(range(8)) - {i for e in _hull_edges(v)[0] for i in e})
    assert len(inner) == 2 and np.abs(exact[inner]).max() == 0.0


def test_cube_occluding_cube():
    # a near cube hides part of a far one: the far cube's outline edges behind
    # the near cube see the near cube's colour on both sides and contribute
    # nothing; its visible outline edges see (far colour, background)
    v1, f1 = _cube(3, 0.2, [-0.08, 0.02, 1.2])
    v2, f2 = _cube(4, 0.3, [0.12, -0.02, 1.9])
    v = np.concatenate([v1, v2])
    f = np.concatenate([f1, f2 + 8]).astype(np.int32)
    uv = np.array([[0.25, 0.5]] * 8 + [[0.75, 0.5]] * 8)
    sc = _scene(f, uv)
    c1, c2, b = _f32([0.9, 0.1, 0.5]), _f32([0.2, 0.6, 0.9]), _f32([0.5, 0.5, 0.0])
    tex = np.stack([c1, c2])[None]
    g = np.random.default_rng(21).normal(0, 1, (W * H, 3))
    est, se = _estimate(sc, v, tex, b, g)
    gimg = g.reshape(H, W, 3)

    def expected_L(x):
        h1 = convex_hull(_project(x[:8]))
        h2 = convex_hull(_project(x[8:]))
        a1 = polygon_pixel_areas(h1, W, H)
        a2 = polygon_pixel_areas(h2, W, H)
        a12 = polygon_pixel_areas(clip_to_convex(h2, h1), W, H)
        return (gimg * ((c1 - b) * a1[..., None] + (c2 - b) * (a2 - a12)[..., None])).sum()

    h1, h2 = convex_hull(_project(v1)), convex_hull(_project(v2))
    overlap = polygon_pixel_areas(clip_to_convex(h2, h1), W, H).sum()
    assert overlap > 5.0 and overlap < 0.8 * polygon_pixel_areas(h2, W, H).sum()
    _check(est, se, _exact_grad(expected_L, v))
