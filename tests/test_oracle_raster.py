"""Pins of the oracle's hard rasteriser (oracle/raster.py; Section 4.2.2,
"Ray tracing vs rasterization"):

- coverage of pixel centres against an exact rational point-in-triangle test
  (fractions of the same projected coordinates), for a triangle of each
  orientation;
- the nearest triangle wins whichever is listed first, and of two identical
  triangles the one with the smaller index;
- perspective-correct depth: the winning 1/z at every covered centre equals
  1/z of the exact intersection of the centre's ray with the triangle's plane
  (an independent solve in camera space);
- a flat triangle's image is its centre-coverage mask times the closed-form
  Lambert colour over the background;
- with distinct vertex normals and texture coordinates and an affine colour
  map, every covered pixel equals the closed form at barycentrics from an
  independent solve (renormalised normal, texel centres, row/column order,
  light direction);
- the derivative at fixed coverage against central differences of the
  oracle's own image (vertex positions, through the vertex normals), and the
  colour-map gradient by exact linearity.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from oracle import raster
from paper_2107_05509_amd import scene

SHADING = scene.SHADING


def _cam(W=40, H=32, f=60.0):
    R = np.eye(3, dtype=np.float32).reshape(9)
    o = np.array([0.0, 0.0, -1.0], np.float32)
    return R, o, np.array([f, f, W / 2.0, H / 2.0], np.float32), W, H


def _tab(cams):
    R = np.stack([c[0] for c in cams]).astype(np.float32)
    o = np.stack([c[1] for c in cams]).astype(np.float32)
    intr = np.stack([c[2] for c in cams]).astype(np.float32)
    wh = np.array([[c[3], c[4]] for c in cams], np.int32)
    off = np.zeros(len(cams) + 1, np.int64)
    off[1:] = np.cumsum([c[3] * c[4] for c in cams])
    return dict(R=R, o=o, intr=intr, wh=wh, hand=np.zeros(len(cams), np.int32), pix_off=off)


@pytest.mark.parametrize("flip", [False, True])
def test_coverage_is_exact_point_in_triangle(flip):
    R, o, intr, W, H = _cam()
    v = np.array([[-0.21, -0.13, 0.05], [0.26, -0.07, 0.1], [0.02, 0.24, -0.04]], np.float32)
    faces = np.array([[0, 2, 1] if flip else [0, 1, 2]])
    face = raster.raster_view(v, faces, R, o, intr, W, H)
    px, py, _ = raster.project(v, R, o, *intr)
    P = [(Fraction(float(x)), Fraction(float(y))) for x, y in zip(px, py)]
    a, b, c = (P[i] for i in faces[0])
    want = np.zeros((H, W), bool)
    dmin = 1.0
    for i in range(H):
        for j in range(W):
            p = (Fraction(2 * j + 1, 2), Fraction(2 * i + 1, 2))
            e = [(q[0] - s[0]) * (p[1] - s[1]) - (q[1] - s[1]) * (p[0] - s[0]) for s, q in ((b, c), (c, a), (a, b))]
            dmin = min(dmin, min(abs(float(x)) for x in e))
            want[i, j] = all(x >= 0 for x in e) or all(x <= 0 for x in e)
    assert dmin > 1e-9   # no centre within rounding of an edge: float64 signs are the exact signs
    assert want.sum() > 50
    assert np.array_equal(face >= 0, want)
    assert set(np.unique(face)) <= {-1, 0}


def test_nearest_wins_and_ties_take_the_smaller_index():
    R, o, intr, W, H = _cam()
    near = np.array([[-0.2, -0.15, 0.0], [0.25, -0.1, 0.0], [0.0, 0.22, 0.0]], np.float32)
    # the same screen triangle twice as far from the camera (o = (0,0,-1))
    far = (o + 2.0 * (near - o)).astype(np.float32)
    v = np.concatenate([far, near, near])
    faces = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
    face = raster.raster_view(v, faces, R, o, intr, W, H)
    cov = face >= 0
    assert cov.sum() > 50
    assert np.all(face[cov] == 1)          # nearer than face 0, tie with 2 -> smaller index
    # listed alone, the far copy covers the same centres
    assert np.array_equal(raster.raster_view(v, faces[:1], R, o, intr, W, H) == 0, cov)


def test_depth_is_perspective_correct():
    R, o, intr, W, H = _cam()
    v = np.array([[-0.25, -0.2, 0.3], [0.3, -0.1, -0.2], [-0.05, 0.25, 0.05]], np.float32)
    face, zinv = raster.raster_view(v, np.array([[0, 1, 2]]), R, o, intr, W, H, want_zinv=True)
    fx, fy, cx, cy = (float(t) for t in intr)
    vc = v.astype(np.float64) - o.astype(np.float64)   # camera frame (R = I)
    nrm = np.cross(vc[1] - vc[0], vc[2] - vc[0])
    ii, jj = np.nonzero(face >= 0)
    assert len(ii) > 50
    for i, j in zip(ii, jj):
        d = np.array([(j + 0.5 - cx) / fx, (i + 0.5 - cy) / fy, 1.0])
        t = nrm @ vc[0] / (nrm @ d)    # ray t d with d_z = 1: z = t
        assert abs(zinv[i, j] * t - 1.0) < 1e-12


def test_flat_triangle_image():
    R, o, intr, W, H = _cam()
    v = np.array([[-0.2, -0.15, 0.0], [0.25, -0.1, 0.05], [0.0, 0.22, -0.05]], np.float32)
    faces = np.array([[0, 1, 2]])
    tab = _tab([(R, o, intr, W, H)])
    fpp = raster.raster_faces(v[None], faces, tab)
    vt = torch.as_tensor(v.astype(np.float64))[None]
    nrm = oracle.vertex_normals(vt, torch.as_tensor(faces))
    a = np.array([0.3, 0.55, 0.8])
    albedo = torch.as_tensor(np.broadcast_to(a, (4, 4, 3)).copy())[None]
    bg = np.random.default_rng(0).uniform(size=(W * H, 3))
    uv = np.zeros((3, 2))
    img = raster.raster_image(vt, nrm, uv, albedo, bg, faces, tab, SHADING, fpp).numpy()
    n = np.cross(v[1].astype(np.float64) - v[0], v[2].astype(np.float64) - v[0])
    n /= np.linalg.norm(n)
    light = np.array([float(np.float32(c)) for c in SHADING[2:5]])
    shade = float(np.float32(SHADING[0])) + float(np.float32(SHADING[1])) * max(0.0, n @ light)
    want = np.where((fpp >= 0)[:, None], a[None] * shade, bg)
    assert (fpp >= 0).sum() > 50
    assert np.abs(img - want).max() < 1e-14


@pytest.fixture(scope="module")
def tiny():
    w = scene.workload_tiny(3)
    om = oracle.Model(w.model)
    v, _ = oracle.skin(om, torch.as_tensor(np.asarray(w.params_init, np.float64)))
    v32 = v.numpy().astype(np.float32)
    tab = scene.camera_arrays(w.cams)
    fpp = raster.raster_faces(v32, w.model.faces, tab)
    return w, om, v32, tab, fpp


def _image(w, om, tab, fpp, v64, alb):
    nrm = oracle.vertex_normals(v64, om.faces)
    return raster.raster_image(v64, nrm, w.model.uv, alb, w.packed_background(), w.model.faces, tab, SHADING, fpp)


def test_gradient_matches_central_differences(tiny):
    w, om, v32, tab, fpp = tiny
    assert (fpp >= 0).mean() > 0.02
    rng = np.random.default_rng(1)
    wts = torch.as_tensor(rng.normal(size=(len(fpp), 3)))
    alb = torch.as_tensor(np.asarray(w.albedo_true, np.float64))
    v = torch.as_tensor(v32.astype(np.float64)).requires_grad_(True)
    (wts * _image(w, om, tab, fpp, v, alb)).sum().backward()
    g = v.grad.numpy()
    eps = 1e-7
    for k in range(6):
        d = rng.normal(size=v32.shape)
        d /= np.linalg.norm(d)
        vals = []
        for s in (1.0, -1.0):
            vs = v32.astype(np.float64) + s * eps * d
            # coverage held fixed: the perturbation must not move any centre across an edge
            assert np.array_equal(raster.raster_faces(vs.astype(np.float32), w.model.faces, tab), fpp)
            vals.append(float((wts * _image(w, om, tab, fpp, torch.as_tensor(vs), alb)).sum()))
        fd = (vals[0] - vals[1]) / (2 * eps)
        an = float((g * d).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, fd, an)


def test_colour_map_gradient_is_linear(tiny):
    w, om, v32, tab, fpp = tiny
    rng = np.random.default_rng(2)
    wts = torch.as_tensor(rng.normal(size=(len(fpp), 3)))
    v = torch.as_tensor(v32.astype(np.float64))
    a0 = np.asarray(w.albedo_true, np.float64)
    alb = torch.as_tensor(a0).requires_grad_(True)
    L0 = (wts * _image(w, om, tab, fpp, v, alb)).sum()
    L0.backward()
    delta = rng.normal(size=a0.shape)
    L1 = float((wts * _image(w, om, tab, fpp, v, torch.as_tensor(a0 + delta))).sum())
    assert abs((L1 - float(L0.detach())) - float((alb.grad.numpy() * delta).sum())) < 1e-9 * max(1.0, abs(L1))


def test_interpolated_normal_and_linear_texture():
    # distinct unit vertex normals and texture coordinates, a colour map that
    # is affine in the texel grid: at every covered centre the colour is the
    # affine map at (u W - 1/2, v H - 1/2) (bilinear with texel centres is
    # exact on affine data away from the clamped border) times
    # ka + kd max(0, n.l), n the renormalised barycentric mix of the vertex
    # normals; barycentrics from an independent camera-space solve
    R, o, intr, W, H = _cam()
    v = np.array([[-0.22, -0.16, 0.04], [0.27, -0.09, -0.06], [0.01, 0.24, 0.08]], np.float32)
    faces = np.array([[0, 1, 2]])
    tab = _tab([(R, o, intr, W, H)])
    fpp = raster.raster_faces(v[None], faces, tab)
    rng = np.random.default_rng(5)
    nv = rng.normal(size=(3, 3)) + np.array([0.0, 0.0, -2.0])
    nv /= np.linalg.norm(nv, axis=1, keepdims=True)
    uv = np.array([[0.2, 0.25], [0.75, 0.3], [0.4, 0.8]])
    th, tw = 16, 24
    ii, jj = np.meshgrid(np.arange(th), np.arange(tw), indexing="ij")
    coef = np.array([[0.1, 0.02, 0.01], [0.2, 0.005, 0.03], [0.3, 0.015, 0.02]])   # (const, per column, per row)
    tex = np.stack([c[0] + c[1] * jj + c[2] * ii for c in coef], -1)
    img = raster.raster_image(torch.as_tensor(v.astype(np.float64))[None], torch.as_tensor(nv)[None], uv,
                              torch.as_tensor(tex)[None], np.zeros((W * H, 3)), faces, tab, SHADING, fpp).numpy()
    fx, fy, cx, cy = (float(t) for t in intr)
    vc = v.astype(np.float64) - o.astype(np.float64)
    light = np.array([float(np.float32(c)) for c in SHADING[2:5]])
    ka, kd = float(np.float32(SHADING[0])), float(np.float32(SHADING[1]))
    cov = np.nonzero(fpp >= 0)[0]
    assert len(cov) > 50
    for p in cov:
        i, j = divmod(int(p), W)
        d = np.array([(j + 0.5 - cx) / fx, (i + 0.5 - cy) / fy, 1.0])
        # t d = b0 v0 + b1 v1 + b2 v2, b0 + b1 + b2 = 1
        A = np.zeros((4, 4))
        A[:3, 0] = -d
        A[:3, 1:] = vc.T
        A[3, 1:] = 1.0
        b = np.linalg.solve(A, np.array([0.0, 0.0, 0.0, 1.0]))[1:]
        u_, v_ = b @ uv
        n = b @ nv
        n /= np.linalg.norm(n)
        x, y = u_ * tw - 0.5, v_ * th - 0.5
        col = np.array([c[0] + c[1] * x + c[2] * y for c in coef])
        want = col * (ka + kd * max(0.0, n @ light))
        assert np.abs(img[p] - want).max() < 1e-12, (p, img[p], want)
