"""Pins of the oracle's interior adjoint (the derivative of the Monte Carlo
estimate with the samples held fixed): central finite differences of the
oracle's own forward with common random numbers, and exact linearity in the
albedo (a dot-product test)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2107_05509_amd import scene


@pytest.fixture(scope="module")
def setup():
    w = scene.workload_tiny(1)
    m = oracle.Model(w.model)
    cam = scene.camera_arrays(w.cams[:2])
    sc = oracle.Scene(w.model.faces, w.model.uv, cam, scene.SHADING, w.model.edges, w.model.edge_faces)
    v, _ = oracle.skin(m, torch.as_tensor(w.params_true))
    n = oracle.vertex_normals(v, m.faces)
    rng = np.random.default_rng(2)
    g = rng.normal(0, 1, (sc.P, 3))
    bg = np.concatenate([b.reshape(-1, 3) for b in w.backgrounds[:2]]).astype(np.float32).astype(np.float64)
    alb = w.albedo_true.astype(np.float32).astype(np.float64)
    return sc, v.numpy(), n.numpy(), alb, bg, g


SPP, SEED, IT = 4, 9, 2


def _L(sc, v, n, alb, bg, g):
    img, hits = oracle.render(sc, v, n, alb, bg, SPP, SEED, IT, want_hits=True)
    return (img * g).sum(), hits


def test_albedo_gradient_is_exact_adjoint(setup):
    sc, v, n, alb, bg, g = setup
    ga, gv, gn = oracle.backward_interior(sc, v, n, alb, g, SPP, SEED, IT)
    rng = np.random.default_rng(3)
    d = rng.normal(0, 1, alb.shape)
    L0, _ = _L(sc, v, n, alb, bg, g)
    L1, _ = _L(sc, v, n, alb + 1e-3 * d, bg, g)
    assert abs((L1 - L0) / 1e-3 - (ga * d).sum()) <= 1e-9 * abs((ga * d).sum()) + 1e-12


def test_vertex_gradient_matches_crn_differences(setup):
    sc, v, n, alb, bg, g = setup
    ga, gv, gn = oracle.backward_interior(sc, v, n, alb, g, SPP, SEED, IT)
    _, hits0 = _L(sc, v, n, alb, bg, g)
    idx = np.argsort(-np.abs(gv[0]).sum(1))[:12]
    # small step: the bilinear texture and the clamped shading have kinks, and
    # the finite-difference error from samples straddling them grows with h
    h = 1e-7
    checked = 0
    for vi in idx:
        for k in range(3):
            vp = v.copy(); vp[0, vi, k] += h
            vm = v.copy(); vm[0, vi, k] -= h
            Lp, hp = _L(sc, vp, n, alb, bg, g)
            Lm, hm = _L(sc, vm, n, alb, bg, g)
            if not (np.array_equal(hp, hits0) and np.array_equal(hm, hits0)):
                continue  # a sample changed face: finite differences see a jump
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - gv[0, vi, k]) <= 1e-6 * max(abs(gv[0, vi, k]), 1e-3), (vi, k, fd, gv[0, vi, k])
            checked += 1
    assert checked >= 30


def test_normal_gradient_matches_differences(setup):
    sc, v, n, alb, bg, g = setup
    ga, gv, gn = oracle.backward_interior(sc, v, n, alb, g, SPP, SEED, IT)
    idx = np.argsort(-np.abs(gn[0]).sum(1))[:10]
    h = 1e-6
    for vi in idx:
        for k in range(3):
            npl = n.copy(); npl[0, vi, k] += h
            nmi = n.copy(); nmi[0, vi, k] -= h
            fd = (_L(sc, v, npl, alb, bg, g)[0] - _L(sc, v, nmi, alb, bg, g)[0]) / (2 * h)
            assert abs(fd - gn[0, vi, k]) <= 1e-6 * max(abs(gn[0, vi, k]), 1e-3), (vi, k)
