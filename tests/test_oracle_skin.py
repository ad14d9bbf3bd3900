"""Pins of the oracle's skinning and normals (paper Section 3.1 'Geometry', the
decoders G_v and G_J): library rotations, special cases with closed forms, and
central finite differences of the autograd gradient."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

import oracle
from paper_2107_05509_amd import scene


@pytest.fixture(scope="module")
def model(hand_model):
    return oracle.Model(hand_model)


def test_rodrigues_matches_scipy():
    rng = np.random.default_rng(0)
    r = rng.normal(0, 1.0, (200, 3))
    r[:20] *= 1e-6   # tiny angles take the series branch
    r[20:30] *= 3.0
    R = oracle.rodrigues(torch.as_tensor(r)).numpy()
    ref = Rotation.from_rotvec(r).as_matrix()
    assert np.abs(R - ref).max() < 1e-13


def test_rest_pose_is_template(model, hand_model):
    v, j = oracle.skin(model, torch.zeros(1, 64, dtype=torch.float64))
    assert np.abs(v[0].numpy() - hand_model.v_template).max() < 1e-15
    assert np.allclose(j[0].numpy(), hand_model.j_regressor @ hand_model.v_template, atol=1e-15)


def test_shape_only_is_linear(model, hand_model):
    rng = np.random.default_rng(1)
    p = np.zeros((1, 64))
    p[0, scene.SHAPE] = rng.standard_normal(10)
    v, _ = oracle.skin(model, torch.as_tensor(p))
    ref = hand_model.v_template + hand_model.shapedirs @ p[0, scene.SHAPE]
    assert np.abs(v[0].numpy() - ref).max() < 1e-15


def test_global_transform_is_rigid(model, hand_model):
    rng = np.random.default_rng(2)
    p = np.zeros((1, 64))
    p[0, scene.ROT] = rng.normal(0, 1, 3)
    p[0, scene.TRANS] = rng.normal(0, 0.1, 3)
    v, _ = oracle.skin(model, torch.as_tensor(p))
    ref = Rotation.from_rotvec(p[0, scene.ROT]).apply(hand_model.v_template) + p[0, scene.TRANS]
    assert np.abs(v[0].numpy() - ref).max() < 1e-14


def test_root_joint_rotates_about_root(model, hand_model):
    p = np.zeros((1, 64))
    p[0, 0:3] = [0.3, -0.2, 0.5]
    v, j = oracle.skin(model, torch.as_tensor(p))
    J0 = hand_model.j_regressor[0] @ hand_model.v_template
    ref = Rotation.from_rotvec(p[0, 0:3]).apply(hand_model.v_template - J0) + J0
    assert np.abs(v[0].numpy() - ref).max() < 1e-14


def test_finger_joint_moves_only_its_chain(model, hand_model):
    # rotate the middle finger's second joint (joint 2 + 3*3 = 8)
    jt = 8
    p = np.zeros((1, 64))
    p[0, 3 * jt:3 * jt + 3] = [0.0, 0.0, 0.7]
    v, j = oracle.skin(model, torch.as_tensor(p))
    v = v[0].numpy()
    W = hand_model.weights
    chain = [jt, jt + 1]
    untouched = W[:, chain].sum(1) == 0
    assert np.abs(v[untouched] - hand_model.v_template[untouched]).max() < 1e-15
    rigid = W[:, chain].sum(1) > 1 - 1e-12
    Jr = hand_model.j_regressor @ hand_model.v_template
    ref = Rotation.from_rotvec([0, 0, 0.7]).apply(hand_model.v_template[rigid] - Jr[jt]) + Jr[jt]
    assert rigid.sum() > 10
    assert np.abs(v[rigid] - ref).max() < 1e-14


def test_skin_gradient_matches_central_differences(model):
    rng = np.random.default_rng(3)
    p0 = scene.true_params(rng)[None]
    p0[0, 0:3] = rng.normal(0, 0.2, 3)
    p0[0, scene.TRANS] = rng.normal(0, 0.05, 3)
    w = torch.as_tensor(rng.standard_normal((1, 778, 3)))
    wj = torch.as_tensor(rng.standard_normal((1, 16, 3)))
    p = torch.as_tensor(p0).requires_grad_(True)
    v, j = oracle.skin(model, p)
    ((v * w).sum() + (j * wj).sum()).backward()
    g = p.grad.numpy()[0]
    h = 1e-6
    for k in range(64):
        d = np.zeros((1, 64))
        d[0, k] = h
        vp, jp = oracle.skin(model, torch.as_tensor(p0 + d))
        vm, jm = oracle.skin(model, torch.as_tensor(p0 - d))
        fd = (((vp - vm) * w).sum() + ((jp - jm) * wj).sum()).item() / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_normals_closed_forms():
    # planar fan: every vertex normal is the plane normal
    rng = np.random.default_rng(4)
    ang = np.sort(rng.uniform(0, 2 * np.pi, 7))
    pts = np.c_[np.cos(ang), np.sin(ang), np.zeros(7)]
    verts = np.vstack([[0, 0, 0], pts])
    faces = np.array([[0, 1 + i, 1 + (i + 1) % 7] for i in range(7)])
    n = oracle.vertex_normals(torch.as_tensor(verts[None]), torch.as_tensor(faces)).numpy()[0]
    assert np.abs(n - [0, 0, 1]).max() < 1e-15
    # regular tetrahedron: vertex normals point away from the centroid
    t = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64)
    f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]])
    n = oracle.vertex_normals(torch.as_tensor(t[None]), torch.as_tensor(f)).numpy()[0]
    assert np.abs(n - t / np.sqrt(3)).max() < 1e-15
