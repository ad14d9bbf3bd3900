"""Pins of the oracle's joint prior (paper Section 3.2, Eq. 5: the prior term E2 of
the objective E = E1 + lambda E2): the smooth L1 function against the library
routine that defines the same function, its two regimes and their meeting
point, and the gradient through the skinning against central differences."""
import numpy as np
import pytest
import torch

import oracle
from paper_2107_05509_amd import scene


@pytest.fixture(scope="module")
def model(hand_model):
    return oracle.Model(hand_model)


def test_matches_library_smooth_l1():
    rng = np.random.default_rng(0)
    gamma, lam = 0.005, 1e-3
    x = torch.as_tensor(rng.normal(0, 0.01, (3, 16, 3)))
    y = rng.normal(0, 0.01, (3, 16, 3))
    e = oracle.joint_prior(x, y, lam, gamma).numpy()
    for h in range(3):
        ref = torch.nn.functional.smooth_l1_loss(x[h], torch.as_tensor(y[h]), reduction="sum", beta=gamma).item()
        assert abs(e[h] - lam * ref) <= 1e-15 + 1e-12 * abs(ref)
    # both regimes occur in this draw
    d = np.abs(x.numpy() - y)
    assert (d < gamma).any() and (d >= gamma).any()


def test_regimes_and_continuity():
    gamma = 0.005
    one = lambda dx: oracle.joint_prior(torch.tensor([[[dx, 0.0, 0.0]]], dtype=torch.float64),
                                        np.zeros((1, 1, 3)), 1.0, gamma).item()
    assert one(0.0) == 0.0
    assert abs(one(0.002) - 0.5 * 0.002 ** 2 / gamma) < 1e-18     # quadratic below gamma
    assert abs(one(-0.03) - (0.03 - 0.5 * gamma)) < 1e-15          # linear above, symmetric
    assert abs(one(gamma * (1 - 1e-9)) - one(gamma)) < 1e-11        # the two meet at gamma (gamma / 2)
    assert abs(one(gamma) - 0.5 * gamma) < 1e-15


def test_prior_gradient_matches_central_differences(model):
    rng = np.random.default_rng(5)
    p0 = scene.true_params(rng)[None]
    p0[0, scene.TRANS] = rng.normal(0, 0.05, 3)
    gamma, lam = 0.005, 0.7
    _, j0 = oracle.skin(model, torch.as_tensor(p0))
    # targets near the joints: some coordinates inside gamma, most outside
    target = j0.numpy() + rng.normal(0, 0.008, j0.shape)
    p = torch.as_tensor(p0).requires_grad_(True)
    _, j = oracle.skin(model, p)
    oracle.joint_prior(j, target, lam, gamma).sum().backward()
    g = p.grad.numpy()[0]
    h = 1e-7
    for k in range(64):
        d = np.zeros((1, 64))
        d[0, k] = h
        _, jp = oracle.skin(model, torch.as_tensor(p0 + d))
        _, jm = oracle.skin(model, torch.as_tensor(p0 - d))
        fd = (oracle.joint_prior(jp, target, lam, gamma) - oracle.joint_prior(jm, target, lam, gamma)).item() / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])
