"""Pins of the oracle's loss (the colour term D_c of Eq. 4 summed over views as
in Eq. 3) and optimiser step (Adam, Section 3.3) against torch's library
implementations (F.l1_loss with autograd, torch.optim.Adam), in float64."""
import numpy as np
import torch
import torch.nn.functional as Fn

import oracle


def test_l1_loss_matches_torch():
    rng = np.random.default_rng(0)
    sizes = [30, 0, 50, 20]
    off = np.concatenate([[0], np.cumsum(sizes)])
    P = off[-1]
    img = rng.uniform(0, 1, (P, 3))
    tgt = rng.uniform(0, 1, (P, 3))
    tgt[5] = img[5]  # exact ties: sign(0) = 0
    mask = rng.uniform(0, 1, P) < 0.7
    view_hand = np.array([0, 0, 1, 1])
    loss, dimg = oracle.l1_loss(img, tgt, mask, off, view_hand, 2)
    I = torch.as_tensor(img).requires_grad_(True)
    O = torch.as_tensor(tgt)
    ref = torch.zeros(2, dtype=torch.float64)
    for v in range(4):
        a, b = off[v], off[v + 1]
        m = torch.as_tensor(mask[a:b])
        if m.sum() == 0:
            continue
        ref[view_hand[v]] = ref[view_hand[v]] + Fn.l1_loss(I[a:b][m], O[a:b][m], reduction="mean")
    ref.sum().backward()
    assert np.allclose(loss, ref.detach().numpy(), rtol=1e-15, atol=0)
    assert np.allclose(dimg, I.grad.numpy(), rtol=1e-15, atol=0)


def test_adam_matches_torch():
    rng = np.random.default_rng(1)
    x0 = rng.normal(0, 1, 50)
    lr = np.where(np.arange(50) < 40, 1e-2, 1e-3)
    lr[45:] = 0.0  # frozen entries
    grads = rng.normal(0, 1, (7, 50))
    x, m, v = x0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        x, m, v = oracle.adam_step(x, grads[t - 1], m, v, t, lr)
    # reference: one torch optimiser per distinct learning rate
    for val in (1e-2, 1e-3):
        idx = np.nonzero(lr == val)[0]
        p = torch.as_tensor(x0[idx].copy()).requires_grad_(True)
        opt = torch.optim.Adam([p], lr=val, betas=(0.9, 0.999), eps=1e-8)
        for t in range(7):
            p.grad = torch.as_tensor(grads[t, idx])
            opt.step()
        assert np.allclose(x[idx], p.detach().numpy(), rtol=0, atol=1e-15)
    assert np.array_equal(x[45:], x0[45:])


def test_adam_clamp():
    x, m, v = oracle.adam_step(np.array([0.999, 0.001]), np.array([-1.0, 1.0]), np.zeros(2), np.zeros(2),
                               1, 0.1, lo=0.0, hi=1.0)
    assert x[0] == 1.0 and x[1] == 0.0
