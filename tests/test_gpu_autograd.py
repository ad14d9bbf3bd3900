"""torch.autograd wrappers of the C ABI: forward and backward must equal the
raw hr_* calls on the same samples (images bit for bit, gradients within the
atomic-order tolerance), and the loss wrapper must chain the incoming gradient
per hand."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, block_rel, f32
from paper_2107_05509_amd import autograd as hra
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype)


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = scene.workload_batched(1, n_hands=2, spp=4)
    print("case: batched 2 hands,", len(w.cams), "views", flush=True)
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=8)
    return w, g


def test_render_images_matches_raw(case):
    w, g = case
    p = _t(f32(w.params_init)).requires_grad_(True)
    alb = _t(f32(w.albedo_true)).requires_grad_(True)
    bg = _t(f32(w.packed_background()))
    img = hra.render_images(g, p, alb, bg, it=3)
    d = _t(np.random.default_rng(0).normal(size=(g.P, 3)).astype(np.float32))
    gp, ga = torch.autograd.grad(img, (p, alb), d)
    # raw calls
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(p.detach(), v)
    ref = torch.empty(g.P, 3, device=DEV)
    g.render(v, alb.detach(), bg, 3, ref)
    rp, ra = torch.empty_like(gp), torch.empty_like(ga)
    g.backward(p.detach(), v, alb.detach(), bg, d, 3, rp, ra)
    torch.cuda.synchronize()
    assert torch.equal(img.detach(), ref)
    assert block_rel(gp.cpu().numpy(), rp.cpu().numpy()) <= 1e-5
    assert block_rel(ga.cpu().numpy(), ra.cpu().numpy()) <= 1e-5
    assert gp.abs().sum() > 0


def test_photometric_loss_matches_raw(case):
    w, g = case
    p = _t(f32(w.params_init)).requires_grad_(True)
    alb = _t(f32(w.albedo_init)).requires_grad_(True)
    bg = _t(f32(w.packed_background()))
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(_t(f32(w.params_true)), v)
    target = torch.empty(g.P, 3, device=DEV)
    g.render(v, _t(f32(w.albedo_true)), bg, 50, target)
    loss = hra.photometric_loss(g, w.cams, p, alb, bg, target, None, it=1)
    weights = torch.tensor([0.25, 2.0], device=DEV)
    (loss * weights).sum().backward()
    # raw: per-hand dimage scaled by the hand's weight
    g.skin(p.detach(), v)
    img = torch.empty(g.P, 3, device=DEV)
    g.render(v, alb.detach(), bg, 1, img)
    rl = torch.empty(w.n_hands, device=DEV)
    dimg = torch.empty(g.P, 3, device=DEV)
    g.loss(img, target, None, rl, dimg)
    off = w.pixel_offsets()
    for i, c in enumerate(w.cams):
        dimg[int(off[i]):int(off[i + 1])] *= weights[c.hand]
    rp = torch.empty(w.n_hands, 64, device=DEV)
    ra = torch.empty_like(alb)
    g.backward(p.detach(), v, alb.detach(), bg, dimg, 1, rp, ra)
    torch.cuda.synchronize()
    assert torch.equal(loss.detach(), rl)
    assert block_rel(p.grad.cpu().numpy(), rp.cpu().numpy()) <= 1e-5
    assert block_rel(alb.grad.cpu().numpy(), ra.cpu().numpy()) <= 1e-5


def test_wrappers_leave_a_set_joint_prior_out(case):
    # with a joint prior set on the scene (hr_iterate's objective), the
    # wrappers still return and differentiate the data term alone
    w, g = case
    p0 = _t(f32(w.params_init))
    alb0 = _t(f32(w.albedo_init))
    bg = _t(f32(w.packed_background()))
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(_t(f32(w.params_true)), v)
    target = torch.empty(g.P, 3, device=DEV)
    g.render(v, _t(f32(w.albedo_true)), bg, 50, target)
    weights = torch.tensor([0.25, 2.0], device=DEV)

    d = _t(np.random.default_rng(5).normal(size=(g.P, 3)).astype(np.float32))

    def grads():
        p = p0.clone().requires_grad_(True)
        alb = alb0.clone().requires_grad_(True)
        loss = hra.photometric_loss(g, w.cams, p, alb, bg, target, None, it=1)
        (loss * weights).sum().backward()
        pi = p0.clone().requires_grad_(True)
        img = hra.render_images(g, pi, alb0, bg, it=2)
        (gi,) = torch.autograd.grad(img, (pi,), d)
        torch.cuda.synchronize()
        return loss.detach().clone(), p.grad.clone(), alb.grad.clone(), gi

    l0, gp0, ga0, gi0 = grads()
    jt = torch.empty(w.n_hands, g.J, 3, device=DEV)
    g.skin(p0, torch.empty(w.n_hands, g.V, 3, device=DEV), jt)
    jt = (jt + 0.02).contiguous()     # 2 cm off: the prior's gradient is large
    g.set_joint_prior(jt, 1.0, 0.005)
    try:
        l1, gp1, ga1, gi1 = grads()
        # the raw backward without HR_SKIP_PRIOR does include it
        g.skin(p0, v)
        img = torch.empty(g.P, 3, device=DEV)
        g.render(v, alb0, bg, 1, img)
        rl = torch.empty(w.n_hands, device=DEV)
        dimg = torch.empty(g.P, 3, device=DEV)
        g.loss(img, target, None, rl, dimg)
        rp = torch.empty(w.n_hands, 64, device=DEV)
        g.backward(p0, v, alb0, bg, dimg, 1, rp, torch.empty_like(alb0))
        rs = torch.empty_like(rp)
        g.backward(p0, v, alb0, bg, dimg, 1, rs, torch.empty_like(alb0),
                   flags=binding.HR_GRAD_ALL | binding.HR_SKIP_PRIOR)
        torch.cuda.synchronize()
    finally:
        g.set_joint_prior(None)
    assert torch.equal(l0, l1)
    assert block_rel(gp1.cpu().numpy(), gp0.cpu().numpy()) <= 1e-5
    assert block_rel(ga1.cpu().numpy(), ga0.cpu().numpy()) <= 1e-5
    assert block_rel(gi1.cpu().numpy(), gi0.cpu().numpy()) <= 1e-5
    assert block_rel(rp.cpu().numpy(), rs.cpu().numpy()) > 1e-2
