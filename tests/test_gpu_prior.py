"""The joint prior lambda E2 (paper Section 3.2, Eq. 5) on the HIP path, through the
C ABI, against the oracle: its gradient with respect to the hand parameters
(the difference of two backwards, with and without the prior, on the same
inputs) and its value in the loss of a whole iteration.  Bars: 1e-4 relative
per parameter block for the gradient, 1e-5 relative for lambda E2."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, Case, block_rel, f32
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu

LAM, GAMMA = 5.0, 0.005


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, seed 0, joint prior", flush=True)
    c = Case(scene.workload_tiny(0))
    rng = np.random.default_rng(11)
    _, j = oracle.skin(c.om, torch.as_tensor(c.params.astype(np.float64)))
    # targets near the posed joints: coordinates in both regimes of f2
    c.jtarget = f32(j.numpy() + rng.normal(0, 0.008, j.shape))
    return c


def _oracle_prior(c):
    p = torch.as_tensor(c.params.astype(np.float64)).requires_grad_(True)
    _, j = oracle.skin(c.om, p)
    e = oracle.joint_prior(j, c.jtarget.astype(np.float64), LAM, GAMMA)
    e.sum().backward()
    return e.detach().numpy(), p.grad.numpy()


def _gpu_grad(c, dimage):
    gp = torch.empty(1, 64, device=DEV)
    ga = torch.empty(1, c.th, c.tw, 3, device=DEV)
    c.gsc.backward(c.t(c.params), c.t(c.v32), c.t(c.albedo), c.t(c.bg), c.t(dimage), 0, gp, ga)
    torch.cuda.synchronize()
    return gp.cpu().numpy()


def test_prior_gradient(case):
    c = case
    img = f32(c.oracle_render(0))
    rng = np.random.default_rng(2)
    tgt = np.clip(img + rng.normal(0, 0.1, img.shape), 0, 1)
    _, d = oracle.l1_loss(img, tgt, None, c.tab["pix_off"], c.tab["hand"], 1)
    d = f32(d)
    g0 = _gpu_grad(c, d)
    c.gsc.set_joint_prior(c.t(c.jtarget), LAM, GAMMA)
    try:
        g1 = _gpu_grad(c, d)
    finally:
        c.gsc.set_joint_prior(None)
    g_off = _gpu_grad(c, d)
    _, og = _oracle_prior(c)
    assert np.abs(og).max() > 0.1   # the prior's part dominates the atomics' reordering noise
    for name, sl in {"pose": slice(0, 48), "shape": slice(48, 58), "global": slice(58, 64)}.items():
        e = block_rel((g1 - g0)[:, sl], og[:, sl])
        print(name, e, flush=True)
        assert e <= 1e-4, name
    # switched off again: the E1 gradient alone
    assert block_rel(g_off, g0) <= 1e-5


def test_prior_in_iteration_loss(case):
    c = case
    img = f32(c.oracle_render(0))
    rng = np.random.default_rng(3)
    tgt = f32(np.clip(img + rng.normal(0, 0.1, img.shape), 0, 1))
    lrs = (0.0,) * 6
    losses = []
    for with_prior in (False, True):
        st = c.gsc.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), c.t(tgt))
        if with_prior:
            c.gsc.set_joint_prior(c.t(c.jtarget), LAM, GAMMA)
        try:
            c.gsc.iterate(st, lrs)
            torch.cuda.synchronize()
        finally:
            c.gsc.set_joint_prior(None)
        losses.append(st.loss.cpu().numpy().astype(np.float64))
    e2, _ = _oracle_prior(c)
    diff = losses[1] - losses[0]
    print("lambda E2", diff, e2, flush=True)
    assert np.abs(diff - e2).max() <= 1e-5 * np.abs(e2).max() + 1e-6 * np.abs(losses[0]).max()


def test_prior_argument_errors(case):
    c = case
    for lam, gamma in ((-1.0, 0.005), (1.0, 0.0), (1.0, -0.1), (float("nan"), 0.005), (1.0, float("inf"))):
        with pytest.raises(binding.HRError):
            c.gsc.set_joint_prior(c.t(c.jtarget), lam, gamma)
    with pytest.raises(binding.HRError):
        c.gsc.set_joint_prior(c.t(c.jtarget[:, :4]), 1.0, 0.005)   # wrong shape


def test_prior_in_graphs():
    # a graph captured after hr_set_joint_prior carries the prior: one
    # iteration replayed from a saved state equals hr_iterate with the prior,
    # and differs from the prior-free iteration
    from test_gpu_loop import Loop, _restore, _save, _snap
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, joint prior in graphs", flush=True)
    lp = Loop(scene.workload_tiny(0))
    g = lp.g
    v = torch.empty(1, lp.w.model.n_verts, 3, device=DEV)
    j = torch.empty(1, g.J, 3, device=DEV)
    g.skin(torch.as_tensor(f32(lp.w.params_init)).to(DEV), v, j)
    target = (j + 0.01).contiguous()
    g.set_joint_prior(target, LAM, GAMMA)
    try:
        r = lp.refiner(warm=0)
        r.run(2, graph=False)
        saved = _save(r)
        outs = []
        for graph in (True, False):
            _restore(r, saved)
            r.run(1, graph=graph)
            outs.append(_snap(r))
    finally:
        g.set_joint_prior(None)
    _restore(r, saved)
    r.run(1, graph=False)
    off = _snap(r)
    for key in ("params", "loss", "grad_params"):
        e = block_rel(outs[0][key], outs[1][key])
        print(key, e, flush=True)
        assert e <= 1e-5, key
    assert block_rel(off["grad_params"], outs[1]["grad_params"]) > 1e-2
    assert outs[1]["loss"][0] > off["loss"][0]
