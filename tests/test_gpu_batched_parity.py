"""Parity with the oracle on a batched scene: three hands of the same model
with uneven view counts (3, 1, 2) and mixed resolutions (64x64, 48x32,
96x64), the hands' views interleaved in the camera list, 4 spp.  Every
per-hand and per-view index of the HIP path (hand of a view, a hand's views,
packed pixel offsets, per-hand colour maps and parameters) is exercised.

Through the separate calls (render, loss, backward) both sides take the same
float32 vertices (the oracle's skinning rounded): hit ids bit-exact, images
1e-5 relative, gradients 1e-4 per block and element-wise.  Through
hr_iterate the GPU skins the hand itself (float64 arithmetic rounded to
float32: the oracle's vertices rounded, bar a rare tie that moves a
coordinate by one ulp), so a ray grazing an edge could pick the other
triangle: at most 1e-4 of the samples may differ, the loss within the L1
effect of the differing pixels, and the interior gradient within 1e-4 per
block plus what those samples and the vertices' rounding move the oracle's
own gradient by."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, Case, block_rel, check_grad, f32, rel_err
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu

LRS = (1e-2, 1e-2, 1e-2, 1e-2, 1e-3, 1e-2)
BLOCKS = {"pose": slice(0, 48), "shape": slice(48, 58), "global": slice(58, 64)}


@pytest.fixture(scope="module")
def mixed():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: mixed batch, 3 hands, views (3, 1, 2) of 64x64 / 48x32 / 96x64, 4 spp", flush=True)
    return Case(scene.workload_mixed(0))


def _hand_views(c):
    hands = np.asarray(c.tab["hand"])
    return [list(np.nonzero(hands == h)[0]) for h in range(c.w.n_hands)]


def _target(c):
    """Targets rendered by the oracle from the true parameters at 64 spp."""
    vt, _ = oracle.skin(c.om, torch.as_tensor(f32(c.w.params_true).astype(np.float64)))
    nt = oracle.vertex_normals(vt, c.om.faces)
    return f32(oracle.render(c.osc, vt.numpy(), nt.numpy(), c.albedo, c.bg, 64, 777, 0))


def _mask(c):
    m = (np.random.default_rng(9).uniform(size=c.P) < 0.85).astype(np.uint8)
    return m


def _gpu_backward(c, dimage, flags):
    H = c.w.n_hands
    gp = torch.empty(H, 64, device=DEV)
    ga = torch.empty(H, c.th, c.tw, 3, device=DEV)
    gv = torch.empty(H, c.model.n_verts, 3, device=DEV)
    gn = torch.empty(H, c.model.n_verts, 3, device=DEV)
    c.gsc.backward(c.t(c.params), c.t(c.v32), c.t(c.albedo), c.t(c.bg), c.t(dimage), 0, gp, ga, gv, gn, flags)
    torch.cuda.synchronize()
    return dict(ga=ga.cpu().numpy(), gn=gn.cpu().numpy(), gv=gv.cpu().numpy(), gp=gp.cpu().numpy())


def _oracle_backward(c, dimage, flags):
    v64 = c.v32.astype(np.float64)
    ga = np.zeros((c.w.n_hands, c.th, c.tw, 3))
    gv = np.zeros_like(v64)
    gn = np.zeros_like(v64)
    if flags & binding.HR_GRAD_INTERIOR:
        ga, gvi, gn = oracle.backward_interior(c.osc, v64, c.n64, c.albedo, dimage, c.w.spp, c.seed, 0)
        gv = gv + gvi
    if flags & binding.HR_GRAD_EDGES:
        gv = gv + oracle.backward_edges(c.osc, v64, c.n64, c.albedo, c.bg, dimage, c.seed, 0, 1e-3)
    p = torch.as_tensor(c.params.astype(np.float64)).requires_grad_(True)
    vs, _ = oracle.skin(c.om, p)
    vt = torch.as_tensor(v64).requires_grad_(True)
    nt = oracle.vertex_normals(vt, c.om.faces)
    torch.autograd.backward([nt], [torch.as_tensor(gn)])
    gv_total = gv + vt.grad.numpy()
    torch.autograd.backward([vs], [torch.as_tensor(gv_total)])
    return dict(ga=ga, gn=gn, gv=gv_total, gp=p.grad.numpy())


def test_render(mixed):
    c = mixed
    img_g, hit_g = c.gpu_render(0, hits=True)
    img_o, hit_o = c.oracle_render(0, hits=True)
    assert np.array_equal(hit_g, hit_o), f"hit ids differ on {(hit_g != hit_o).sum()} samples"
    off = c.tab["pix_off"]
    for v in range(len(c.cams)):   # every view sees its hand
        assert (hit_o[off[v]:off[v + 1]] >= 0).mean() > 0.01, v
    e = rel_err(img_g, img_o)
    print("image rel err max %.3g" % e.max(), flush=True)
    assert e.max() <= 1e-5


def test_loss(mixed):
    c = mixed
    img = f32(c.oracle_render(0))
    target, mask = _target(c), _mask(c)
    H = c.w.n_hands
    loss = torch.empty(H, device=DEV)
    dimg = torch.empty(c.P, 3, device=DEV)
    c.gsc.loss(c.t(img), c.t(target), c.t(mask, torch.uint8), loss, dimg)
    torch.cuda.synchronize()
    lo, do = oracle.l1_loss(img, target, mask, c.tab["pix_off"], c.tab["hand"], H)
    print("loss", loss.cpu().numpy(), lo, flush=True)
    assert np.abs(loss.cpu().numpy() - lo).max() <= 1e-5 * np.abs(lo).max()
    dg = dimg.cpu().numpy()
    assert np.array_equal(np.sign(dg), np.sign(do))
    assert rel_err(dg, do, 1e-30).max() <= 1e-6


@pytest.mark.parametrize("flags", [binding.HR_GRAD_INTERIOR, binding.HR_GRAD_EDGES,
                                   binding.HR_GRAD_INTERIOR | binding.HR_GRAD_EDGES])
def test_backward(mixed, flags):
    c = mixed
    img = f32(c.oracle_render(0))
    _, d = oracle.l1_loss(img, _target(c), _mask(c), c.tab["pix_off"], c.tab["hand"], c.w.n_hands)
    d = f32(d)
    g = _gpu_backward(c, d, flags)
    o = _oracle_backward(c, d, flags)
    tot, bud = c.gsc.edge_stats()
    _, _, tot_o, bud_o = oracle.edge_weights(c.osc, c.v32.astype(np.float64))
    assert np.array_equal(tot, tot_o) and np.array_equal(bud, bud_o)
    keys = ("ga", "gn", "gv") if flags & binding.HR_GRAD_INTERIOR else ("gv",)
    for h in range(c.w.n_hands):
        for k in keys:
            check_grad(f"hand {h} {k}", g[k][h], o[k][h])
        for name, sl in BLOCKS.items():
            check_grad(f"hand {h} {name}", g["gp"][h, sl], o["gp"][h, sl])


def test_iterate_interior_against_oracle(mixed):
    c = mixed
    H = c.w.n_hands
    target, mask = _target(c), _mask(c)
    st = c.gsc.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), c.t(target), c.t(mask, torch.uint8))
    c.gsc.iterate(st, LRS, flags=binding.HR_GRAD_INTERIOR)
    torch.cuda.synchronize()
    r = oracle.gradient(c.om, c.osc, c.params.astype(np.float64), c.albedo.astype(np.float64), c.bg, target, mask,
                        c.w.spp, c.seed, 0, edges=False)
    # the GPU's own skinning (float64 arithmetic rounded to float32): the
    # oracle's float64 vertices rounded, bar a rare tie
    verts = st.verts.cpu().numpy()
    assert np.abs(verts - r["verts"]).max() <= 1e-5 * np.abs(r["verts"]).max()
    n_off = int((verts != f32(r["verts"])).sum())
    print("vertex coordinates off the oracle's rounding:", n_off, flush=True)
    assert n_off <= 2
    # samples: at most 1e-4 of them may take another triangle (rays grazing
    # an edge, the vertices a few ulps apart)
    img = st.image.cpu().numpy()
    diff = (rel_err(img, r["image"]) > 1e-5).any(1)
    print("pixels differing", int(diff.sum()), "of", c.P, flush=True)
    assert diff.sum() <= 1e-4 * c.P * c.w.spp
    # loss: within the exact L1 effect of the differing pixels
    loss = st.loss.cpu().numpy().astype(np.float64)
    off, hands = c.tab["pix_off"], c.tab["hand"]
    bound = np.zeros(H)
    for v in range(len(c.cams)):
        sl = slice(off[v], off[v + 1])
        n = max(int(mask[sl].sum()), 1)
        bound[hands[v]] += np.abs(img[sl] - r["image"][sl])[diff[sl] & (mask[sl] != 0)].sum() / (3 * n)
    print("loss", loss, r["loss"], "bound", bound, flush=True)
    assert (np.abs(loss - r["loss"]) <= bound + 1e-5 * np.abs(r["loss"])).all()
    # gradients: 1e-4 per block, plus three times (a) the oracle's gradient of
    # the differing pixels' loss share alone (samples that took another
    # triangle) and (b) the change of the oracle's own gradient when its
    # vertices are rounded to float32 (the gradient's sensitivity to vertices
    # a few ulps apart, which the GPU's own skinning also moves them by)
    d_flip = np.where(diff[:, None], r["dimage"], 0.0)
    flip = _oracle_backward(c, d_flip, binding.HR_GRAD_INTERIOR)
    rounded = _oracle_backward(c, r["dimage"], binding.HR_GRAD_INTERIOR)
    gp = st.grad_params.cpu().numpy()
    for h in range(H):
        for name, sl in BLOCKS.items():
            ref = r["grad_params"][h, sl]
            err = np.linalg.norm(gp[h, sl] - ref)
            bar = (1e-4 * np.linalg.norm(ref) + 3 * np.linalg.norm(flip["gp"][h, sl])
                   + 3 * np.linalg.norm(rounded["gp"][h, sl] - ref))
            print(f"hand {h} {name}: |d| {err:.3g}, bar {bar:.3g}", flush=True)
            assert err <= bar, (h, name)
    ga = st.grad_albedo.cpu().numpy()
    assert np.linalg.norm(ga - r["grad_albedo"]) <= (1e-4 * np.linalg.norm(r["grad_albedo"])
                                                    + 3 * np.linalg.norm(flip["ga"])
                                                    + 3 * np.linalg.norm(rounded["ga"] - r["grad_albedo"]))
    # Adam's first step: -lr m/(sqrt(v) + eps) with m, v of this gradient
    lr = np.empty(64)
    lr[0:3], lr[3:48], lr[48:58], lr[58:61], lr[61:64] = LRS[:5]
    po, _, _ = oracle.adam_step(c.params.astype(np.float64), r["grad_params"], 0.0, 0.0, 1, lr[None])
    g = np.abs(r["grad_params"])
    firm = g > 1e-3 * g.max(1, keepdims=True)   # signs far above the rounding noise
    dp = np.abs(st.params.cpu().numpy() - po)
    assert dp[firm].max() <= 1e-6 and dp.max() <= 2 * max(LRS) + 1e-6


def test_iterate_matches_calls(mixed):
    # hr_iterate (all terms) equals the five separate calls on the batch
    c = mixed
    target, mask = c.t(_target(c)), c.t(_mask(c), torch.uint8)
    st = c.gsc.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), target, mask)
    c.gsc.iterate(st, LRS)
    g = c.gsc
    H = c.w.n_hands
    p, a = c.t(c.params), c.t(c.albedo)
    v = torch.empty(H, c.model.n_verts, 3, device=DEV)
    g.skin(p, v)
    img = torch.empty(c.P, 3, device=DEV)
    g.render(v, a, c.t(c.bg), 0, img)
    loss = torch.empty(H, device=DEV)
    d = torch.empty(c.P, 3, device=DEV)
    g.loss(img, target, mask, loss, d)
    gp = torch.empty(H, 64, device=DEV)
    ga = torch.empty_like(a)
    g.backward(p, v, a, c.t(c.bg), d, 0, gp, ga, flags=binding.HR_GRAD_ALL | binding.HR_REUSE_GEOMETRY)
    torch.cuda.synchronize()
    assert torch.equal(st.image, img)
    assert torch.equal(st.dimage, d)
    assert np.abs(st.loss.cpu().numpy() - loss.cpu().numpy()).max() <= 1e-6 * loss.abs().max().item()
    assert block_rel(st.grad_params.cpu().numpy(), gp.cpu().numpy()) <= 1e-5
    assert block_rel(st.grad_albedo.cpu().numpy(), ga.cpu().numpy()) <= 1e-5


def test_joint_prior_per_hand(mixed):
    c = mixed
    H = c.w.n_hands
    lam, gamma = 5.0, 0.005
    _, j = oracle.skin(c.om, torch.as_tensor(c.params.astype(np.float64)))
    jt = f32(j.numpy() + np.random.default_rng(12).normal(0, 0.008, j.shape))
    img = f32(c.oracle_render(0))
    _, d = oracle.l1_loss(img, _target(c), None, c.tab["pix_off"], c.tab["hand"], H)
    d = f32(d)
    g0 = _gpu_backward(c, d, binding.HR_GRAD_ALL)["gp"]
    c.gsc.set_joint_prior(c.t(jt), lam, gamma)
    try:
        g1 = _gpu_backward(c, d, binding.HR_GRAD_ALL)["gp"]
        st = c.gsc.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), c.t(_target(c)))
        c.gsc.iterate(st, (0.0,) * 6)
        torch.cuda.synchronize()
        l1 = st.loss.cpu().numpy().astype(np.float64)
    finally:
        c.gsc.set_joint_prior(None)
    st = c.gsc.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), c.t(_target(c)))
    c.gsc.iterate(st, (0.0,) * 6)
    torch.cuda.synchronize()
    l0 = st.loss.cpu().numpy().astype(np.float64)
    p = torch.as_tensor(c.params.astype(np.float64)).requires_grad_(True)
    _, jj = oracle.skin(c.om, p)
    e2 = oracle.joint_prior(jj, jt.astype(np.float64), lam, gamma)
    e2.sum().backward()
    og, e2 = p.grad.numpy(), e2.detach().numpy()
    for h in range(H):
        for name, sl in BLOCKS.items():
            check_grad(f"hand {h} prior {name}", (g1 - g0)[h, sl], og[h, sl])
    print("lambda E2 per hand", l1 - l0, e2, flush=True)
    assert np.abs((l1 - l0) - e2).max() <= 1e-5 * np.abs(e2).max() + 1e-6 * np.abs(l0).max()


def test_camera_coverage_per_hand(mixed):
    c = mixed
    _, ghits = c.gpu_render(0, hits=True)
    _, ohits = c.oracle_render(0, hits=True)
    assert np.array_equal(ghits, ohits)
    vis = torch.empty(len(c.cams), c.model.n_faces, dtype=torch.int32, device=DEV)
    c.gsc.face_visibility(torch.as_tensor(ghits).to(DEV), vis)
    order = torch.empty(len(c.cams), dtype=torch.int32, device=DEV)
    covered = torch.empty_like(order)
    c.gsc.camera_order(vis, order, covered)
    torch.cuda.synchronize()
    ovis = oracle.face_visibility(ohits, np.asarray(c.tab["pix_off"]), c.model.n_faces)
    assert np.array_equal(vis.cpu().numpy() != 0, ovis)
    oorder, ocovered = oracle.camera_order(ovis, _hand_views(c))
    print("order", order.cpu().numpy().tolist(), "covered", covered.cpu().numpy().tolist(), flush=True)
    assert order.cpu().numpy().tolist() == oorder.tolist()
    assert covered.cpu().numpy().tolist() == ocovered.tolist()
