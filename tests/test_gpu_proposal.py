"""The learned edge-sampling proposal on the GPU against the oracle.

- the network on the matrix cores (bfloat16 operands) against the oracle's
  float64 network at the same rounding points;
- the KL gradient and one Adam step against the oracle's;
- features of the silhouette edges against the oracle's;
- logits given to both sides: integer sampling weights bit-exact, boundary
  gradient and per-edge statistics 1e-4 relative;
- a network with zero output reproduces length-proportional sampling exactly."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, Case, block_rel, f32
from oracle import proposal as op
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu


def _theta(seed, w3_scale=0.5):
    p = scene.mlp_init(seed, out_scale=w3_scale)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = f32(rng.normal(0, 0.1, 64))
    p["b2"] = f32(rng.normal(0, 0.1, 64))
    p["b3"] = f32([0.3])
    return binding.flat_mlp(p)


@pytest.fixture(scope="module")
def tiny():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, proposal", flush=True)
    return Case(scene.workload_tiny(0))


def _dimage(c):
    img = f32(c.oracle_render(0))
    rng = np.random.default_rng(2)
    target = np.clip(img + rng.normal(0, 0.1, img.shape), 0, 1)
    _, d = oracle.l1_loss(img, target, None, c.tab["pix_off"], c.tab["hand"], 1)
    return f32(d)


def test_network_forward_parity(tiny):
    c = tiny
    theta = _theta(1)
    c.gsc.proposal_set(binding.HR_PROPOSAL_LEARNED, theta)
    rng = np.random.default_rng(7)
    X = f32(rng.uniform(0, 1, (3000, 16)))
    X[:, 10:] = 0.0
    z = c.gsc.proposal_eval(c.t(X)).cpu().numpy()
    zo, _ = op.mlp_forward(theta.astype(np.float64), X.astype(np.float64), rounded=True)
    d = np.abs(z - zo)
    print("logit |diff|: max %.3g, p99 %.3g, median %.3g, |z| max %.3g"
          % (d.max(), np.quantile(d, 0.99), np.median(d), np.abs(zo).max()), flush=True)
    # float32 against float64 accumulation; a hidden value that rounds to the
    # other bfloat16 neighbour moves a logit by ~2^-8 of one term
    assert np.median(d) <= 1e-5 * (1 + np.abs(zo).max())
    assert np.quantile(d, 0.99) <= 1e-5 * (1 + np.abs(zo).max())
    assert d.max() <= 2e-2 * (1 + np.abs(zo).max())


def test_network_gradient_and_step_parity(tiny):
    c = tiny
    theta = _theta(2)
    lr = 1e-3
    c.gsc.proposal_set(binding.HR_PROPOSAL_LEARNED, theta, lr=lr)
    rng = np.random.default_rng(8)
    n = 2000
    X = f32(rng.uniform(0, 1, (n, 16)))
    X[:, 10:] = 0.0
    w = rng.integers(1, 4000, n).astype(np.uint32)
    w[::11] = 0
    a = f32(rng.exponential(1.0, n) * (w > 0))
    g = c.gsc.proposal_fit(c.t(X), c.t(w.astype(np.int32), torch.int32), c.t(a), apply=True).cpu().numpy()
    go = op.kl_grad(theta.astype(np.float64), X.astype(np.float64), w, a.astype(np.float64), np.zeros(n, int))
    e = block_rel(g, go)
    print("KL gradient block rel %.3g" % e, flush=True)
    assert e <= 1e-4
    th1 = c.gsc.proposal_get()
    to, _, _ = oracle.adam_step(theta.astype(np.float64), go, np.zeros(op.N_PARAMS), np.zeros(op.N_PARAMS), 1, lr)
    # the first Adam step moves each parameter by lr sign(g); compare where the
    # sign is not in doubt
    firm = np.abs(go) > 1e-2 * np.abs(go).max()
    assert firm.sum() > 1000
    assert np.abs(th1[firm] - to[firm]).max() <= 1e-6


def _edge_case_grads(c, d, theta=None, z=None, kind=binding.HR_PROPOSAL_LEARNED):
    c.gsc.proposal_set(kind, theta if theta is not None else binding.flat_mlp(scene.mlp_init(0)), lr=0.0)
    c.gsc.proposal_override(z)
    gp = torch.empty(1, 64, device=DEV)
    ga = torch.empty(1, c.th, c.tw, 3, device=DEV)
    gv = torch.empty(1, c.model.n_verts, 3, device=DEV)
    c.gsc.backward(c.t(c.params), c.t(c.v32), c.t(c.albedo), c.t(c.bg), c.t(d), 0, gp, ga, gv, None,
                   binding.HR_GRAD_EDGES)
    zz, wq, a, dc = c.gsc.proposal_stats()
    torch.cuda.synchronize()
    out = dict(gv=gv.cpu().numpy(), wq=wq.cpu().numpy().astype(np.uint32), a=a.cpu().numpy(), dc=dc.cpu().numpy(),
               z=zz.cpu().numpy())
    c.gsc.proposal_override(None)
    return out


def test_zero_output_reproduces_length_sampling(tiny):
    c = tiny
    d = _dimage(c)
    learned = _edge_case_grads(c, d)                       # w3 = 0: every logit 0
    length = _edge_case_grads(c, d, kind=binding.HR_PROPOSAL_LENGTH)
    w, _, _, _ = oracle.edge_weights(c.osc, c.v32.astype(np.float64))
    assert np.array_equal(learned["wq"], w)
    assert np.array_equal(length["wq"], w)
    assert (learned["z"][w > 0] == 0).all()
    assert block_rel(learned["gv"], length["gv"]) <= 1e-6


def test_given_logits_parity(tiny):
    c = tiny
    d = _dimage(c)
    E = c.model.n_edges
    z = f32(np.random.default_rng(9).normal(0, 1.5, (len(c.cams), E)))
    g = _edge_case_grads(c, d, z=c.t(z))
    v64 = c.v32.astype(np.float64)
    w, _, _, bud = oracle.edge_weights(c.osc, v64)
    wq = np.stack([op.proposal_weights(w[v], z[v].astype(np.float64)) for v in range(len(c.cams))])
    assert np.array_equal(g["wq"], wq), f"{(g['wq'] != wq).sum()} weights differ"
    assert (wq != w).sum() > 0.5 * (w > 0).sum()
    gv, st, dc = oracle.backward_edges(c.osc, v64, c.n64, c.albedo, c.bg, d, c.seed, 0, 1e-3, want_stats=True,
                                       wq=wq, want_dc=True)
    e = block_rel(g["gv"], gv)
    print("edge gradient with given logits: block rel %.3g" % e, flush=True)
    assert e <= 1e-4
    assert block_rel(g["a"], st) <= 1e-4
    assert np.array_equal(g["dc"][..., 3], dc[..., 3])
    assert block_rel(g["dc"][..., :3], dc[..., :3]) <= 1e-5


def test_feature_parity(tiny):
    c = tiny
    d = _dimage(c)
    _edge_case_grads(c, d, theta=_theta(3))
    f = c.gsc.proposal_features().cpu().numpy()
    fo = op.edge_features(c.osc, c.v32.astype(np.float64), c.n64, c.albedo, c.bg)
    fob = op.bf16(fo)
    w, _, _, _ = oracle.edge_weights(c.osc, c.v32.astype(np.float64))
    assert (f[w == 0] == 0).all()
    live = w > 0
    # equal, or one bfloat16 step apart where float32 and float64 straddle a rounding boundary
    diff = np.abs(f[live] - fob[live])
    ulp = np.maximum(np.abs(fob[live]), 1e-30) * 2.0 ** -7
    print("features: %d of %d differ by <= 1 bfloat16 step" % ((diff > 0).sum(), diff.size), flush=True)
    assert (diff <= ulp + 1e-30).all()
    assert (diff > 0).mean() < 0.01


def _loop_scene(w, seed=4):
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=seed)
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(DEV, torch.float32)
    bg = t(f32(w.packed_background()))
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(t(f32(w.params_true)), v)
    target = torch.empty(g.P, 3, device=DEV)
    g.render(v, t(f32(w.albedo_true)), bg, 77, target)
    return g, t(f32(w.params_init)), t(f32(w.albedo_init)), bg, target


def test_training_inside_captured_iterations():
    """hr_iterate with the learned proposal (its passes on the side stream) as
    a captured graph and as eager calls: the first iteration's loss and
    gradient agree (atomic-order tolerance); over several iterations the
    network trains and the loss falls.  (Parameter trajectories are not
    compared: Adam turns last-bit gradient differences of near-zero components
    into steps of a learning rate.)"""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2107_05509_amd import refine
    w = scene.workload_tiny(0)
    first = []
    for graph in (False, True):
        g, p, a, bg, target = _loop_scene(w)
        g.proposal_set(binding.HR_PROPOSAL_LEARNED, scene.mlp_init(5), lr=1e-2)
        r = refine.Refiner(g, p, a, bg, target, None, warm=0, graph_chunk=3)
        r.run(1, graph=graph)
        torch.cuda.synchronize()
        first.append((float(r.loss.item()), r.state.grad_params.cpu().numpy().copy()))
        l0 = first[-1][0]
        r.run(8, graph=graph)
        torch.cuda.synchronize()
        th = g.proposal_get()
        assert int(r.state.iter.item()) == 9
        assert np.abs(th - binding.flat_mlp(scene.mlp_init(5))).max() > 1e-3   # the network trained
        assert np.isfinite(r.params.cpu().numpy()).all() and float(r.loss.item()) < l0
    (la, ga), (lb, gb) = first
    assert abs(la - lb) <= 1e-6 * abs(la)
    assert block_rel(gb, ga) <= 1e-5


def _trained_spread(eps, n_keys):
    """Boundary-term gradients (61 free parameters) over n_keys sample keys at
    equal edge-sample budget, length-proportional and learned (trained for 150
    iterations on a fixed pose) with the given floor.  The loss mask keeps the
    left half of every image, so silhouette edges on the right contribute
    nothing and a good proposal learns to leave them out (the features
    include the edges' screen positions)."""
    w = scene.workload_realistic(0, n_views=2)
    res = {}
    for kind in (binding.HR_PROPOSAL_LENGTH, binding.HR_PROPOSAL_LEARNED):
        g, p, a, bg, target = _loop_scene(w, seed=6)
        mask = torch.zeros(g.P, dtype=torch.uint8, device=DEV)
        off = w.pixel_offsets()
        for i, c in enumerate(w.cams):
            mask[int(off[i]):int(off[i + 1])].view(c.H, c.W)[:, : c.W // 2] = 1
        v = torch.empty(1, w.model.n_verts, 3, device=DEV)
        img = torch.empty(g.P, 3, device=DEV)
        g.skin(p, v)
        g.build_hierarchy(v)
        g.render(v, a, bg, 0, img)
        loss = torch.empty(1, device=DEV)
        d = torch.empty(g.P, 3, device=DEV)
        g.loss(img, target, mask, loss, d)
        gp = torch.empty(1, 64, device=DEV)
        ga = torch.empty_like(a)
        g.proposal_set(kind, scene.mlp_init(1), lr=1e-2, eps=eps)
        if kind == binding.HR_PROPOSAL_LEARNED:
            for it in range(150):
                g.backward(p, v, a, bg, d, 1000 + it, gp, ga, flags=binding.HR_GRAD_EDGES)
                g.proposal_train()
        rows = torch.empty(n_keys, 64, dtype=torch.float64, device=DEV)
        for s in range(n_keys):
            g.backward(p, v, a, bg, d, 5000 + s, gp, ga, flags=binding.HR_GRAD_EDGES)
            rows[s] = gp[0].double()
        res[kind] = rows.cpu().numpy()[:, 3:]
    return res[binding.HR_PROPOSAL_LENGTH], res[binding.HR_PROPOSAL_LEARNED]


def test_trained_proposal_is_unbiased():
    """At the proposal's default floor (eps = 1e-3 of the length-proportional
    weights) the learned and the length-proportional estimates must agree in
    the mean over 1024 sample keys, within 4.5 standard errors per parameter.
    (Their spreads are not compared here: an edge the network suppresses keeps
    1e-3 of its length share, so its rare samples carry up to 1000 times the
    weight and the sample variance over 1024 keys swings between runs.)"""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: realistic workload, 2 views, left-half mask, learned proposal, floor 1e-3", flush=True)
    L, Q = _trained_spread(1e-3, 1024)
    se = np.sqrt(L.var(0, ddof=1) / len(L) + Q.var(0, ddof=1) / len(Q)) + 1e-30
    z = np.abs(L.mean(0) - Q.mean(0)) / se
    print("max |z| %.2f over %d parameters" % (z.max(), z.size), flush=True)
    assert z.max() <= 4.5


def test_trained_proposal_reduces_variance():
    """With a floor of 0.05 (importance weights below 20, so 256 keys
    estimate the spread reliably) the learned proposal is unbiased (4.5
    standard errors) and its boundary gradient has the smaller spread (trace
    of the covariance over the 61 free parameters)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: realistic workload, 2 views, left-half mask, learned proposal, floor 0.05", flush=True)
    L, Q = _trained_spread(0.05, 256)
    se = np.sqrt(L.var(0, ddof=1) / len(L) + Q.var(0, ddof=1) / len(Q)) + 1e-30
    z = np.abs(L.mean(0) - Q.mean(0)) / se
    ratio = np.trace(np.cov(L.T)) / np.trace(np.cov(Q.T))
    print("max |z| %.2f over %d parameters; variance ratio length/learned %.3f" % (z.max(), z.size, ratio),
          flush=True)
    assert z.max() <= 4.5
    assert ratio > 1.2
