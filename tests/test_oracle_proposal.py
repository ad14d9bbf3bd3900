"""Pins of the oracle of the learned edge-sampling proposal.

- bfloat16 rounding against torch's float32 -> bfloat16 conversion;
- erf-GELU and its derivative against torch;
- the unrounded network against a torch.nn model with the same weights;
- the KL gradient against central finite differences of the KL loss;
- the integer proposal weights against their defining properties (equal
  logits reproduce the length weights exactly; totals; floors);
- the boundary estimate with arbitrary positive sampling weights against the
  exact coverage gradient of a flat triangle (unbiasedness), and the
  colour-jump statistics against the triangle's known colour step;
- the edge features of a flat triangle against their closed forms."""
import numpy as np
import torch

import oracle
from oracle import proposal as op
from oracle_geom import identity_camera, pixel_areas, unproject
from test_oracle_edge import H, W, F_, _check, _f32, _project, _scene

rng0 = np.random.default_rng(1234)


def _theta(rng, w3_scale=0.5):
    p = {"W1": rng.normal(0, 0.25, (16, 64)), "b1": rng.normal(0, 0.1, 64),
         "W2": rng.normal(0, 0.125, (64, 64)), "b2": rng.normal(0, 0.1, 64),
         "w3": rng.normal(0, w3_scale, 64), "b3": rng.normal(0, 0.1, 1)}
    return op.flatten({k: v.astype(np.float32) for k, v in p.items()})


def test_bf16_matches_torch():
    x = np.concatenate([rng0.normal(0, 3, 20000), rng0.uniform(-1e-3, 1e-3, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 1.0078125 + 2 ** -9, 3.0e38]])
    # values exactly halfway between bfloat16 neighbours (ties to even)
    base = np.float32(1.0 + 2 ** -7).view(np.uint32)
    ties = np.array([base + 0x8000, base + 0x18000], dtype=np.uint32).view(np.float32)
    x = np.concatenate([x, ties.astype(np.float64)])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(op.bf16(x), ref)


def test_gelu_matches_torch():
    x = np.linspace(-8, 8, 4001)
    t = torch.tensor(x, requires_grad=True)
    y = torch.nn.functional.gelu(t, approximate="none")
    y.sum().backward()
    assert np.allclose(op.gelu(x), y.detach().numpy(), rtol=1e-14, atol=1e-15)
    assert np.allclose(op.gelu_grad(x), t.grad.numpy(), rtol=1e-12, atol=1e-14)


def _torch_mlp(theta):
    p = op.unflatten(theta)
    m = torch.nn.Sequential(torch.nn.Linear(16, 64), torch.nn.GELU(), torch.nn.Linear(64, 64), torch.nn.GELU(),
                            torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        m[0].weight.copy_(torch.tensor(p["W1"].T)); m[0].bias.copy_(torch.tensor(p["b1"]))
        m[2].weight.copy_(torch.tensor(p["W2"].T)); m[2].bias.copy_(torch.tensor(p["b2"]))
        m[4].weight.copy_(torch.tensor(p["w3"][None])); m[4].bias.copy_(torch.tensor(p["b3"]))
    return m


def test_unrounded_forward_matches_torch_model():
    rng = np.random.default_rng(2)
    theta = _theta(rng)
    X = rng.uniform(0, 1, (300, 16))
    z, _ = op.mlp_forward(theta, X, rounded=False)
    ref = _torch_mlp(theta)(torch.tensor(X))[:, 0].detach().numpy()
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_rounded_forward_uses_bf16_values():
    rng = np.random.default_rng(3)
    theta = _theta(rng)
    X = rng.uniform(0, 1, (300, 16))
    z, c = op.mlp_forward(theta, X, rounded=True)
    for k in ("X", "H1", "H2"):
        assert np.array_equal(op.bf16(c[k]), c[k])
    z0, _ = op.mlp_forward(theta, X, rounded=False)
    # bfloat16 keeps 8 significant bits: the logits move by a few parts in 1e3
    assert np.abs(z - z0).max() <= 2e-2 * (1 + np.abs(z0).max())


def test_kl_grad_matches_finite_differences():
    rng = np.random.default_rng(4)
    theta = _theta(rng)
    n = 120
    X = rng.uniform(0, 1, (n, 16))
    w = rng.integers(1, 3000, n).astype(np.uint32)
    w[::9] = 0                                # non-silhouette rows carry no weight
    a = rng.exponential(1.0, n) * (w > 0)
    a[::7] = 0.0                              # edges that saw no signal
    group = np.repeat(np.arange(4), n // 4)
    g = op.kl_grad(theta, X, w, a, group, rounded=False)
    idx = np.concatenate([rng.choice(op.N_PARAMS, 60, replace=False), np.arange(op.N_PARAMS - 65, op.N_PARAMS)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (op.kl_loss(tp, X, w, a, group) - op.kl_loss(tm, X, w, a, group)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])
    # the device's rounding points change the gradient by bfloat16 precision only
    gr = op.kl_grad(theta, X, w, a, group, rounded=True)
    assert np.linalg.norm(gr - g) <= 2e-2 * np.linalg.norm(g)


def test_kl_grad_vanishes_when_proposal_matches_target():
    rng = np.random.default_rng(5)
    theta = _theta(rng)
    X = rng.uniform(0, 1, (50, 16))
    w = rng.integers(1, 500, 50).astype(np.uint32)
    z, _ = op.mlp_forward(theta, X, rounded=False)
    q = w * np.exp(z - z.max())
    g = op.kl_grad(theta, X, w, 3.7 * q / q.sum(), np.zeros(50, int), rounded=False)
    assert np.abs(g).max() <= 1e-12


def test_proposal_weights_properties():
    rng = np.random.default_rng(6)
    w = rng.integers(1, 5000, 400).astype(np.uint32)
    w[::5] = 0
    for zc in (0.0, -3.25, 17.0):
        assert np.array_equal(op.proposal_weights(w, np.full(400, zc)), w)
    z = rng.normal(0, 2, 400)
    Wq = op.proposal_weights(w, z, eps=1e-3)
    live = w > 0
    assert (Wq[~live] == 0).all() and (Wq[live] >= 1).all()
    # total preserved up to the floors
    assert abs(int(Wq.sum()) - int(w.sum())) <= live.sum()
    # every edge keeps the floor eps * w_e
    assert (Wq[live] >= np.floor(1e-3 * w[live])).all()
    # the ratio W/w follows (1 - eps) E/Ebar + eps
    E = np.exp(z[live] - z[live].max())
    ratio = (1 - 1e-3) * E / (np.sum(w[live] * E) / np.sum(w[live])) + 1e-3
    assert (np.abs(Wq[live] - w[live] * ratio) <= 1.0 + 1e-9 * w[live] * ratio).all()
    # ordering: a larger logit never gets a smaller ratio
    order = np.argsort(z[live])
    r = (Wq[live] + 1.0) / w[live]
    assert (np.diff(ratio[order]) >= 0).all()
    assert r[order][-1] >= r[order][0]


def _flat_triangle():
    tri_s = np.array([[2.3, 1.7], [13.6, 4.2], [5.1, 10.4]])
    zs = [1.0, 1.2, 0.9]
    verts = _f32([unproject(x, y, z, W, H, F_) for (x, y), z in zip(tri_s, zs)])
    return verts, _scene(verts, [[0, 1, 2]])


def test_arbitrary_sampling_weights_stay_unbiased():
    verts, sc = _flat_triangle()
    c0, b = _f32([0.9, 0.5, 0.2]), _f32([0.1, 0.2, 0.3])
    g = np.random.default_rng(0).normal(0, 1, (W * H, 3))
    w, _, _, _ = oracle.edge_weights(sc, verts)
    # skewed weights: one edge 20x over-sampled, one under-sampled
    wq = np.maximum(1, (w.astype(np.float64) * np.array([20.0, 0.05, 1.0])[None, :w.shape[1]])).astype(np.uint32)
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    alb = np.tile(c0, (2, 2, 1))
    bg = np.tile(b, (W * H, 1))
    ests = np.array([oracle.backward_edges(sc, verts, normals, alb, bg, g, 500 + s, 0, 1e-3, budget=40000,
                                           wq=wq)[0] for s in range(12)])
    est, se = ests.mean(0), ests.std(0, ddof=1) / np.sqrt(12)
    gw = (g * (c0 - b)).sum(1).reshape(H, W)
    exact = np.zeros_like(verts)
    h = 1e-7
    for i in range(3):
        for k in range(3):
            vp = verts.copy(); vp[i, k] += h
            vm = verts.copy(); vm[i, k] -= h
            Ap = pixel_areas(np.array([_project(x) for x in vp]), W, H)
            Am = pixel_areas(np.array([_project(x) for x in vm]), W, H)
            exact[i, k] = (gw * (Ap - Am)).sum() / (2 * h)
    _check(est, se, exact)


def test_colour_jump_statistics_of_a_flat_triangle():
    verts, sc = _flat_triangle()
    c0, b = _f32([0.9, 0.5, 0.2]), _f32([0.1, 0.7, 0.3])
    g = np.ones((W * H, 3))
    g[:W] = 0.0                               # first image row: no signal, not counted
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    _, stats, dc = oracle.backward_edges(sc, verts, normals, np.tile(c0, (2, 2, 1)), np.tile(b, (W * H, 1)), g,
                                         7, 0, 1e-3, budget=5000, want_stats=True, want_dc=True)
    cnt = dc[0, :, 3]
    assert cnt.sum() > 4000
    live = cnt > 0
    mean = dc[0, live, :3] / cnt[live, None]
    assert np.allclose(mean, np.abs(c0 - b)[None], atol=2e-3)
    # |contribution| sums: each sample adds |g.(c- - c+)| / pdf, whose expectation
    # is the length of the edge inside rows >= 1 times |sum (c0 - b)|
    assert (stats[0][live] > 0).all() and (stats[0][~live] == 0).all()


def test_features_of_a_flat_triangle():
    tri_s = np.array([[2.0, 2.0], [10.0, 3.0], [4.0, 9.0]])
    verts = _f32([unproject(x, y, 1.5, W, H, F_) for x, y in tri_s])
    faces = [[0, 2, 1]]                         # normal towards the camera (-z)
    sc = _scene(verts, faces)
    sc.shading = np.array([0.3, 0.7, 0.0, 0.0, -1.0])
    c0, b = np.array([0.6, 0.4, 0.2]), np.array([0.1, 0.9, 0.5])
    normals = np.tile([0.0, 0.0, -1.0], (3, 1))
    alb = np.tile(c0, (4, 4, 1))
    bg = np.tile(b, (W * H, 1))
    feats = op.edge_features(sc, verts, normals, alb, bg)
    w, _, _, _ = oracle.edge_weights(sc, verts)
    assert (w[0] > 0).all()
    shade = c0 * (0.3 + 0.7 * 1.0)
    diag = np.hypot(W, H)
    for e, (a, bb) in enumerate(sc.edges):
        f = feats[0, e]
        pa, pb = _project(verts[a]), _project(verts[bb])
        got = {tuple(np.round(f[0:2] * [W, H], 4)), tuple(np.round(f[2:4] * [W, H], 4))}
        assert got == {tuple(np.round(pa, 4)), tuple(np.round(pb, 4))}
        assert abs(f[4] - np.linalg.norm(pb - pa) / diag) < 1e-5
        mid = 0.5 * (verts[a] + verts[bb])
        assert abs(f[5] - mid[2] / np.linalg.norm(mid)) < 1e-6 and f[6] == 0.0
        assert np.allclose(f[7:10], np.abs(shade - b), atol=1e-12)
        assert (f[10:] == 0).all()
    ema = np.full((1, len(sc.edges), 3), 0.25)
    valid = np.zeros((1, len(sc.edges)), bool)
    valid[0, 1] = True
    f2 = op.edge_features(sc, verts, normals, alb, bg, ema, valid)
    assert np.allclose(f2[0, 1, 7:10], 0.25) and np.allclose(f2[0, 0, 7:10], feats[0, 0, 7:10])
