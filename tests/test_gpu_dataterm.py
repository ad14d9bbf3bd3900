"""The paper's full data term on the HIP path (Eq. 3 with f1 = D_c + D_e of
Eq. 4, colour transforms T_i, the two-level colour map), through the C ABI,
against the oracle (oracle/data_term.py) on identical float32 inputs: the
rendered images come from the oracle, colour transforms near the identity.
Bars: edge maps 1e-6 relative (float32 outputs of float64 sums), the loss
1e-6 relative per hand, dE/dR element-wise 1e-4 of max(|g|, 1e-3 max|g|),
dE/dT 1e-5 relative per view; the colour map and its low-map gradient 1e-6;
Adam 1e-6 absolute.  The kernels take the Canny selection in float64 with
the oracle's operation order: it must agree pixel for pixel (checked through
the edge maps, which are zero away from selected pixels' blur support)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, Case, check_grad, f32, rel_err
from oracle import data_term as dt
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu

LOW, HIGH = 0.02, 0.04


@pytest.fixture(scope="module", params=["tiny", "mixed"])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"case: {request.param} workload, full data term", flush=True)
    c = Case(scene.workload_tiny(0) if request.param == "tiny" else scene.workload_mixed(0))
    # thresholds below the defaults: the synthetic scenes' luma contrast
    # (a textured hand over per-pixel noise) stays under 0.1 after smoothing
    c.gsc.data_term_set(1.0, LOW, HIGH)
    c.img = f32(c.oracle_render(0))
    rng = np.random.default_rng(3)
    c.T = f32(np.eye(3).reshape(1, 9) + rng.normal(0, 0.03, (len(c.cams), 9)))
    # observed images: the true pose rendered by the oracle
    vt, _ = oracle.skin(c.om, torch.as_tensor(f32(c.w.params_true).astype(np.float64)))
    nt = oracle.vertex_normals(vt, c.om.faces)
    c.O = f32(oracle.render(c.osc, vt.numpy(), nt.numpy(), c.albedo, c.bg, 16, 777, 0))
    c.mask = (rng.uniform(size=c.P) < 0.9).astype(np.uint8)
    return c


def test_edge_map(case):
    c = case
    out = torch.empty(c.P, device=DEV)
    c.gsc.edge_map(c.t(c.img), c.t(c.T), out)
    torch.cuda.synchronize()
    wh, off = c.tab["wh"], c.tab["pix_off"]
    ref = dt.edge_maps(dt.colour_transform(c.img, c.T, off), wh, off, LOW, HIGH)
    g = out.cpu().numpy()
    assert (ref > 1e-3).mean() > 0.05, "too few edges"
    e = rel_err(g, ref, 1e-6 * np.abs(ref).max())
    print("edge map rel err max %.3g" % e.max(), flush=True)
    assert e.max() <= 1e-6


def test_loss_full(case):
    c = case
    wh, off, hands = c.tab["wh"], c.tab["pix_off"], c.tab["hand"]
    H = c.w.n_hands
    Be = f32(dt.edge_maps(c.O, wh, off, LOW, HIGH))
    loss = torch.empty(H, device=DEV)
    d = torch.empty(c.P, 3, device=DEV)
    gT = torch.empty(len(c.cams), 9, device=DEV)
    c.gsc.loss_full(c.t(c.img), c.t(c.T), c.t(c.O), c.t(Be), c.t(c.mask, torch.uint8), loss, d, gT)
    torch.cuda.synchronize()
    lo, gR, gTo, rp, br, sel = dt.data_term(c.img, c.T, c.O, Be, c.mask, wh, off, hands, H, low=LOW, high=HIGH)
    print("selected pixels", int(sel.sum()), "of", c.P, flush=True)
    assert sel.mean() > 0.01
    l = loss.cpu().numpy()
    print("loss", l, lo, flush=True)
    assert np.abs(l - lo).max() <= 1e-6 * np.abs(lo).max()
    check_grad("dE/dR", d.cpu().numpy(), gR)
    g = gT.cpu().numpy()
    for v in range(len(c.cams)):
        assert np.linalg.norm(g[v] - gTo[v]) <= 1e-5 * np.linalg.norm(gTo[v]), v


def test_two_level_colour_map(case):
    c = case
    H, th, tw = c.w.n_hands, c.th, c.tw
    rng = np.random.default_rng(5)
    low = f32(rng.uniform(size=(H, 8, 8, 3)))
    high = f32(rng.normal(0, 0.1, (H, th, tw, 3)))
    out = torch.empty(H, th, tw, 3, device=DEV)
    c.gsc.compose_albedo(c.t(low), c.t(high), out)
    gl = torch.empty(H, 8, 8, 3, device=DEV)
    w = f32(rng.normal(size=(H, th, tw, 3)))
    c.gsc.albedo_low_grad(c.t(w), gl)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - dt.compose_albedo(low, high)).max() <= 1e-6
    ref = dt.albedo_low_grad(w, 8)
    assert np.abs(gl.cpu().numpy() - ref).max() <= 1e-6 * np.abs(ref).max()


def test_adam_clamped(case):
    c = case
    rng = np.random.default_rng(6)
    x0, g = f32(rng.uniform(size=(4, 9))), f32(rng.normal(size=(4, 9)))
    x, m, v = c.t(x0), torch.zeros(4, 9, device=DEV), torch.zeros(4, 9, device=DEV)
    xo, mo, vo = x0.astype(np.float64), np.zeros((4, 9)), np.zeros((4, 9))
    for t in (1, 2, 3):
        c.gsc.adam(x, c.t(g), m, v, t, 0.2, 0.0, 1.0)
        xo, mo, vo = oracle.adam_step(xo, g, mo, vo, t, 0.2, lo=0.0, hi=1.0)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-6
