"""Refinement with the paper's full data term (colour transforms, two-level
colour map, blurred-Canny edge term; warm-up on {T, V_low}, Section 3.3) on
the HIP path: the warm-up leaves the hand and V_high untouched, every
variable moves afterwards, and the loss falls.  Without the edge term and
with identity transforms hr_loss_full reduces to hr_loss."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, f32
from paper_2107_05509_amd import binding, refine, scene

pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype)


def _setup(w, spp=None):
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, spp or w.spp, th, tw, seed=11)
    bg = _t(f32(w.packed_background()))
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(_t(f32(w.params_true)), v)
    target = torch.empty(g.P, 3, device=DEV)
    g.render(v, _t(f32(w.albedo_true)), bg, 900, target)
    return g, bg, target


def test_full_data_term_without_edges_is_the_colour_term():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, hr_loss_full (w_edge 0, T = I) against hr_loss", flush=True)
    w = scene.workload_tiny(0)
    g, bg, target = _setup(w)
    g.data_term_set(0.0, 0.02, 0.04)
    v = torch.empty(1, w.model.n_verts, 3, device=DEV)
    g.skin(_t(f32(w.params_init)), v)
    img = torch.empty(g.P, 3, device=DEV)
    g.render(v, _t(f32(w.albedo_true)), bg, 0, img)
    mask = _t((np.random.default_rng(1).uniform(size=g.P) < 0.8).astype(np.uint8), torch.uint8)
    edges = torch.empty(g.P, device=DEV)
    g.edge_map(target, None, edges)
    l0, d0 = torch.empty(1, device=DEV), torch.empty(g.P, 3, device=DEV)
    g.loss(img, target, mask, l0, d0)
    l1, d1 = torch.empty(1, device=DEV), torch.empty(g.P, 3, device=DEV)
    g.loss_full(img, None, target, edges, mask, l1, d1)
    torch.cuda.synchronize()
    assert abs(l1.item() - l0.item()) <= 1e-6 * l0.item()
    assert torch.equal(d0, d1)


def test_full_refinement_schedule():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, full data term, warm-up 4 + 16 iterations", flush=True)
    w = scene.workload_tiny(0)
    g, bg, target = _setup(w)
    p0 = _t(f32(w.params_init))
    r = refine.FullRefiner(g, p0.clone(), bg, target, warm=4)
    r.run(1)
    torch.cuda.synchronize()
    loss0 = float(r.loss.sum())
    r.run(3)
    torch.cuda.synchronize()
    assert torch.equal(r.params, p0) and float(r.high.abs().max()) == 0.0
    assert float((r.T - torch.eye(3, device=DEV).reshape(1, 9)).abs().max()) > 0.0
    assert float((r.low - 0.5).abs().max()) > 0.0
    r.run(16)
    torch.cuda.synchronize()
    loss1 = float(r.loss.sum())
    print("loss", loss0, "->", loss1, flush=True)
    assert not torch.equal(r.params, p0) and float(r.high.abs().max()) > 0.0
    assert np.isfinite(loss1) and loss1 < loss0
