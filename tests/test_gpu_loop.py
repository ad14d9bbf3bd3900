"""The refinement loop entry points: hr_iterate and captured graphs against the
separate calls, launch-grid invariance (the tuner's knob), sample-stream
offsets (view_base) and the batched multi-hand scene against one scene per
hand.  Images must agree bit for bit wherever the samples are the same;
gradients and updated parameters within the atomic-order tolerance (1e-5
relative per block for a few iterations, 1e-3 after ten: Adam's normalised
steps amplify them)."""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import DEV, block_rel, f32
from paper_2107_05509_amd import binding, refine, scene

pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dtype)


class Loop:
    """A tiny workload's loop buffers, fresh for each call."""

    def __init__(self, w, seed=3, spp=None):
        self.w = w
        th, tw = w.albedo_true.shape[1:3]
        self.g = binding.Scene(w.model, w.cams, w.n_hands, spp or w.spp, th, tw, seed=seed)
        self.bg = _t(f32(w.packed_background()))
        img = torch.empty(self.g.P, 3, device=DEV)
        v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
        self.g.skin(_t(f32(w.params_true)), v)
        self.g.render(v, _t(f32(w.albedo_true)), self.bg, 99, img)
        self.target = img
        rng = np.random.default_rng(0)
        self.mask = _t((rng.uniform(size=self.g.P) < 0.9).astype(np.uint8), torch.uint8)

    def refiner(self, warm=2):
        return refine.Refiner(self.g, _t(f32(self.w.params_init)), _t(f32(self.w.albedo_init)), self.bg,
                              self.target, self.mask, warm=warm, graph_chunk=3)


@pytest.fixture(scope="module")
def loop():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: tiny workload, loop entry points", flush=True)
    return Loop(scene.workload_tiny(0))


def _snap(r):
    q = r.state
    torch.cuda.synchronize()
    return {k: getattr(q, k).detach().cpu().numpy().copy() for k in
            ("params", "albedo", "loss", "image", "grad_params", "grad_albedo", "iter")}


def test_iterate_matches_calls(loop):
    # one iteration through hr_iterate and through the five calls, from one
    # saved state, in the colour-only phase and with all variables
    r = loop.refiner()
    for n_before in (0, 3):
        _restore_or_run(r, n_before)
        saved = _save(r)
        outs = []
        for eager in (True, False):
            _restore(r, saved)
            r.step_eager() if eager else r.step()
            outs.append(_snap(r))
        sa, sb = outs
        assert int(sb["iter"][0]) == n_before + 1 == int(sa["iter"][0])
        assert np.array_equal(sa["image"], sb["image"])
        for key in ("params", "albedo", "loss", "grad_params", "grad_albedo"):
            assert block_rel(sb[key], sa[key]) <= 1e-5, (n_before, key, block_rel(sb[key], sa[key]))


def _restore_or_run(r, n):
    """Bring refiner r to iteration n (eager steps)."""
    while r.it < n:
        r.step_eager()
    torch.cuda.synchronize()


_STATE = ("params", "albedo", "m_params", "v_params", "m_albedo", "v_albedo", "iter")


def _save(r):
    torch.cuda.synchronize()
    return {k: getattr(r.state, k).clone() for k in _STATE}, r.it


def _restore(r, saved):
    tensors, it = saved
    for k in _STATE:
        getattr(r.state, k).copy_(tensors[k])
    r.it = it
    torch.cuda.synchronize()


def test_graph_matches_iterate(loop):
    # from one saved state: one iteration as a graph replay and as hr_iterate
    # (tight), then three (loose: Adam's normalised steps amplify the last-bit
    # differences of atomic sums, and a moved silhouette changes single
    # samples, so the last gradient is compared after one iteration only)
    r = loop.refiner()
    r.run(4, graph=False)
    saved = _save(r)
    for n, tol in ((1, 1e-5), (3, 1e-3)):
        outs = []
        for graph in (True, False, True):
            _restore(r, saved)
            r.run(n, graph=graph)
            outs.append(_snap(r))
        g1, it_, g2 = outs
        for sb in outs:
            assert int(sb["iter"][0]) == 4 + n
        for key in ("params", "albedo", "loss") + (("grad_params",) if n == 1 else ()):
            assert block_rel(g1[key], it_[key]) <= tol, (n, key, block_rel(g1[key], it_[key]))
            assert block_rel(g2[key], g1[key]) <= tol, (n, key, block_rel(g2[key], g1[key]))
    # the warm-up graph (colour map only) leaves the pose untouched
    r2 = loop.refiner(warm=5)
    p0 = r2.params.clone()
    r2.run(5, graph=True)
    torch.cuda.synchronize()
    assert torch.equal(r2.params, p0) and int(r2.state.iter.item()) == 5


def test_grid_does_not_change_images(loop):
    # this small scene's tiles are few (all views' tiles at most one per
    # SIMD): grids of two blocks or more render with k_render_few (the waves
    # of a block share each tile, edge packets shrink), a one-block grid with
    # k_render (a wave per tile): the images must agree bit for bit
    g = loop.g
    w = loop.w
    v = torch.empty(1, w.model.n_verts, 3, device=DEV)
    g.skin(_t(f32(w.params_init)), v)
    alb = _t(f32(w.albedo_true))
    d = _t(np.random.default_rng(2).normal(size=(g.P, 3)).astype(np.float32))
    outs = []
    for blocks in ((1, 1), (7, 5), (4096, 4096)):
        g.set_grid(*blocks)
        img = torch.empty(g.P, 3, device=DEV)
        g.render(v, alb, loop.bg, 4, img)
        gp = torch.empty(1, 64, device=DEV)
        ga = torch.empty_like(alb)
        g.backward(_t(f32(w.params_init)), v, alb, loop.bg, d, 4, gp, ga)
        torch.cuda.synchronize()
        outs.append((img.cpu().numpy(), gp.cpu().numpy(), ga.cpu().numpy()))
    r = loop.refiner()
    chosen = r.tune(reps=1)
    print("tuned grids", chosen, flush=True)
    assert all(c >= 1 for c in chosen)
    for img, gp, ga in outs[1:]:
        assert np.array_equal(img, outs[0][0])
        assert block_rel(gp, outs[0][1]) <= 1e-5
        assert block_rel(ga, outs[0][2]) <= 1e-5


def test_view_base_reproduces_streams():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = scene.workload_tiny(1)
    th, tw = w.albedo_true.shape[1:3]
    full = binding.Scene(w.model, w.cams, 1, w.spp, th, tw, seed=11)
    part = binding.Scene(w.model, w.cams[2:], 1, w.spp, th, tw, seed=11, view_base=2)
    v = torch.empty(1, w.model.n_verts, 3, device=DEV)
    full.skin(_t(f32(w.params_init)), v)
    bg = _t(f32(w.packed_background()))
    off = w.pixel_offsets()
    a = torch.empty(full.P, 3, device=DEV)
    b = torch.empty(part.P, 3, device=DEV)
    full.render(v, _t(f32(w.albedo_true)), bg, 5, a)
    part.render(v, _t(f32(w.albedo_true)), bg[off[2]:].contiguous(), 5, b)
    torch.cuda.synchronize()
    assert np.array_equal(a[off[2]:].cpu().numpy(), b.cpu().numpy())


def test_batched_matches_per_hand():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = scene.workload_batched(0, n_hands=3, spp=4)
    print("case: batched 3 hands,", len(w.cams), "views", flush=True)
    th, tw = w.albedo_true.shape[1:3]
    seed = 21
    g = binding.Scene(w.model, w.cams, w.n_hands, w.spp, th, tw, seed=seed)
    off = w.pixel_offsets()
    bg = _t(f32(w.packed_background()))
    p = _t(f32(w.params_init))
    alb = _t(f32(w.albedo_true))
    v = torch.empty(w.n_hands, w.model.n_verts, 3, device=DEV)
    g.skin(p, v)
    img = torch.empty(g.P, 3, device=DEV)
    g.render(v, alb, bg, 2, img)
    d = _t(np.random.default_rng(4).normal(size=(g.P, 3)).astype(np.float32) * 1e-3)
    gp = torch.empty_like(p)
    ga = torch.empty_like(alb)
    g.backward(p, v, alb, bg, d, 2, gp, ga)
    torch.cuda.synchronize()
    hands = np.array([c.hand for c in w.cams])
    for h in range(w.n_hands):
        idx = np.nonzero(hands == h)[0]
        v0, v1 = int(idx[0]), int(idx[-1]) + 1
        assert np.array_equal(idx, np.arange(v0, v1))
        cams = [dataclasses.replace(c, hand=0) for c in w.cams[v0:v1]]
        gh = binding.Scene(w.model, cams, 1, w.spp, th, tw, seed=seed, view_base=v0)
        vh = v[h:h + 1].contiguous()
        ih = torch.empty(gh.P, 3, device=DEV)
        gh.skin(p[h:h + 1].contiguous(), vh)
        gh.render(vh, alb[h:h + 1].contiguous(), bg[off[v0]:off[v1]].contiguous(), 2, ih)
        gph = torch.empty(1, 64, device=DEV)
        gah = torch.empty_like(alb[h:h + 1])
        gh.backward(p[h:h + 1].contiguous(), vh, alb[h:h + 1].contiguous(), bg[off[v0]:off[v1]].contiguous(),
                    d[off[v0]:off[v1]].contiguous(), 2, gph, gah)
        torch.cuda.synchronize()
        assert np.array_equal(ih.cpu().numpy(), img[off[v0]:off[v1]].cpu().numpy()), h
        assert block_rel(gph.cpu().numpy(), gp[h:h + 1].cpu().numpy()) <= 1e-5, h
        assert block_rel(gah.cpu().numpy(), ga[h:h + 1].cpu().numpy()) <= 1e-5, h


def test_stored_hits_match_retrace(loop):
    # the adjoint reuses the render's hits (same geometry and iteration) or
    # re-traces (other iteration, or geometry not declared reused): same gradients
    g, w = loop.g, loop.w
    v = torch.empty(1, w.model.n_verts, 3, device=DEV)
    p = _t(f32(w.params_init))
    g.skin(p, v)
    alb = _t(f32(w.albedo_true))
    d = _t(np.random.default_rng(6).normal(size=(g.P, 3)).astype(np.float32))
    img = torch.empty(g.P, 3, device=DEV)
    outs = {}
    for name, render_it, flags in (("stored", 3, binding.HR_REUSE_GEOMETRY), ("retraced", 3, 0),
                                   ("other iteration", 8, binding.HR_REUSE_GEOMETRY)):
        g.render(v, alb, loop.bg, render_it, img)
        gp = torch.empty(1, 64, device=DEV)
        ga = torch.empty_like(alb)
        g.backward(p, v, alb, loop.bg, d, 3, gp, ga, flags=binding.HR_GRAD_INTERIOR | flags)
        torch.cuda.synchronize()
        outs[name] = (gp.cpu().numpy(), ga.cpu().numpy())
    for name in ("retraced", "other iteration"):
        assert block_rel(outs[name][0], outs["stored"][0]) <= 1e-5, name
        assert block_rel(outs[name][1], outs["stored"][1]) <= 1e-5, name
