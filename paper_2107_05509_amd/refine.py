"""Render-and-compare refinement loop (Section 3.3) on top of the handrt C ABI.

`Refiner` owns the loop buffers (hr_state) of one scene and runs iterations
either call by call (`step_eager`) or as captured HIP graphs of whole
iterations (`run`), with the iteration index kept in device memory so that a
replayed graph draws fresh samples each iteration and needs no host
synchronisation.  The schedule follows the paper's: a first phase in which only
the colour variables move, then all variables.
"""
from __future__ import annotations

import torch

from . import binding

# learning rates (root pose, finger pose, shape, global rotation, translation, colour map)
LR_WARM = (0.0, 0.0, 0.0, 0.0, 0.0, 1e-2)
LR_ALL = (1e-2, 1e-2, 1e-2, 1e-2, 1e-3, 1e-2)


def lr_schedule(it, warm=50):
    """Rates of iteration `it`: colour map only for the first `warm` iterations."""
    return LR_WARM if it < warm else LR_ALL


def coverage_mask(hit_face, cams, pix_off, dilate=9):
    """uint8 [P] mask: pixels any of whose samples hit the hand, dilated by a
    dilate x dilate box (per view)."""
    cover = (hit_face >= 0).any(1).float()
    out = []
    for i, c in enumerate(cams):
        m = cover[int(pix_off[i]):int(pix_off[i + 1])].view(1, 1, c.H, c.W)
        if dilate > 1:
            m = torch.nn.functional.max_pool2d(m, dilate, 1, dilate // 2)
        out.append(m.reshape(-1))
    return (torch.cat(out) > 0).to(torch.uint8).contiguous()


class Refiner:
    """Refinement of `params` [H,64] and `albedo` [H,th,tw,3] (updated in place)
    against `target` images under `mask`."""

    def __init__(self, scene: binding.Scene, params, albedo, background, target, mask=None, warm=50,
                 graph_chunk=10, flags=binding.HR_GRAD_ALL, rebuild_ratio=None):
        """rebuild_ratio: after every `graph_chunk` iterations (a host
        synchronisation), rebuild the hierarchy topology around the current
        pose once a hand's hierarchy cost (hr_hierarchy_cost) exceeds
        rebuild_ratio times its value after the last build; None: never."""
        self.scene = scene
        self.state = scene.make_state(params, albedo, background, target, mask)
        self.warm, self.chunk, self.flags = int(warm), int(graph_chunk), int(flags)
        self.it = 0            # host mirror of state.iter
        self._graphs = {}
        self.rebuild_ratio = rebuild_ratio
        self.rebuilds = 0
        self._cost0 = None     # the costs first seen after the last build

    @property
    def params(self):
        return self.state.params

    @property
    def albedo(self):
        return self.state.albedo

    @property
    def loss(self):
        return self.state.loss

    def build_hierarchy(self):
        """Rebuild the hierarchy topology around the current pose (host work, synchronising)."""
        self.scene.skin(self.state.params, self.state.verts)
        self.scene.build_hierarchy(self.state.verts)
        self._cost0 = None

    def _check_hierarchy(self):
        """With rebuild_ratio: rebuild once a hand's hierarchy has degraded."""
        if self.rebuild_ratio is None:
            return
        cost = self.scene.hierarchy_cost()
        if self._cost0 is None:
            self._cost0 = cost
        elif (cost > self.rebuild_ratio * self._cost0).any():
            self.build_hierarchy()
            self.rebuilds += 1

    def tune(self, reps=3):
        return self.scene.tune(self.state, reps)

    def step_eager(self):
        """One iteration through the separate calls (skin, render, loss, backward, step)."""
        g, q, it = self.scene, self.state, self.it
        g.skin(q.params, q.verts)
        g.render(q.verts, q.albedo, q.background, it, q.image)
        g.loss(q.image, q.target, q.mask, q.loss, q.dimage)
        g.backward(q.params, q.verts, q.albedo, q.background, q.dimage, it, q.grad_params, q.grad_albedo,
                   flags=self.flags | binding.HR_REUSE_GEOMETRY)
        g.step(q.params, q.albedo, q.grad_params, q.grad_albedo, q.m_params, q.v_params, q.m_albedo, q.v_albedo,
               it + 1, lr_schedule(it, self.warm))
        q.iter.fill_(it + 1)
        self.it += 1

    def step(self):
        """One iteration through hr_iterate (device iteration index)."""
        self.scene.iterate(self.state, lr_schedule(self.it, self.warm), self.flags)
        self.it += 1

    def _graph(self, phase, n):
        key = (phase, n)
        if key not in self._graphs:
            lrs = LR_WARM if phase == 0 else LR_ALL
            self._graphs[key] = self.scene.graph(self.state, lrs, n, self.flags)
        return self._graphs[key]

    def _plan(self, n_iters):
        """(phase, length) of the graph launches covering the next n_iters iterations."""
        it, end, out = self.it, self.it + int(n_iters), []
        while it < end:
            phase = 0 if it < self.warm else 1
            stop = min(end, self.warm) if phase == 0 else end
            n = min(self.chunk, stop - it)
            out.append((phase, n))
            it += n
        return out

    def prepare_graphs(self, n_iters):
        """Capture the graphs the next n_iters iterations need (runs nothing)."""
        for phase, n in self._plan(n_iters):
            self._graph(phase, n)

    def run(self, n_iters, graph=True):
        """Enqueue n_iters iterations (graph replays of `graph_chunk` iterations
        where the schedule allows); no host synchronisation unless
        rebuild_ratio is set (then one per `graph_chunk` iterations)."""
        if not graph:
            for _ in range(int(n_iters)):
                self.step()
                if self.rebuild_ratio is not None and self.it % self.chunk == 0:
                    self._check_hierarchy()
            return
        for phase, n in self._plan(n_iters):
            self._graph(phase, n).launch()
            self.it += n
            self._check_hierarchy()


class FullRefiner:
    """Refinement with the paper's full data term (Section 3.1 and Eq. 4):
    per-camera colour transforms T_i, the two-level colour map V = V_high +
    V_low (L x L, nearest-upsampled) and the blurred-Canny edge term beside
    the colour term.  Schedule of Section 3.3: a warm-up of `warm`
    iterations on {T, V_low} only, then every variable.  Each iteration
    enqueues: colour map, skinning, render, full data term (hr_loss_full),
    backward, the low map's gradient, and Adam steps (hr_adam for T, V_low
    and V_high, hr_step for the hand parameters); no host synchronisation.

    T starts at the identity (clamped to [-2, 2]), V_low at `low_init`
    (clamped to [0, 1]), V_high at zero (clamped to [-1, 1])."""

    def __init__(self, scene: binding.Scene, params, background, target, mask=None, L=8, low_init=0.5, warm=50,
                 w_edge=1.0, low=0.02, high=0.04, lr_T=1e-3, lr_low=1e-2, lr_high=1e-2, lr_params=LR_ALL[:5],
                 flags=binding.HR_GRAD_ALL):
        g = self.scene = scene
        dev = params.device
        H, th, tw, V = g.n_hands, g.tex_h, g.tex_w, g.V
        z = lambda *shape: torch.zeros(*shape, device=dev)
        self.params = params
        self.T = torch.eye(3, device=dev).reshape(1, 9).repeat(g.n_views, 1).contiguous()
        self.low = torch.full((H, L, L, 3), float(low_init), device=dev)
        self.high = z(H, th, tw, 3)
        self.albedo = z(H, th, tw, 3)
        self.background, self.target, self.mask = background, target, mask
        self.m = {k: z(*t.shape) for k, t in (("T", self.T), ("low", self.low), ("high", self.high))}
        self.v = {k: z(*t.shape) for k, t in (("T", self.T), ("low", self.low), ("high", self.high))}
        self.mp, self.vp = z(H, 64), z(H, 64)
        self.verts = z(H, V, 3)
        self.image = z(g.P, 3)
        self.dimage = z(g.P, 3)
        self.loss = z(H)
        self.gT = z(g.n_views, 9)
        self.gp = z(H, 64)
        self.galb = z(H, th, tw, 3)
        self.glow = z(H, L, L, 3)
        self.warm, self.flags = int(warm), int(flags)
        self.lr_T, self.lr_low, self.lr_high, self.lr_params = lr_T, lr_low, lr_high, tuple(lr_params)
        self.it = 0
        g.data_term_set(w_edge, low, high)
        # the render traces the edge samples that the reusing backward weighs
        g.set_render_edges(True)
        self.target_edges = z(g.P)
        g.edge_map(target, None, self.target_edges)

    def step(self):
        g, it = self.scene, self.it
        g.compose_albedo(self.low, self.high, self.albedo)
        g.skin(self.params, self.verts)
        g.render(self.verts, self.albedo, self.background, it, self.image)
        g.loss_full(self.image, self.T, self.target, self.target_edges, self.mask, self.loss, self.dimage, self.gT)
        g.backward(self.params, self.verts, self.albedo, self.background, self.dimage, it, self.gp, self.galb,
                   flags=self.flags | binding.HR_REUSE_GEOMETRY)
        g.albedo_low_grad(self.galb, self.glow)
        g.adam(self.T, self.gT, self.m["T"], self.v["T"], it + 1, self.lr_T, -2.0, 2.0)
        g.adam(self.low, self.glow, self.m["low"], self.v["low"], it + 1, self.lr_low, 0.0, 1.0)
        if it >= self.warm:
            t = it - self.warm + 1
            g.adam(self.high, self.galb, self.m["high"], self.v["high"], t, self.lr_high, -1.0, 1.0)
            g.step(self.params, self.albedo, self.gp, self.galb, self.mp, self.vp, self.m["high"], self.v["high"], t,
                   self.lr_params + (0.0,))
        self.it += 1

    def run(self, n):
        for _ in range(int(n)):
            self.step()
