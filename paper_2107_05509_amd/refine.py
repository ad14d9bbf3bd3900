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
                 graph_chunk=10, flags=binding.HR_GRAD_ALL):
        self.scene = scene
        self.state = scene.make_state(params, albedo, background, target, mask)
        self.warm, self.chunk, self.flags = int(warm), int(graph_chunk), int(flags)
        self.it = 0            # host mirror of state.iter
        self._graphs = {}

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
        where the schedule allows); no host synchronisation."""
        if not graph:
            for _ in range(int(n_iters)):
                self.step()
            return
        for phase, n in self._plan(n_iters):
            self._graph(phase, n).launch()
            self.it += n
