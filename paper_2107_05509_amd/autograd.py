"""torch.autograd integration of the handrt C ABI.

`render_images` is differentiable with respect to the hand parameters and the
colour map: its backward hands the incoming image gradient to hr_backward,
which re-traces the forward's samples from their counters (nothing per sample
is stored) and adds the silhouette-edge term.  `photometric_loss` fuses render
and the L1 data term (Eq. 3 with D_c of Eq. 4) and returns the per-hand loss.
Both differentiate exactly what they return: a joint prior set on the scene
(part of hr_iterate's objective) stays out of their gradients.
"""
from __future__ import annotations

import torch

from . import binding


def _pixel_hand(scene: binding.Scene, cams, device):
    """[P] index of the hand each packed pixel belongs to."""
    idx = torch.empty(scene.P, dtype=torch.long, device=device)
    off = scene.pix_off
    for v, c in enumerate(cams):
        idx[int(off[v]):int(off[v + 1])] = int(c.hand)
    return idx


class _RenderImages(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, albedo, scene, background, it):
        verts = torch.empty(scene.n_hands, scene.V, 3, device=params.device)
        scene.skin(params, verts)
        image = torch.empty(scene.P, 3, device=params.device)
        scene.render(verts, albedo, background, it, image)
        ctx.scene, ctx.it = scene, int(it)
        ctx.save_for_backward(params, albedo, background)
        return image

    @staticmethod
    def backward(ctx, grad_image):
        params, albedo, background = ctx.saved_tensors
        scene = ctx.scene
        verts = torch.empty(scene.n_hands, scene.V, 3, device=params.device)
        scene.skin(params, verts)   # recomputed; hr_backward re-prepares the geometry
        gp = torch.empty_like(params)
        ga = torch.empty_like(albedo)
        scene.backward(params, verts, albedo, background, grad_image.contiguous(), ctx.it, gp, ga,
                       flags=binding.HR_GRAD_ALL | binding.HR_SKIP_PRIOR)
        return gp, ga, None, None, None


def render_images(scene: binding.Scene, params, albedo, background, it=0):
    """Images [P,3] of all views; differentiable in params [H,64] and albedo [H,th,tw,3]."""
    return _RenderImages.apply(params.contiguous(), albedo.contiguous(), scene, background.contiguous(), it)


class _PhotometricLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, albedo, scene, background, target, mask, pixel_hand, it):
        dev = params.device
        verts = torch.empty(scene.n_hands, scene.V, 3, device=dev)
        scene.skin(params, verts)
        image = torch.empty(scene.P, 3, device=dev)
        scene.render(verts, albedo, background, it, image)
        loss = torch.empty(scene.n_hands, device=dev)
        dimage = torch.empty(scene.P, 3, device=dev)
        scene.loss(image, target, mask, loss, dimage)
        ctx.scene, ctx.it = scene, int(it)
        ctx.save_for_backward(params, albedo, background, dimage, pixel_hand)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        params, albedo, background, dimage, pixel_hand = ctx.saved_tensors
        scene = ctx.scene
        verts = torch.empty(scene.n_hands, scene.V, 3, device=params.device)
        scene.skin(params, verts)
        d = (dimage * grad_loss[pixel_hand][:, None]).contiguous()
        gp = torch.empty_like(params)
        ga = torch.empty_like(albedo)
        scene.backward(params, verts, albedo, background, d, ctx.it, gp, ga,
                       flags=binding.HR_GRAD_ALL | binding.HR_SKIP_PRIOR)
        return gp, ga, None, None, None, None, None, None


def photometric_loss(scene: binding.Scene, cams, params, albedo, background, target, mask=None, it=0,
                     pixel_hand=None):
    """Per-hand E1 [H]; differentiable in params and albedo."""
    if pixel_hand is None:
        pixel_hand = _pixel_hand(scene, cams, params.device)
    return _PhotometricLoss.apply(params.contiguous(), albedo.contiguous(), scene, background.contiguous(),
                                  target.contiguous(), mask, pixel_hand, it)
