"""Thin ctypes binding of the handrt C ABI (include/handrt.h).

Argument marshalling only: every step runs in the HIP kernels of libhandrt.so.
Tensors are torch CUDA tensors (float32 unless stated, contiguous); work is
enqueued on torch's current stream.  If the library is not built, importing
this module works but any call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhandrt.so")

HR_GRAD_INTERIOR = 1
HR_GRAD_EDGES = 2
HR_GRAD_ALL = 3
HR_REUSE_GEOMETRY = 4
HR_SKIP_PRIOR = 8
HR_ACCEL_AUTO = 0
HR_ACCEL_HIERARCHY = 1

EXPORTS = ("hr_scene_create", "hr_scene_destroy", "hr_num_pixels", "hr_skin", "hr_build_hierarchy",
           "hr_hierarchy_cost", "hr_render",
           "hr_loss", "hr_loss_noalloc", "hr_backward", "hr_set_joint_prior", "hr_face_visibility", "hr_camera_order", "hr_step", "hr_iterate", "hr_graph_create", "hr_graph_launch",
           "hr_graph_destroy", "hr_set_grid", "hr_set_accel", "hr_set_tiles", "hr_get_tiles", "hr_set_renderer", "hr_set_edge_budget", "hr_set_render_edges", "hr_get_grid", "hr_tune", "hr_edge_stats", "hr_set_counting", "hr_read_counts",
           "hr_timing_enable", "hr_timing_read", "hr_proposal_set", "hr_proposal_get", "hr_proposal_override",
           "hr_proposal_train", "hr_proposal_features", "hr_proposal_stats", "hr_proposal_eval", "hr_proposal_fit",
           "hr_data_term_set", "hr_edge_map", "hr_loss_full", "hr_compose_albedo", "hr_albedo_low_grad", "hr_adam",
           "hr_last_error")

HR_RENDERER_RAY = 0
HR_RENDERER_RASTER = 1
HR_PROPOSAL_LENGTH = 0
HR_PROPOSAL_LEARNED = 1
HR_MLP_PARAMS = 5313
MLP_LAYOUT = (("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("w3", (64,)), ("b3", (1,)))


class HRError(RuntimeError):
    pass


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_verts", ctypes.c_int32), ("n_faces", ctypes.c_int32), ("n_joints", ctypes.c_int32),
                ("n_shape", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("v_template", ctypes.c_void_p), ("shapedirs", ctypes.c_void_p),
                ("j_regressor", ctypes.c_void_p), ("weights", ctypes.c_void_p), ("parents", ctypes.c_void_p),
                ("faces", ctypes.c_void_p), ("uv", ctypes.c_void_p), ("edges", ctypes.c_void_p),
                ("edge_faces", ctypes.c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_float * 9), ("o", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("W", ctypes.c_int32), ("H", ctypes.c_int32), ("hand", ctypes.c_int32)]


class Config(ctypes.Structure):
    _fields_ = [("ka", ctypes.c_float), ("kd", ctypes.c_float), ("light", ctypes.c_float * 3),
                ("spp", ctypes.c_int32), ("edge_delta", ctypes.c_float), ("tex_h", ctypes.c_int32),
                ("tex_w", ctypes.c_int32), ("seed", ctypes.c_uint64), ("view_base", ctypes.c_uint32)]


class AdamConfig(ctypes.Structure):
    _fields_ = [("lr_pose_root", ctypes.c_float), ("lr_pose", ctypes.c_float), ("lr_shape", ctypes.c_float),
                ("lr_rot", ctypes.c_float), ("lr_trans", ctypes.c_float), ("lr_albedo", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class ProposalConfig(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("eps", ctypes.c_float), ("ema", ctypes.c_float), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float)]


class DataTerm(ctypes.Structure):
    _fields_ = [("w_edge", ctypes.c_float), ("low", ctypes.c_float), ("high", ctypes.c_float)]


class State(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "params", "albedo", "m_params", "v_params", "m_albedo", "v_albedo", "background", "target", "mask", "verts",
        "image", "dimage", "loss", "grad_params", "grad_albedo", "iter")]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HRError(f"handrt library not built: {LIB_PATH} is missing "
                          "(run `python -c 'import __graft_entry__ as g; g.build()'`)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
        L.hr_scene_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(MeshDesc), i32, ctypes.POINTER(Camera),
                                      i32, ctypes.POINTER(Config)]
        L.hr_scene_destroy.argtypes = [vp]
        L.hr_scene_destroy.restype = None
        L.hr_num_pixels.argtypes = [vp]
        L.hr_num_pixels.restype = ctypes.c_int64
        L.hr_skin.argtypes = [vp, vp, vp, vp, vp]
        L.hr_render.argtypes = [vp, vp, vp, vp, u32, vp, vp, vp]
        L.hr_loss.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.hr_loss_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.hr_backward.argtypes = [vp, vp, vp, vp, vp, vp, u32, u32, vp, vp, vp, vp, vp]
        L.hr_set_joint_prior.argtypes = [vp, vp, ctypes.c_float, ctypes.c_float]
        L.hr_face_visibility.argtypes = [vp, vp, vp, vp]
        L.hr_camera_order.argtypes = [vp, vp, vp, vp, vp]
        L.hr_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, ctypes.POINTER(AdamConfig), vp]
        L.hr_iterate.argtypes = [vp, ctypes.POINTER(State), ctypes.POINTER(AdamConfig), u32, vp]
        L.hr_graph_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(State), ctypes.POINTER(AdamConfig), u32,
                                      i32]
        L.hr_graph_launch.argtypes = [vp, vp]
        L.hr_graph_destroy.argtypes = [vp]
        L.hr_graph_destroy.restype = None
        L.hr_set_grid.argtypes = [vp, i32, i32]
        L.hr_set_accel.argtypes = [vp, i32]
        L.hr_get_grid.argtypes = [vp, vp]
        L.hr_tune.argtypes = [vp, ctypes.POINTER(State), i32, vp, vp]
        L.hr_proposal_set.argtypes = [vp, ctypes.POINTER(ProposalConfig), vp]
        L.hr_proposal_get.argtypes = [vp, vp, vp]
        L.hr_proposal_override.argtypes = [vp, vp]
        L.hr_proposal_train.argtypes = [vp, vp]
        L.hr_proposal_features.argtypes = [vp, vp, vp]
        L.hr_proposal_stats.argtypes = [vp, vp, vp, vp, vp, vp]
        L.hr_proposal_eval.argtypes = [vp, vp, i32, vp, vp]
        L.hr_proposal_fit.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp]
        L.hr_edge_stats.argtypes = [vp, vp, vp, vp]
        L.hr_build_hierarchy.argtypes = [vp, vp, vp]
        L.hr_hierarchy_cost.argtypes = [vp, vp]
        L.hr_set_counting.argtypes = [vp, i32]
        L.hr_read_counts.argtypes = [vp, vp, vp]
        L.hr_timing_enable.argtypes = [vp, i32]
        L.hr_timing_read.argtypes = [vp, vp, vp, vp, i32, vp, vp]
        L.hr_data_term_set.argtypes = [vp, ctypes.POINTER(DataTerm)]
        L.hr_edge_map.argtypes = [vp, vp, vp, vp, vp]
        L.hr_loss_full.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.hr_compose_albedo.argtypes = [vp, vp, i32, vp, vp, vp]
        L.hr_albedo_low_grad.argtypes = [vp, vp, i32, vp, vp]
        L.hr_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int64, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                              ctypes.POINTER(AdamConfig), vp]
        L.hr_last_error.restype = ctypes.c_char_p
        for name in ("hr_scene_create", "hr_skin", "hr_render", "hr_loss", "hr_loss_noalloc", "hr_backward", "hr_set_joint_prior",
                     "hr_face_visibility", "hr_camera_order",
                     "hr_step", "hr_iterate",
                     "hr_graph_create", "hr_graph_launch", "hr_set_grid", "hr_set_accel", "hr_set_tiles", "hr_get_tiles",
                     "hr_set_renderer", "hr_set_edge_budget", "hr_set_render_edges", "hr_get_grid", "hr_tune", "hr_edge_stats",
                     "hr_build_hierarchy", "hr_hierarchy_cost", "hr_set_counting", "hr_read_counts", "hr_timing_enable", "hr_timing_read",
                     "hr_proposal_set", "hr_proposal_get", "hr_proposal_override", "hr_proposal_train",
                     "hr_proposal_features", "hr_proposal_stats", "hr_proposal_eval", "hr_proposal_fit",
                     "hr_data_term_set", "hr_edge_map", "hr_loss_full", "hr_compose_albedo", "hr_albedo_low_grad",
                     "hr_adam"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        msg = lib().hr_last_error().decode()
        raise HRError(f"{what} failed ({rc}): {msg}")


def _ptr(t, dtype=torch.float32, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HRError(f"{name}: expected a CUDA tensor")
    if t.dtype != dtype:
        raise HRError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise HRError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise HRError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Scene:
    """A handrt scene: hand model + cameras + estimator configuration."""

    def __init__(self, model, cams, n_hands, spp, tex_h, tex_w, seed=0, shading=None, edge_delta=1e-3, view_base=0):
        from . import scene as _scene
        shading = _scene.SHADING if shading is None else shading
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a.ctypes.data_as(ctypes.c_void_p)

        md = MeshDesc()
        md.n_verts, md.n_faces = model.n_verts, model.n_faces
        md.n_joints, md.n_shape, md.n_edges = model.j_regressor.shape[0], model.shapedirs.shape[2], model.n_edges
        md.v_template = arr(model.v_template, np.float32)
        md.shapedirs = arr(model.shapedirs, np.float32)
        md.j_regressor = arr(model.j_regressor, np.float32)
        md.weights = arr(model.weights, np.float32)
        md.parents = arr(model.parents, np.int32)
        md.faces = arr(model.faces, np.int32)
        md.uv = arr(model.uv, np.float32)
        md.edges = arr(model.edges, np.int32)
        md.edge_faces = arr(model.edge_faces, np.int32)
        cam_arr = (Camera * len(cams))()
        tables = _scene.camera_arrays(cams)
        for i, c in enumerate(cams):
            cam_arr[i].R[:] = [float(x) for x in tables["R"][i]]
            cam_arr[i].o[:] = [float(x) for x in tables["o"][i]]
            cam_arr[i].fx, cam_arr[i].fy, cam_arr[i].cx, cam_arr[i].cy = [float(x) for x in tables["intr"][i]]
            cam_arr[i].W, cam_arr[i].H = int(c.W), int(c.H)
            cam_arr[i].hand = int(c.hand)
        cfg = Config()
        cfg.ka, cfg.kd = float(shading[0]), float(shading[1])
        cfg.light[:] = [float(x) for x in shading[2:5]]
        cfg.spp, cfg.edge_delta = int(spp), float(edge_delta)
        cfg.tex_h, cfg.tex_w, cfg.seed = int(tex_h), int(tex_w), int(seed)
        cfg.view_base = int(view_base)
        h = ctypes.c_void_p()
        _check(lib().hr_scene_create(ctypes.byref(h), ctypes.byref(md), int(n_hands), cam_arr, len(cams),
                                     ctypes.byref(cfg)), "hr_scene_create")
        self._h = h
        self._keep = []
        self.n_hands, self.n_views = int(n_hands), len(cams)
        self.V, self.F, self.J = model.n_verts, model.n_faces, model.j_regressor.shape[0]
        self.spp, self.tex_h, self.tex_w = int(spp), int(tex_h), int(tex_w)
        self.P = int(lib().hr_num_pixels(h))
        self._n_edges = int(model.n_edges)
        self.pix_off = tables["pix_off"]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hr_scene_destroy(h)
            self._h = None

    # -- calls ---------------------------------------------------------------
    def skin(self, params, verts, joints=None):
        _check(lib().hr_skin(self._h, _ptr(params, shape=(self.n_hands, 64), name="params"),
                             _ptr(verts, shape=(self.n_hands, self.V, 3), name="verts"),
                             _ptr(joints, shape=(self.n_hands, self.J, 3), name="joints"), _stream()), "hr_skin")

    def build_hierarchy(self, verts):
        _check(lib().hr_build_hierarchy(self._h, _ptr(verts, shape=(self.n_hands, self.V, 3), name="verts"),
                                        _stream()), "hr_build_hierarchy")

    def hierarchy_cost(self):
        """Each hand's hierarchy cost as last refit (numpy float32 [n_hands];
        synchronises the device)."""
        out = np.zeros(self.n_hands, np.float32)
        _check(lib().hr_hierarchy_cost(self._h, out.ctypes.data_as(ctypes.c_void_p)), "hr_hierarchy_cost")
        return out

    def render(self, verts, albedo, background, it, image, hit_face=None):
        _check(lib().hr_render(self._h, _ptr(verts, shape=(self.n_hands, self.V, 3), name="verts"),
                               _ptr(albedo, shape=(self.n_hands, self.tex_h, self.tex_w, 3), name="albedo"),
                               _ptr(background, shape=(self.P, 3), name="background"), int(it),
                               _ptr(image, shape=(self.P, 3), name="image"),
                               _ptr(hit_face, torch.int32, (self.P, self.spp), "hit_face"), _stream()), "hr_render")

    def loss(self, image, target, mask, loss, dimage):
        _check(lib().hr_loss(self._h, _ptr(image, shape=(self.P, 3), name="image"),
                             _ptr(target, shape=(self.P, 3), name="target"),
                             _ptr(mask, torch.uint8, (self.P,), "mask"),
                             _ptr(loss, shape=(self.n_hands,), name="loss"),
                             _ptr(dimage, shape=(self.P, 3), name="dimage"), _stream()), "hr_loss")

    def loss_noalloc(self, image, target, mask, loss, dimage):
        """hr_loss with its scratch in the library's fixed array (allocates nothing)."""
        _check(lib().hr_loss_noalloc(self._h, _ptr(image, shape=(self.P, 3), name="image"),
                                     _ptr(target, shape=(self.P, 3), name="target"),
                                     _ptr(mask, torch.uint8, (self.P,), "mask"),
                                     _ptr(loss, shape=(self.n_hands,), name="loss"),
                                     _ptr(dimage, shape=(self.P, 3), name="dimage"), _stream()), "hr_loss_noalloc")

    def backward(self, params, verts, albedo, background, dimage, it, grad_params, grad_albedo,
                 grad_verts=None, grad_normals=None, flags=HR_GRAD_ALL):
        _check(lib().hr_backward(
            self._h, _ptr(params, shape=(self.n_hands, 64), name="params"),
            _ptr(verts, shape=(self.n_hands, self.V, 3), name="verts"),
            _ptr(albedo, shape=(self.n_hands, self.tex_h, self.tex_w, 3), name="albedo"),
            _ptr(background, shape=(self.P, 3), name="background"), _ptr(dimage, shape=(self.P, 3), name="dimage"),
            int(it), int(flags), _ptr(grad_params, shape=(self.n_hands, 64), name="grad_params"),
            _ptr(grad_albedo, shape=(self.n_hands, self.tex_h, self.tex_w, 3), name="grad_albedo"),
            _ptr(grad_verts, shape=(self.n_hands, self.V, 3), name="grad_verts"),
            _ptr(grad_normals, shape=(self.n_hands, self.V, 3), name="grad_normals"), _stream()), "hr_backward")

    def face_visibility(self, hit_face, visible):
        """visible [n_views,F] int32 <- faces hit by each view's samples (hit_face [P,spp])."""
        _check(lib().hr_face_visibility(self._h, _ptr(hit_face, torch.int32, (self.P, self.spp), "hit_face"),
                                        _ptr(visible, torch.int32, (self.n_views, self.F), "visible"), _stream()),
               "hr_face_visibility")

    def camera_order(self, visible, order, covered):
        """Greedy coverage order of each hand's views (order, covered: [n_views] int32)."""
        _check(lib().hr_camera_order(self._h, _ptr(visible, torch.int32, (self.n_views, self.F), "visible"),
                                     _ptr(order, torch.int32, (self.n_views,), "order"),
                                     _ptr(covered, torch.int32, (self.n_views,), "covered"), _stream()),
               "hr_camera_order")

    def set_joint_prior(self, target_joints=None, lam=0.0, gamma=0.005):
        """Joint prior lambda E2 (Section 3.2, Eq. 5) for the backwards enqueued from now
        on: target_joints a CUDA float32 tensor [n_hands,J,3], None to switch off.
        The scene keeps a reference to every target it was given: backwards and
        graphs captured while it was set read it."""
        ptr = _ptr(target_joints, shape=(self.n_hands, self.J, 3), name="target_joints")
        _check(lib().hr_set_joint_prior(self._h, ptr, float(lam), float(gamma)), "hr_set_joint_prior")
        if target_joints is not None:
            self._keep.append(target_joints)

    def step(self, params, albedo, grad_params, grad_albedo, m_p, v_p, m_a, v_a, t, lrs, betas=(0.9, 0.999),
             eps=1e-8):
        c = adam_config(lrs, betas, eps)
        shp_p, shp_a = (self.n_hands, 64), (self.n_hands, self.tex_h, self.tex_w, 3)
        _check(lib().hr_step(self._h, _ptr(params, shape=shp_p, name="params"),
                             _ptr(albedo, shape=shp_a, name="albedo"), _ptr(grad_params, shape=shp_p, name="gp"),
                             _ptr(grad_albedo, shape=shp_a, name="ga"), _ptr(m_p, shape=shp_p, name="m_p"),
                             _ptr(v_p, shape=shp_p, name="v_p"), _ptr(m_a, shape=shp_a, name="m_a"),
                             _ptr(v_a, shape=shp_a, name="v_a"), int(t), ctypes.byref(c), _stream()), "hr_step")

    # -- whole iterations ----------------------------------------------------
    def make_state(self, params, albedo, background, target, mask=None, iter0=0):
        """Allocate the buffers of a refinement loop around the given tensors (which
        it owns from now on: params/albedo are updated in place)."""
        return LoopState(self, params, albedo, background, target, mask, iter0)

    def iterate(self, state, lrs, flags=HR_GRAD_ALL, betas=(0.9, 0.999), eps=1e-8):
        _check(lib().hr_iterate(self._h, ctypes.byref(state.c), ctypes.byref(adam_config(lrs, betas, eps)),
                                int(flags), _stream()), "hr_iterate")

    def graph(self, state, lrs, n_iters=1, flags=HR_GRAD_ALL, betas=(0.9, 0.999), eps=1e-8):
        return Graph(self, state, adam_config(lrs, betas, eps), int(flags), int(n_iters))

    def set_grid(self, render_blocks=0, adjoint_blocks=0):
        _check(lib().hr_set_grid(self._h, int(render_blocks), int(adjoint_blocks)), "hr_set_grid")

    # -- the full data term (colour transforms, blurred-Canny edge term, two-level colour map) --
    def data_term_set(self, w_edge=1.0, low=0.1, high=0.2):
        c = DataTerm()
        c.w_edge, c.low, c.high = float(w_edge), float(low), float(high)
        _check(lib().hr_data_term_set(self._h, ctypes.byref(c)), "hr_data_term_set")

    def edge_map(self, image, T, out):
        """B(Canny(T image)) [P] of every view (T [n_views,9] or None)."""
        _check(lib().hr_edge_map(self._h, _ptr(image, shape=(self.P, 3), name="image"),
                                 _ptr(T, shape=(self.n_views, 9), name="T"),
                                 _ptr(out, shape=(self.P,), name="edge_map"), _stream()), "hr_edge_map")

    def loss_full(self, image, T, target, target_edges, mask, loss, dimage, grad_T=None, edge_map=None):
        _check(lib().hr_loss_full(self._h, _ptr(image, shape=(self.P, 3), name="image"),
                                  _ptr(T, shape=(self.n_views, 9), name="T"),
                                  _ptr(target, shape=(self.P, 3), name="target"),
                                  _ptr(target_edges, shape=(self.P,), name="target_edges"),
                                  _ptr(mask, torch.uint8, (self.P,), "mask"),
                                  _ptr(loss, shape=(self.n_hands,), name="loss"),
                                  _ptr(dimage, shape=(self.P, 3), name="dimage"),
                                  _ptr(grad_T, shape=(self.n_views, 9), name="grad_T"),
                                  _ptr(edge_map, shape=(self.P,), name="edge_map"), _stream()), "hr_loss_full")

    def compose_albedo(self, low, high, out):
        L = int(low.shape[1])
        _check(lib().hr_compose_albedo(self._h, _ptr(low, shape=(self.n_hands, L, L, 3), name="low"), L,
                                       _ptr(high, shape=(self.n_hands, self.tex_h, self.tex_w, 3), name="high"),
                                       _ptr(out, shape=(self.n_hands, self.tex_h, self.tex_w, 3), name="albedo"),
                                       _stream()), "hr_compose_albedo")

    def albedo_low_grad(self, grad_albedo, grad_low):
        L = int(grad_low.shape[1])
        _check(lib().hr_albedo_low_grad(self._h, _ptr(grad_albedo, shape=(self.n_hands, self.tex_h, self.tex_w, 3),
                                                      name="grad_albedo"), L,
                                        _ptr(grad_low, shape=(self.n_hands, L, L, 3), name="grad_low"), _stream()),
               "hr_albedo_low_grad")

    def adam(self, x, g, m, v, t, lr, lo=-3.4e38, hi=3.4e38, betas=(0.9, 0.999), eps=1e-8):
        """One Adam step on the float32 tensor x in place (clamped to [lo, hi])."""
        n = int(x.numel())
        c = adam_config((0.0,) * 6, betas, eps)
        _check(lib().hr_adam(self._h, _ptr(x, shape=tuple(x.shape), name="x"), _ptr(g, shape=tuple(x.shape), name="g"),
                             _ptr(m, shape=tuple(x.shape), name="m"), _ptr(v, shape=tuple(x.shape), name="v"), n,
                             int(t), float(lr), float(lo), float(hi), ctypes.byref(c), _stream()), "hr_adam")

    def set_accel(self, mode):
        """HR_ACCEL_AUTO (screen bins for the camera rays) or HR_ACCEL_HIERARCHY."""
        _check(lib().hr_set_accel(self._h, int(mode)), "hr_set_accel")

    def set_render_edges(self, enable):
        """hr_render also traces the edge samples for a following reusing backward."""
        _check(lib().hr_set_render_edges(self._h, int(bool(enable))), "hr_set_render_edges")

    def set_edge_budget(self, units_per_sample=256):
        """Edge samples per view = ceil(quantised silhouette length / units) (256: one per pixel)."""
        _check(lib().hr_set_edge_budget(self._h, int(units_per_sample)), "hr_set_edge_budget")

    def set_renderer(self, mode):
        """HR_RENDERER_RAY (Monte Carlo ray tracing) or HR_RENDERER_RASTER (hard
        rasterisation at pixel centres; scenes of 1 sample per pixel)."""
        _check(lib().hr_set_renderer(self._h, int(mode)), "hr_set_renderer")

    def set_tiles(self, tile_w_log2, bin_log2):
        """Wave tiles of 2^tile_w_log2 pixels across (the height follows from the
        samples per pixel) and screen bins of 2^bin_log2 pixels; images never change."""
        _check(lib().hr_set_tiles(self._h, int(tile_w_log2), int(bin_log2)), "hr_set_tiles")

    def tiles(self):
        """(tile width log2, tile height log2, bin size log2)."""
        out = np.zeros(3, dtype=np.int32)
        _check(lib().hr_get_tiles(self._h, out.ctypes.data_as(ctypes.c_void_p)), "hr_get_tiles")
        return int(out[0]), int(out[1]), int(out[2])

    def grids(self):
        """(render blocks, adjoint blocks) of the persistent ray-tracing grids."""
        out = np.zeros(2, dtype=np.int32)
        _check(lib().hr_get_grid(self._h, out.ctypes.data_as(ctypes.c_void_p)), "hr_get_grid")
        return int(out[0]), int(out[1])

    def tune(self, state, reps=3):
        """Time candidate tile shapes and bin sizes, then persistent grids; returns
        (render blocks, adjoint blocks) (the tile choice: tiles())."""
        out = np.zeros(2, dtype=np.int32)
        _check(lib().hr_tune(self._h, ctypes.byref(state.c), int(reps), out.ctypes.data_as(ctypes.c_void_p),
                             _stream()), "hr_tune")
        return int(out[0]), int(out[1])

    # -- learned edge-sampling proposal ----------------------------------------
    def proposal_set(self, kind=HR_PROPOSAL_LEARNED, theta=None, eps=1e-3, ema=0.9, lr=1e-3, betas=(0.9, 0.999),
                     adam_eps=1e-8):
        """Select the edge proposal; theta: flat [HR_MLP_PARAMS] or a dict of the
        MLP_LAYOUT arrays (None keeps the current network)."""
        c = ProposalConfig()
        c.kind, c.eps, c.ema, c.lr = int(kind), float(eps), float(ema), float(lr)
        c.beta1, c.beta2, c.adam_eps = float(betas[0]), float(betas[1]), float(adam_eps)
        buf = None
        if theta is not None:
            buf = np.ascontiguousarray(flat_mlp(theta), dtype=np.float32)
        _check(lib().hr_proposal_set(self._h, ctypes.byref(c),
                                     buf.ctypes.data_as(ctypes.c_void_p) if buf is not None else None),
               "hr_proposal_set")
        self._z_override = None

    def proposal_get(self):
        out = np.zeros(HR_MLP_PARAMS, dtype=np.float32)
        _check(lib().hr_proposal_get(self._h, out.ctypes.data_as(ctypes.c_void_p), _stream()), "hr_proposal_get")
        return out

    def proposal_override(self, z=None):
        """Logits [n_views,E] (CUDA float32) to use instead of the network, or None."""
        E = self._n_edges
        _check(lib().hr_proposal_override(self._h, _ptr(z, shape=(self.n_views, E), name="z")),
               "hr_proposal_override")
        self._z_override = z   # keep alive

    def proposal_train(self):
        _check(lib().hr_proposal_train(self._h, _stream()), "hr_proposal_train")

    def proposal_features(self):
        out = torch.empty(self.n_views, self._n_edges, 16, device=torch.cuda.current_device())
        _check(lib().hr_proposal_features(self._h, _ptr(out), _stream()), "hr_proposal_features")
        return out

    def proposal_stats(self):
        """(z, wq, a, dc) of the last proposal pass / backward records."""
        dev = torch.cuda.current_device()
        shp = (self.n_views, self._n_edges)
        z = torch.empty(shp, device=dev)
        wq = torch.empty(shp, device=dev, dtype=torch.int32)
        a = torch.empty(shp, device=dev)
        dc = torch.empty(*shp, 4, device=dev)
        _check(lib().hr_proposal_stats(self._h, _ptr(z), _ptr(wq, torch.int32), _ptr(a), _ptr(dc), _stream()),
               "hr_proposal_stats")
        return z, wq, a, dc

    def proposal_eval(self, X):
        X = X.contiguous()
        z = torch.empty(X.shape[0], device=X.device)
        _check(lib().hr_proposal_eval(self._h, _ptr(X, shape=(X.shape[0], 16), name="X"), int(X.shape[0]), _ptr(z),
                                      _stream()), "hr_proposal_eval")
        return z

    def proposal_fit(self, X, w, a, apply=False):
        n = int(X.shape[0])
        grad = torch.empty(HR_MLP_PARAMS, device=X.device)
        _check(lib().hr_proposal_fit(self._h, _ptr(X.contiguous(), shape=(n, 16), name="X"),
                                     _ptr(w.contiguous(), torch.int32, (n,), "w"),
                                     _ptr(a.contiguous(), shape=(n,), name="a"), n, _ptr(grad), int(bool(apply)),
                                     _stream()), "hr_proposal_fit")
        return grad

    def edge_stats(self):
        tot = np.zeros(self.n_views, dtype=np.uint64)
        bud = np.zeros(self.n_views, dtype=np.int64)
        _check(lib().hr_edge_stats(self._h, tot.ctypes.data_as(ctypes.c_void_p),
                                   bud.ctypes.data_as(ctypes.c_void_p), _stream()), "hr_edge_stats")
        return tot, bud

    # -- profiling aids --------------------------------------------------------
    def set_counting(self, enable):
        _check(lib().hr_set_counting(self._h, int(bool(enable))), "hr_set_counting")

    def read_counts(self):
        """{kernel: (rays, nodes, triangle tests, hits, packet node visits,
        packet triangle tests)} since the last read (per-ray counts, then the
        wave packets' counts per active lane)."""
        c = np.zeros(18, dtype=np.uint64)
        _check(lib().hr_read_counts(self._h, c.ctypes.data_as(ctypes.c_void_p), _stream()), "hr_read_counts")
        c = c.reshape(3, 6).astype(np.int64)
        return {"k_render": tuple(c[0]), "k_adjoint_interior": tuple(c[1]), "k_edge_sample": tuple(c[2])}

    def timing_enable(self, enable):
        _check(lib().hr_timing_enable(self._h, int(bool(enable))), "hr_timing_enable")

    def timing_read(self):
        """{kernel name: (total ms, launches)} since the last read."""
        n_max = 64
        names = ctypes.create_string_buffer(32 * n_max)
        ms = np.zeros(n_max, dtype=np.float64)
        cnt = np.zeros(n_max, dtype=np.int64)
        n = ctypes.c_int32(0)
        _check(lib().hr_timing_read(self._h, names, ms.ctypes.data_as(ctypes.c_void_p),
                                    cnt.ctypes.data_as(ctypes.c_void_p), n_max, ctypes.byref(n), _stream()),
               "hr_timing_read")
        raw = names.raw
        out = {}
        for i in range(n.value):
            nm = raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out


def adam_config(lrs, betas=(0.9, 0.999), eps=1e-8):
    """hr_adam_config from (root pose, pose, shape, rotation, translation, albedo) rates."""
    c = AdamConfig()
    (c.lr_pose_root, c.lr_pose, c.lr_shape, c.lr_rot, c.lr_trans, c.lr_albedo) = [float(x) for x in lrs]
    c.beta1, c.beta2, c.eps = float(betas[0]), float(betas[1]), float(eps)
    return c


class LoopState:
    """Device buffers of a refinement loop (hr_state)."""

    def __init__(self, scene, params, albedo, background, target, mask=None, iter0=0):
        dev = params.device
        H, V, P = scene.n_hands, scene.V, scene.P
        shp_a = (H, scene.tex_h, scene.tex_w, 3)
        self.params, self.albedo = params, albedo
        self.m_params, self.v_params = torch.zeros_like(params), torch.zeros_like(params)
        self.m_albedo, self.v_albedo = torch.zeros_like(albedo), torch.zeros_like(albedo)
        self.background, self.target, self.mask = background, target, mask
        self.verts = torch.empty(H, V, 3, device=dev)
        self.image = torch.empty(P, 3, device=dev)
        self.dimage = torch.empty(P, 3, device=dev)
        self.loss = torch.empty(H, device=dev)
        self.grad_params = torch.empty_like(params)
        self.grad_albedo = torch.empty_like(albedo)
        self.iter = torch.full((1,), int(iter0), dtype=torch.int32, device=dev)
        c = State()
        c.params = _ptr(params, shape=(H, 64), name="params")
        c.albedo = _ptr(albedo, shape=shp_a, name="albedo")
        c.m_params, c.v_params = _ptr(self.m_params), _ptr(self.v_params)
        c.m_albedo, c.v_albedo = _ptr(self.m_albedo), _ptr(self.v_albedo)
        c.background = _ptr(background, shape=(P, 3), name="background")
        c.target = _ptr(target, shape=(P, 3), name="target")
        c.mask = _ptr(mask, torch.uint8, (P,), "mask")
        c.verts, c.image, c.dimage, c.loss = _ptr(self.verts), _ptr(self.image), _ptr(self.dimage), _ptr(self.loss)
        c.grad_params, c.grad_albedo = _ptr(self.grad_params), _ptr(self.grad_albedo)
        c.iter = _ptr(self.iter, torch.int32, (1,), "iter")
        self.c = c


class Graph:
    """n_iters captured iterations (hr_graph); launch() enqueues them."""

    def __init__(self, scene, state, cfg, flags, n_iters):
        self.scene, self.state, self.n_iters = scene, state, n_iters   # keep the buffers alive
        h = ctypes.c_void_p()
        _check(lib().hr_graph_create(ctypes.byref(h), scene._h, ctypes.byref(state.c), ctypes.byref(cfg), flags,
                                     n_iters), "hr_graph_create")
        self._h = h

    def launch(self):
        _check(lib().hr_graph_launch(self._h, _stream()), "hr_graph_launch")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hr_graph_destroy(h)
            self._h = None


def flat_mlp(theta):
    """Flat float32 [HR_MLP_PARAMS] from a dict of the MLP_LAYOUT arrays (or a flat array)."""
    if isinstance(theta, dict):
        return np.concatenate([np.asarray(theta[k], np.float32).reshape(-1) for k, _ in MLP_LAYOUT])
    a = np.asarray(theta, np.float32).reshape(-1)
    if a.size != HR_MLP_PARAMS:
        raise HRError(f"expected {HR_MLP_PARAMS} network parameters, got {a.size}")
    return a
