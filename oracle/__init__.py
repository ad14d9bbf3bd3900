"""Reference implementation of the render-and-compare hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the package smoke check and by
the CPU-baseline leg of the benchmark.  The product path never imports it.

What it computes, step by step (paper Section 3; the data term is Eq. 3 with the
colour difference D_c of Eq. 4, the optimiser is Adam, Section 3.3):

* skin         -- linear blend skinning of the hand model: shape blend, joint
                  regression, per-joint Rodrigues rotations, forward kinematics,
                  blend of joint transforms, global rotation and translation
                  (G_v of Section 3.1; G_J of Section 3.2, Eq. 5).  float64 torch.
* normals      -- area-weighted unit vertex normals.  float64 torch.
* render       -- Monte Carlo pixel integrals (Section 3: each rendered pixel is
                  an integral of samples); brute-force closest hit.  C, float64.
* l1_loss      -- E1 = sum over views of the mean |O - I| over masked pixels
                  and channels, and dE1/dI.  float64 NumPy.
* backward     -- interior term (derivative of the estimate at fixed samples)
                  plus the silhouette-edge boundary term (Section 4.2.2; the
                  edge sampling of Li et al. 2018).  C, float64; the gradient is
                  carried through normals and skinning with torch autograd.
* adam_step    -- Kingma & Ba's update.  float64 NumPy.

The float32 decisions and the Philox streams are described in ora.c.  Pins of
every function live in tests/ (test_oracle_*.py); see there for what fixes each.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ora.c")
_SO = os.path.join(_HERE, "_ora.so")
_lib = None


def build(force=True):
    """Compile ora.c into oracle/_ora.so."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        _lib = ctypes.CDLL(_SO)
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# --------------------------------------------------------------------------
# Philox
# --------------------------------------------------------------------------

def philox4x64(ctr, key):
    """Philox4x64-10 of counters [n,4] (uint64) under key [2] (uint64)."""
    ctr = _c(np.atleast_2d(ctr), np.uint64)
    key = _c(key, np.uint64)
    out = np.zeros_like(ctr)
    lib().ora_philox4x64(_p(ctr), _p(key), _p(out), ctypes.c_int64(len(ctr)))
    return out


# --------------------------------------------------------------------------
# renderer (C)
# --------------------------------------------------------------------------

class Scene:
    """Static description: mesh topology/uv, cameras (float32 tables), shading."""

    def __init__(self, faces, uv, cam, shading, edges=None, edge_faces=None):
        self.faces = _c(faces, np.int32)
        self.uv = _c(uv, np.float64)
        self.V = self.uv.shape[0]
        self.F = self.faces.shape[0]
        dts = dict(R=np.float32, o=np.float32, intr=np.float32, wh=np.int32, hand=np.int32,
                   pix_off=np.int64)
        self.cam = {k: _c(cam[k], dt) for k, dt in dts.items()}
        self.n_views = self.cam["R"].shape[0]
        self.P = int(self.cam["pix_off"][-1])
        self.shading = _c(shading, np.float64)
        self.edges = None if edges is None else _c(edges, np.int32)
        self.edge_faces = None if edge_faces is None else _c(edge_faces, np.int32)

    def _cam_args(self):
        c = self.cam
        return (ctypes.c_int(self.n_views), _p(c["R"]), _p(c["o"]), _p(c["intr"]), _p(c["wh"]),
                _p(c["hand"]), _p(c["pix_off"]))


def render(sc: Scene, verts, normals, albedo, background, spp, seed, it, want_hits=False):
    """Image [P,3] float64 (and per-sample hit face ids [P,spp] if asked)."""
    verts = _c(verts, np.float64).reshape(-1, sc.V, 3)
    normals = _c(normals, np.float64).reshape(-1, sc.V, 3)
    albedo = _c(albedo, np.float64)
    albedo = albedo.reshape(-1, *albedo.shape[-3:])
    th, tw = albedo.shape[1], albedo.shape[2]
    background = _c(background, np.float64).reshape(sc.P, 3)
    img = np.zeros((sc.P, 3))
    hits = np.zeros((sc.P, spp), dtype=np.int32) if want_hits else None
    lib().ora_render(ctypes.c_int(verts.shape[0]), ctypes.c_int(sc.V), ctypes.c_int(sc.F),
                     _p(verts), _p(normals), _p(sc.faces), _p(sc.uv), ctypes.c_int(th),
                     ctypes.c_int(tw), _p(albedo), _p(background), *sc._cam_args(),
                     _p(sc.shading), ctypes.c_int(spp), ctypes.c_uint64(seed), ctypes.c_uint32(it),
                     _p(img), _p(hits) if want_hits else None)
    return (img, hits) if want_hits else img


def face_visibility(hits, pix_off, F):
    """visible [N,F] bool: view i sees face f when one of its camera samples hit
    f (Section 4.2.3, camera coverage: the surface a view makes visible, counted in
    triangles).  hits [P,spp] per-sample face ids (-1 miss), views packed by
    pix_off [N+1]."""
    N = len(pix_off) - 1
    vis = np.zeros((N, F), dtype=bool)
    for i in range(N):
        h = np.asarray(hits[pix_off[i]:pix_off[i + 1]]).ravel()
        vis[i, h[h >= 0]] = True
    return vis


def camera_order(visible, hand_views):
    """Greedy order of each hand's views (Section 4.2.3, camera coverage, Eq. 6):
    each step takes the view that adds the most faces not seen by the views
    taken before (ties: the earlier view of the hand's list).  Returns (order,
    covered), concatenated over the hands: view indices, and the faces seen by
    the first k + 1 views."""
    order, covered = [], []
    for views in hand_views:
        seen = np.zeros(visible.shape[1], dtype=bool)
        left, total = list(views), 0
        while left:
            gains = [int((visible[v] & ~seen).sum()) for v in left]
            k = int(np.argmax(gains))   # the first maximum: the earliest view
            v = left.pop(k)
            seen |= visible[v]
            total += gains[k]
            order.append(v)
            covered.append(total)
    return np.array(order, dtype=np.int64), np.array(covered, dtype=np.int64)


def backward_interior(sc: Scene, verts, normals, albedo, dimage, spp, seed, it):
    """(g_albedo, g_verts, g_normals) of sum(dimage * I) at fixed samples."""
    verts = _c(verts, np.float64).reshape(-1, sc.V, 3)
    normals = _c(normals, np.float64).reshape(-1, sc.V, 3)
    albedo = _c(albedo, np.float64)
    albedo = albedo.reshape(-1, *albedo.shape[-3:])
    th, tw = albedo.shape[1], albedo.shape[2]
    dimage = _c(dimage, np.float64).reshape(sc.P, 3)
    ga = np.zeros_like(albedo)
    gv = np.zeros_like(verts)
    gn = np.zeros_like(verts)
    lib().ora_backward_interior(ctypes.c_int(verts.shape[0]), ctypes.c_int(sc.V), ctypes.c_int(sc.F),
                                _p(verts), _p(normals), _p(sc.faces), _p(sc.uv), ctypes.c_int(th),
                                ctypes.c_int(tw), _p(albedo), *sc._cam_args(), _p(sc.shading),
                                ctypes.c_int(spp), ctypes.c_uint64(seed), ctypes.c_uint32(it),
                                _p(dimage), _p(ga), _p(gv), _p(gn))
    return ga, gv, gn


def edge_weights(sc: Scene, verts, want_rec=False):
    """Per (view, edge): quantised weights w (u32), inclusive prefix sums (u64),
    per-view totals and sample budgets (and, with want_rec, the float32 edge
    records [n_views,E,6]: projected endpoints and clipped interval)."""
    verts = _c(verts, np.float64).reshape(-1, sc.V, 3)
    E = sc.edges.shape[0]
    w = np.zeros((sc.n_views, E), dtype=np.uint32)
    cdf = np.zeros((sc.n_views, E), dtype=np.uint64)
    tot = np.zeros(sc.n_views, dtype=np.uint64)
    bud = np.zeros(sc.n_views, dtype=np.int64)
    rec = np.zeros((sc.n_views, E, 6), dtype=np.float32) if want_rec else None
    lib().ora_edge_weights(ctypes.c_int(verts.shape[0]), ctypes.c_int(sc.V), ctypes.c_int(sc.F),
                           _p(verts), _p(sc.faces), ctypes.c_int(E), _p(sc.edges), _p(sc.edge_faces),
                           *sc._cam_args(), _p(w), _p(cdf), _p(tot), _p(bud), _p(rec) if want_rec else None)
    return (w, cdf, tot, bud, rec) if want_rec else (w, cdf, tot, bud)


def backward_edges(sc: Scene, verts, normals, albedo, background, dimage, seed, it,
                   delta=1e-3, budget=None, want_stats=False, wq=None, want_dc=False):
    """Boundary-term vertex gradient [H,V,3]; with want_stats also the per-edge
    |contribution| sums [n_views,E]; with want_dc the per-edge colour-jump sums
    and counts [n_views,E,4].  wq [n_views,E] (u32, optional): sampling weights
    replacing the length weights on silhouette edges."""
    verts = _c(verts, np.float64).reshape(-1, sc.V, 3)
    normals = _c(normals, np.float64).reshape(-1, sc.V, 3)
    albedo = _c(albedo, np.float64)
    albedo = albedo.reshape(-1, *albedo.shape[-3:])
    th, tw = albedo.shape[1], albedo.shape[2]
    background = _c(background, np.float64).reshape(sc.P, 3)
    dimage = _c(dimage, np.float64).reshape(sc.P, 3)
    E = sc.edges.shape[0]
    gv = np.zeros_like(verts)
    stats = np.zeros((sc.n_views, E)) if want_stats else None
    bud = None if budget is None else _c(np.broadcast_to(budget, (sc.n_views,)), np.int64)
    wq = None if wq is None else _c(wq, np.uint32).reshape(sc.n_views, E)
    dc = np.zeros((sc.n_views, E, 4)) if want_dc else None
    lib().ora_backward_edges(ctypes.c_int(verts.shape[0]), ctypes.c_int(sc.V), ctypes.c_int(sc.F),
                             _p(verts), _p(normals), _p(sc.faces), _p(sc.uv), ctypes.c_int(th),
                             ctypes.c_int(tw), _p(albedo), _p(background), ctypes.c_int(E),
                             _p(sc.edges), _p(sc.edge_faces), *sc._cam_args(), _p(sc.shading),
                             ctypes.c_float(delta), ctypes.c_uint64(seed), ctypes.c_uint32(it),
                             _p(dimage), _p(bud) if bud is not None else None, _p(gv),
                             _p(stats) if want_stats else None, _p(wq) if wq is not None else None,
                             _p(dc) if want_dc else None)
    out = [gv] + ([stats] if want_stats else []) + ([dc] if want_dc else [])
    return out[0] if len(out) == 1 else tuple(out)


def trace_rays32(org, dirs, v32, faces):
    """Closest hit (face id or -1, t) of float32 rays against a triangle soup."""
    org = _c(org, np.float32).reshape(-1, 3)
    dirs = _c(dirs, np.float32).reshape(-1, 3)
    v32 = _c(v32, np.float32).reshape(-1, 3)
    faces = _c(faces, np.int32).reshape(-1, 3)
    n = org.shape[0]
    fo = np.zeros(n, dtype=np.int32)
    to = np.zeros(n, dtype=np.float32)
    lib().ora_trace_rays32(ctypes.c_int(n), _p(org), _p(dirs), ctypes.c_int(v32.shape[0]), _p(v32),
                           ctypes.c_int(faces.shape[0]), _p(faces), _p(fo), _p(to))
    return fo, to


def num_threads():
    return int(lib().ora_num_threads())


# --------------------------------------------------------------------------
# skinning and normals (float64 torch; gradients by autograd)
# --------------------------------------------------------------------------

def rodrigues(r):
    """Rotation matrices [...,3,3] of axis-angle vectors [...,3]:
    R = I + (sin a / a) K + ((1 - cos a) / a^2) K^2, K the cross-product matrix of r."""
    a2 = (r * r).sum(-1, keepdim=True)
    a = torch.sqrt(torch.clamp(a2, min=1e-300))
    small = a < 1e-4
    a_safe = torch.where(small, torch.ones_like(a), a)
    s = torch.where(small, 1.0 - a2 / 6.0, torch.sin(a_safe) / a_safe)
    c = torch.where(small, 0.5 - a2 / 24.0, (1.0 - torch.cos(a_safe)) / (a_safe * a_safe))
    zero = torch.zeros_like(r[..., 0])
    K = torch.stack([torch.stack([zero, -r[..., 2], r[..., 1]], -1),
                     torch.stack([r[..., 2], zero, -r[..., 0]], -1),
                     torch.stack([-r[..., 1], r[..., 0], zero], -1)], -2)
    eye = torch.eye(3, dtype=r.dtype).expand(K.shape)
    return eye + s[..., None] * K + c[..., None] * (K @ K)


class Model:
    """float64 torch copy of the hand model arrays."""

    def __init__(self, hm):
        f = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
        self.T = f(hm.v_template)
        self.S = f(hm.shapedirs)
        self.Jreg = f(hm.j_regressor)
        self.W = f(hm.weights)
        self.parents = [int(p) for p in hm.parents]
        self.faces = torch.as_tensor(np.asarray(hm.faces, dtype=np.int64))


def skin(m: Model, params):
    """params [H,64] float64 -> (verts [H,V,3], joints [H,J,3])."""
    H = params.shape[0]
    theta = params[:, 0:48].reshape(H, 16, 3)
    beta = params[:, 48:58]
    phi = params[:, 58:61]
    tau = params[:, 61:64]
    vs = m.T[None] + torch.einsum("vck,hk->hvc", m.S, beta)
    J = torch.einsum("jv,hvc->hjc", m.Jreg, vs)
    Rj = rodrigues(theta)
    GR, Gt = [], []
    for j, p in enumerate(m.parents):
        if p < 0:
            GR.append(Rj[:, j])
            Gt.append(J[:, j])
        else:
            GR.append(GR[p] @ Rj[:, j])
            Gt.append((GR[p] @ (J[:, j] - J[:, p])[..., None])[..., 0] + Gt[p])
    GR = torch.stack(GR, 1)                     # [H,J,3,3]
    Gt = torch.stack(Gt, 1)                     # [H,J,3]
    At = Gt - (GR @ J[..., None])[..., 0]       # A_j x = GR_j x + At_j
    vj = torch.einsum("hjab,hvb->hvja", GR, vs) + At[:, None]
    vp = torch.einsum("vj,hvja->hva", m.W, vj)
    Rp = rodrigues(phi)
    verts = torch.einsum("hab,hvb->hva", Rp, vp) + tau[:, None]
    joints = torch.einsum("hab,hjb->hja", Rp, Gt) + tau[:, None]
    return verts, joints


def joint_prior(joints, target, lam, gamma):
    """lambda E2 per hand (Section 3.2, Eq. 5: the prior term of the objective
    E = E1 + lambda E2): over joints [H,J,3] and their coordinates, the smooth
    L1 distance to the target joints with threshold gamma, d^2 / (2 gamma)
    where |d| < gamma and |d| - gamma / 2 elsewhere."""
    d = joints - torch.as_tensor(np.asarray(target, dtype=np.float64))
    ad = d.abs()
    f = torch.where(ad < gamma, 0.5 * d * d / gamma, ad - 0.5 * gamma)
    return lam * f.sum(dim=(1, 2))


def vertex_normals(verts, faces):
    """Unit vertex normals: normalised sum of the incident faces' (v1-v0)x(v2-v0)."""
    v0 = verts[:, faces[:, 0]]
    v1 = verts[:, faces[:, 1]]
    v2 = verts[:, faces[:, 2]]
    fn = torch.cross(v1 - v0, v2 - v0, dim=-1)
    n = torch.zeros_like(verts)
    for k in range(3):
        n = n.index_add(1, faces[:, k], fn)
    return n / torch.linalg.norm(n, dim=-1, keepdim=True)


# --------------------------------------------------------------------------
# loss and optimiser
# --------------------------------------------------------------------------

def l1_loss(image, target, mask, pix_off, view_hand, n_hands):
    """Per-hand E1 = sum over the hand's views of mean |I - O| over the view's
    masked pixels and the 3 channels, and dE1/dI (sign(0) = 0)."""
    image = np.asarray(image, dtype=np.float64).reshape(-1, 3)
    target = np.asarray(target, dtype=np.float64).reshape(-1, 3)
    P = image.shape[0]
    mask = np.ones(P, dtype=bool) if mask is None else np.asarray(mask).reshape(-1) != 0
    loss = np.zeros(n_hands)
    dimg = np.zeros_like(image)
    for v in range(len(pix_off) - 1):
        a, b = int(pix_off[v]), int(pix_off[v + 1])
        m = mask[a:b]
        cnt = int(m.sum())
        if cnt == 0:
            continue
        diff = image[a:b] - target[a:b]
        loss[view_hand[v]] += np.abs(diff[m]).sum() / (3.0 * cnt)
        dimg[a:b][m] = np.sign(diff[m]) / (3.0 * cnt)
    return loss, dimg


def adam_step(x, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8, lo=None, hi=None):
    """One Adam step (t counts from 1).  lr may be an array (0 freezes an entry:
    x, m and v of a frozen entry stay unchanged).  Returns (x, m, v)."""
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    lr = np.broadcast_to(np.asarray(lr, dtype=np.float64), x.shape)
    live = lr != 0
    m2 = np.where(live, beta1 * m + (1 - beta1) * g, m)
    v2 = np.where(live, beta2 * v + (1 - beta2) * g * g, v)
    mh = m2 / (1 - beta1 ** t)
    vh = v2 / (1 - beta2 ** t)
    x2 = np.where(live, x - lr * mh / (np.sqrt(vh) + eps), x)
    if lo is not None or hi is not None:
        x2 = np.where(live, np.clip(x2, lo, hi), x2)
    return x2, m2, v2


# --------------------------------------------------------------------------
# one full gradient evaluation
# --------------------------------------------------------------------------

def gradient(model: Model, sc: Scene, params, albedo, background, target, mask, spp, seed, it,
             delta=1e-3, edges=True, interior=True, prior=None):
    """Loss per hand and its gradient w.r.t. params [H,64] and albedo, plus the
    intermediate arrays (for stage-by-stage comparisons).  prior: optional
    (target joints [H,J,3], lambda, gamma) of the joint prior, added to both."""
    p = torch.as_tensor(np.asarray(params, dtype=np.float64)).clone().requires_grad_(True)
    verts, joints = skin(model, p)
    normals = vertex_normals(verts, model.faces)
    v_np = verts.detach().numpy()
    n_np = normals.detach().numpy()
    img = render(sc, v_np, n_np, albedo, background, spp, seed, it)
    loss, dimg = l1_loss(img, target, mask, sc.cam["pix_off"], sc.cam["hand"], p.shape[0])
    ga = np.zeros_like(np.asarray(albedo, dtype=np.float64))
    gv = np.zeros_like(v_np)
    gn = np.zeros_like(v_np)
    if interior:
        ga, gv_i, gn = backward_interior(sc, v_np, n_np, albedo, dimg, spp, seed, it)
        gv = gv + gv_i
    if edges:
        gv = gv + backward_edges(sc, v_np, n_np, albedo, background, dimg, seed, it, delta)
    outs, grads = [verts, normals], [torch.as_tensor(gv), torch.as_tensor(gn)]
    if prior is not None:
        e2 = joint_prior(joints, *prior)
        loss = loss + e2.detach().numpy()
        outs.append(e2.sum())
        grads.append(None)
    torch.autograd.backward(outs, grads)
    return dict(loss=loss, grad_params=p.grad.numpy().copy(), grad_albedo=ga, image=img,
                dimage=dimg, verts=v_np, normals=n_np, joints=joints.detach().numpy(),
                g_verts=gv, g_normals=gn)
