"""Oracle of the learned edge-sampling proposal (test infrastructure only).

A project addition on top of the paper's silhouette sampling (Section 4.2.2,
after Li et al. 2018): edge samples are drawn from a per-view distribution
over silhouette edges that a small multilayer perceptron adapts online, instead
of in proportion to screen length only.  Any distribution that gives every
silhouette edge positive weight keeps the boundary estimate unbiased (each
sample is divided by its own probability), so the proposal only changes the
variance.

Plain float64 numpy, written for checking by eye:
  edge_features   per (view, silhouette edge) 16 inputs
  mlp_forward     16 -> 64 -> 64 -> 1 with erf-GELU, at the rounding points of
                  the device kernels (bfloat16 operands, wider accumulation)
  proposal_weights  integer sampling weights from the logits
  kl_grad         gradient of sum over views of KL(target || proposal)

The rounding points are part of what the device computes (it multiplies
bfloat16 operands and accumulates in float32); the oracle rounds the same
values to bfloat16, through float32, and accumulates in float64.  With
`rounded=False` every function is the exact float64 network.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN, N_HID = 16, 64
# flat parameter layout: W1 [16,64] (input-major), b1 [64], W2 [64,64], b2 [64], w3 [64], b3 [1]
SIZES = (("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("w3", (N_HID,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)   # 5313


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64).ravel()
    assert theta.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def flatten(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), through float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(x))


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def mlp_forward(theta, X, rounded=True):
    """Logits z [n] of the rows X [n,16] and the intermediates of the pass."""
    r = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    p = unflatten(theta)
    Xb = r(X)
    A1 = Xb @ r(p["W1"]) + p["b1"]
    H1 = r(gelu(A1))
    A2 = H1 @ r(p["W2"]) + p["b2"]
    H2 = r(gelu(A2))
    z = H2 @ r(p["w3"]) + p["b3"][0]
    return z, dict(X=Xb, A1=A1, H1=H1, A2=A2, H2=H2)


def _softmax_weighted(w, z):
    """q_e = w_e exp(z_e) / sum_f w_f exp(z_f) over the entries with w > 0."""
    q = np.zeros_like(z, dtype=np.float64)
    live = w > 0
    if not live.any():
        return q
    zl = z[live]
    e = np.asarray(w, dtype=np.float64)[live] * np.exp(zl - zl.max())
    q[live] = e / e.sum()
    return q


def kl_loss(theta, X, w, a, group, rounded=False):
    """sum over groups g of KL(pi_g || q_g), pi = a / sum a within the group,
    q = w exp(z) / sum w exp(z); groups without signal (sum a = 0) add nothing."""
    z, _ = mlp_forward(theta, X, rounded)
    total = 0.0
    for gi in np.unique(group):
        m = group == gi
        wa, aa = np.asarray(w, np.float64)[m], np.asarray(a, np.float64)[m]
        if aa.sum() <= 0:
            continue
        pi = aa / aa.sum()
        q = _softmax_weighted(wa, z[m])
        nz = pi > 0
        total += float(np.sum(pi[nz] * np.log(pi[nz] / q[nz])))
    return total


def kl_grad(theta, X, w, a, group, rounded=True):
    """Gradient of kl_loss with respect to the flat parameters.  dL/dz_e =
    q_e - pi_e per group; back-propagated with the device's rounding points:
    the layer-2 and layer-1 pre-activation gradients are rounded to bfloat16
    where they enter products (the bias gradients use them unrounded)."""
    r = bf16 if rounded else (lambda x: np.asarray(x, dtype=np.float64))
    p = unflatten(theta)
    z, c = mlp_forward(theta, X, rounded)
    dz = np.zeros_like(z)
    w = np.asarray(w, np.float64)
    a = np.asarray(a, np.float64)
    for gi in np.unique(group):
        m = group == gi
        if a[m].sum() <= 0:
            continue
        dz[m] = _softmax_weighted(w[m], z[m]) - a[m] / a[m].sum()
    g = {}
    g["w3"] = c["H2"].T @ dz
    g["b3"] = np.array([dz.sum()])
    dA2 = dz[:, None] * r(p["w3"])[None, :] * gelu_grad(c["A2"])
    g["b2"] = dA2.sum(0)
    dA2r = r(dA2)
    g["W2"] = c["H1"].T @ dA2r
    dH1 = dA2r @ r(p["W2"]).T
    dA1 = dH1 * gelu_grad(c["A1"])
    g["b1"] = dA1.sum(0)
    g["W1"] = c["X"].T @ r(dA1)
    return flatten(g)


EPS = float(np.float32(1e-3))   # the float32 value the device uses


def proposal_weights(w, z, eps=EPS):
    """Integer sampling weights of one view from the length weights w (u32) and
    logits z: with E_e = exp(z_e - max z) and the length-weighted mean
    Ebar = sum w E / sum w, W_e = max(1, floor(w_e (1 + (1 - eps)(E_e / Ebar - 1))))
    on silhouette edges (w_e > 0), 0 elsewhere.  The total stays about sum w;
    every edge keeps at least the share eps w_e of the length-proportional
    proposal; equal logits give W = w exactly."""
    w = np.asarray(w, dtype=np.uint64)
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros(w.shape, dtype=np.uint32)
    live = w > 0
    if not live.any():
        return out
    wl = w[live].astype(np.float64)
    E = np.exp(z[live] - z[live].max())
    ebar = np.sum(wl * E) / np.sum(wl)
    rr = 1.0 + (1.0 - eps) * (E / ebar - 1.0)
    W = np.floor(wl * rr)
    out[live] = np.maximum(1.0, np.minimum(W, 4294967295.0)).astype(np.uint32)
    return out


def _bilinear(tex, u, v):
    """Colour map lookup with texel centres at ((j + 0.5)/T_w, (i + 0.5)/T_h),
    clamp to edge (the shading model of the renderer)."""
    th, tw = tex.shape[:2]
    x = u * tw - 0.5
    y = v * th - 0.5
    j0, i0 = int(np.floor(x)), int(np.floor(y))
    fx, fy = x - j0, y - i0
    out = np.zeros(3)
    for di, wy in ((0, 1.0 - fy), (1, fy)):
        for dj, wx in ((0, 1.0 - fx), (1, fx)):
            i = min(max(i0 + di, 0), th - 1)
            j = min(max(j0 + dj, 0), tw - 1)
            out += wy * wx * tex[i, j]
    return out


def edge_features(sc, verts, normals, albedo, background, ema=None, ema_valid=None):
    """Inputs of the network per (view, edge) [n_views,E,16] for the oracle
    scene `sc`; zero rows where the edge is not sampled (w = 0).

    For a silhouette edge of view v with float32 record (ax, ay, bx, by, t0, t1):
      0-3  clipped endpoints a + t0 d and a + t1 d over (W, H)
      4    clipped screen length over the image diagonal
      5, 6 larger and smaller of n_f . vhat over the adjacent faces (unit face
           normals, vhat the unit direction from the edge midpoint to the
           camera centre; a boundary edge's missing face counts as 0)
      7-9  colour jump across the edge: the running average of measured
           |c- - c+| where the edge has one (ema_valid), else |shade -
           background| at the edge midpoint (smooth normal and colour-map value
           of the midpoint; background pixel under the projected midpoint)
      10-15 zero
    verts [H,V,3] (float32 values), normals [H,V,3] unit vertex normals,
    albedo [H,th,tw,3], background [P,3]; ema [n_views,E,3], ema_valid [n_views,E]."""
    from . import edge_weights   # the oracle's own silhouette tables
    verts = np.asarray(verts, dtype=np.float64).reshape(-1, sc.V, 3)
    normals = np.asarray(normals, dtype=np.float64).reshape(-1, sc.V, 3)
    albedo = np.asarray(albedo, dtype=np.float64)
    albedo = albedo.reshape(-1, *albedo.shape[-3:])
    background = np.asarray(background, dtype=np.float64).reshape(sc.P, 3)
    w, _, _, _, rec = edge_weights(sc, verts, want_rec=True)
    n_views, E = w.shape
    out = np.zeros((n_views, E, 16))
    ka, kd, light = sc.shading[0], sc.shading[1], np.asarray(sc.shading[2:5], dtype=np.float64)
    cam = sc.cam
    for vi in range(n_views):
        Wi, Hi = int(cam["wh"][vi, 0]), int(cam["wh"][vi, 1])
        W, H = float(Wi), float(Hi)
        diag = np.sqrt(W * W + H * H)
        hand = int(cam["hand"][vi])
        o = cam["o"][vi].astype(np.float64)
        vh, nh, tex = verts[hand], normals[hand], albedo[hand]
        p0 = int(cam["pix_off"][vi])
        for e in np.nonzero(w[vi] > 0)[0]:
            ax, ay, bx, by, t0, t1 = (float(x) for x in rec[vi, e])
            dx, dy = bx - ax, by - ay
            f = out[vi, e]
            f[0], f[1] = (ax + t0 * dx) / W, (ay + t0 * dy) / H
            f[2], f[3] = (ax + t1 * dx) / W, (ay + t1 * dy) / H
            f[4] = np.hypot(dx, dy) * (t1 - t0) / diag
            va, vb = sc.edges[e]
            mid = 0.5 * (vh[va] + vh[vb])
            vhat = (o - mid) / np.linalg.norm(o - mid)
            dots = []
            for k in range(2):
                fi = sc.edge_faces[e][k]
                if fi < 0:
                    dots.append(0.0)
                    continue
                q0, q1, q2 = vh[sc.faces[fi]]
                nf = np.cross(q1 - q0, q2 - q0)
                dots.append(float(np.dot(nf / np.linalg.norm(nf), vhat)))
            f[5], f[6] = max(dots), min(dots)
            if ema_valid is not None and ema_valid[vi, e]:
                f[7:10] = ema[vi, e]
            else:
                um = 0.5 * (sc.uv[va] + sc.uv[vb])
                nm = nh[va] + nh[vb]
                nm = nm / np.linalg.norm(nm)
                col = _bilinear(tex, um[0], um[1]) * (ka + kd * max(0.0, float(np.dot(nm, light))))
                px = min(max(int(np.floor(0.5 * (ax + bx))), 0), Wi - 1)
                py = min(max(int(np.floor(0.5 * (ay + by))), 0), Hi - 1)
                f[7:10] = np.abs(col - background[p0 + py * Wi + px])
    return out
