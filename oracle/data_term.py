"""Reference implementation of the paper's full data term (TEST INFRASTRUCTURE
ONLY: imported by tests/ and the CPU-baseline leg of the benchmark, never by
the product path).

The data term of Eq. 3 compares each observed image O_i with the rendering
transformed by a per-camera 3x3 colour transform T_i (Section 3.1,
"Rendering"), through f1 = D_c + D_e of Eq. 4: the L1 colour difference and
the L1 difference of blurred Canny edge maps, D_e(o, r) = |Canny(o) * K -
Canny(r) * K| with K an 11x11 Gaussian of sigma 5 (Section 3.1,
"Render-and-compare").  The colour map is V = V_low + V_high, V_low 8x8
nearest-upsampled to V_high's size (Section 3.1, "Colour mapping").

Readings (the paper names the Canny detector and its library, not its
settings): grey = 0.299 R + 0.587 G + 0.114 B; Gaussian pre-smoothing 5x5,
sigma 1; Sobel kernels divided by 8; magnitude sqrt(gx^2 + gy^2 + 1e-6);
non-maximum suppression along the gradient direction quantised to four
orientations (boundaries at 22.5 and 67.5 degrees, a pixel is kept when it is
at least as large as both neighbours); thresholds 0.1 and 0.2 on the
magnitude; hysteresis by one 8-neighbour step (a weak pixel is kept when a
neighbour is strong).  Canny(x) = magnitude at the kept pixels, 0 elsewhere.
Every filter reads clamped-to-edge pixels outside the image.  The selection
(suppression, thresholds, hysteresis) is piecewise constant: the derivative
flows through the magnitude at the kept pixels only.  E1 per view = mean over
masked pixels and channels of |O - T R| + w_e * mean over masked pixels of
|B(Canny(O)) - B(Canny(T R))|, with B the blur by K.

Everything is float64.  The selection is taken by explicit tap sums in a fixed
order (the order the GPU kernels also use), values by the same code.
"""
from __future__ import annotations

import numpy as np
import torch

GREY = (0.299, 0.587, 0.114)
SMOOTH_SIZE, SMOOTH_SIGMA = 5, 1.0
BLUR_SIZE, BLUR_SIGMA = 11, 5.0
LOW, HIGH = 0.1, 0.2
EPS = 1e-6
TAN1 = np.sqrt(2.0) - 1.0      # tan 22.5 degrees
TAN2 = np.sqrt(2.0) + 1.0      # tan 67.5 degrees
SOBEL_X = np.array([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]]) / 8.0
SOBEL_Y = SOBEL_X.T.copy()


def gaussian_kernel(size, sigma):
    """Normalised 2-D Gaussian weights exp(-(i^2 + j^2) / (2 sigma^2)) on a
    size x size grid centred on the middle tap."""
    c = (size - 1) / 2.0
    i = np.arange(size) - c
    w = np.exp(-(i[:, None] ** 2 + i[None, :] ** 2) / (2.0 * sigma * sigma))
    return w / w.sum()


def correlate(x, w):
    """sum_{a,b} w[a,b] x[y + a - r, x + b - r] over the taps in row-major
    order, with clamped-to-edge pixels outside the image (H x W -> H x W)."""
    r = w.shape[0] // 2
    H, W = x.shape
    xp = np.pad(x, r, mode="edge")
    out = np.zeros_like(x, dtype=np.float64)
    for a in range(w.shape[0]):
        for b in range(w.shape[1]):
            out = out + w[a, b] * xp[a:a + H, b:b + W]
    return out


def grey(img):
    """[H,W,3] -> [H,W] luma."""
    return (GREY[0] * img[..., 0] + GREY[1] * img[..., 1]) + GREY[2] * img[..., 2]


def gradients(g):
    """Smoothed grey image's Sobel gradients and magnitude."""
    s = correlate(g, gaussian_kernel(SMOOTH_SIZE, SMOOTH_SIGMA))
    gx = correlate(s, SOBEL_X)
    gy = correlate(s, SOBEL_Y)
    return gx, gy, np.sqrt((gx * gx + gy * gy) + EPS)


def select(gx, gy, M, low=LOW, high=HIGH):
    """Canny's selection: non-maximum suppression along the quantised
    gradient direction, double threshold, one hysteresis step (bool [H,W])."""
    H, W = M.shape
    Mp = np.pad(M, 1, mode="edge")
    nb = lambda dy, dx: Mp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    ax, ay = np.abs(gx), np.abs(gy)
    horiz = ay <= TAN1 * ax
    vert = ay >= TAN2 * ax
    diag = ~horiz & ~vert & (gx * gy > 0)      # gradient towards (+x, +y): rows grow downwards
    anti = ~horiz & ~vert & ~(gx * gy > 0)
    keep = np.zeros((H, W), bool)
    keep |= horiz & (M >= nb(0, -1)) & (M >= nb(0, 1))
    keep |= vert & (M >= nb(-1, 0)) & (M >= nb(1, 0))
    keep |= diag & (M >= nb(-1, -1)) & (M >= nb(1, 1))
    keep |= anti & (M >= nb(-1, 1)) & (M >= nb(1, -1))
    strong = keep & (M > high)
    weak = keep & (M > low) & ~strong
    sp = np.pad(strong, 1, mode="constant")
    near = np.zeros((H, W), bool)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dy or dx:
                near |= sp[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    return strong | (weak & near)


def canny(img, low=LOW, high=HIGH):
    """Canny(x) of an RGB image [H,W,3]: magnitude at the selected pixels.
    Returns (edges, selection)."""
    gx, gy, M = gradients(grey(img))
    S = select(gx, gy, M, low, high)
    return np.where(S, M, 0.0), S


def edge_map(img, low=LOW, high=HIGH):
    """B(Canny(x)) [H,W]: the edge map blurred by the 11x11, sigma 5 Gaussian."""
    e, _ = canny(img, low, high)
    return correlate(e, gaussian_kernel(BLUR_SIZE, BLUR_SIGMA))


# --------------------------------------------------------------------------
# packed views
# --------------------------------------------------------------------------

def _views(a, wh, pix_off, ch):
    for v in range(len(wh)):
        W, H = int(wh[v][0]), int(wh[v][1])
        sl = slice(int(pix_off[v]), int(pix_off[v + 1]))
        yield v, sl, (a[sl].reshape(H, W, ch) if ch > 1 else a[sl].reshape(H, W))


def colour_transform(image, T, pix_off):
    """r' = T_v r for every pixel of view v: image [P,3], T [n_views,9] (row-major)."""
    image = np.asarray(image, np.float64)
    out = np.empty_like(image)
    for v in range(len(pix_off) - 1):
        sl = slice(int(pix_off[v]), int(pix_off[v + 1]))
        Tv = np.asarray(T, np.float64).reshape(-1, 3, 3)[v]
        x = image[sl]
        out[sl] = np.stack([(Tv[k, 0] * x[:, 0] + Tv[k, 1] * x[:, 1]) + Tv[k, 2] * x[:, 2] for k in range(3)], 1)
    return out


def edge_maps(image, wh, pix_off, low=LOW, high=HIGH):
    """B(Canny(view)) of every view, packed [P]."""
    image = np.asarray(image, np.float64)
    out = np.empty(image.shape[0])
    for v, sl, img in _views(image, wh, pix_off, 3):
        out[sl] = edge_map(img, low, high).reshape(-1)
    return out


def _edge_term_torch(rp, S, Bo, m, n):
    """Value of mean_mask |Bo - B(M S)| for one view, differentiable in rp
    ([H,W,3] torch float64), with the selection S held fixed."""
    import torch.nn.functional as Fn
    g = (GREY[0] * rp[..., 0] + GREY[1] * rp[..., 1]) + GREY[2] * rp[..., 2]

    def corr(x, w):
        r = w.shape[0] // 2
        xp = Fn.pad(x[None, None], (r, r, r, r), mode="replicate")
        return Fn.conv2d(xp, torch.as_tensor(w)[None, None])[0, 0]

    s = corr(g, gaussian_kernel(SMOOTH_SIZE, SMOOTH_SIGMA))
    gx, gy = corr(s, SOBEL_X), corr(s, SOBEL_Y)
    M = torch.sqrt(gx * gx + gy * gy + EPS)
    B = corr(M * torch.as_tensor(S, dtype=torch.float64), gaussian_kernel(BLUR_SIZE, BLUR_SIGMA))
    return (torch.abs(torch.as_tensor(Bo) - B) * torch.as_tensor(m, dtype=torch.float64)).sum() / n


def data_term(render, T, target, target_edges, mask, wh, pix_off, view_hand, n_hands, w_e=1.0, low=LOW,
              high=HIGH):
    """E1 per hand of Eq. 3 with f1 = D_c + w_e D_e (Eq. 4) and its gradients.

    render R [P,3] (what the renderer returns), T [n_views,9], target O [P,3],
    target_edges B(Canny(O)) [P], mask [P] (None = all pixels).  Returns
    (loss [n_hands], dE/dR [P,3], dE/dT [n_views,9], r' = T R [P,3],
    B(Canny(r')) [P], selection [P] bool)."""
    R = np.asarray(render, np.float64)
    T = np.asarray(T, np.float64).reshape(-1, 9)
    O = np.asarray(target, np.float64)
    Be = np.asarray(target_edges, np.float64)
    P = R.shape[0]
    mask = np.ones(P, bool) if mask is None else np.asarray(mask).reshape(-1) != 0
    rp = colour_transform(R, T, pix_off)
    loss = np.zeros(n_hands)
    g_rp = np.zeros_like(rp)
    b_r = np.zeros(P)
    sel = np.zeros(P, bool)
    for v, sl, img in _views(rp, wh, pix_off, 3):
        W, H = int(wh[v][0]), int(wh[v][1])
        m = mask[sl]
        n = int(m.sum())
        gx, gy, M = gradients(grey(img))
        S = select(gx, gy, M, low, high)
        sel[sl] = S.reshape(-1)
        b_r[sl] = correlate(np.where(S, M, 0.0), gaussian_kernel(BLUR_SIZE, BLUR_SIGMA)).reshape(-1)
        if n == 0:
            continue
        d = rp[sl] - O[sl]
        loss[view_hand[v]] += np.abs(d[m]).sum() / (3.0 * n)
        g = np.zeros_like(d)
        g[m] = np.sign(d[m]) / (3.0 * n)
        rt = torch.tensor(img, dtype=torch.float64, requires_grad=True)
        e = _edge_term_torch(rt, S, Be[sl].reshape(H, W), m.reshape(H, W), n)
        (w_e * e).backward()
        loss[view_hand[v]] += w_e * float(e.detach())
        g_rp[sl] = g + rt.grad.numpy().reshape(-1, 3)
    # through r' = T R
    g_R = np.zeros_like(R)
    g_T = np.zeros((len(pix_off) - 1, 9))
    for v in range(len(pix_off) - 1):
        sl = slice(int(pix_off[v]), int(pix_off[v + 1]))
        Tv = T[v].reshape(3, 3)
        g_R[sl] = g_rp[sl] @ Tv
        g_T[v] = (g_rp[sl].T @ R[sl]).reshape(-1)
    return loss, g_R, g_T, rp, b_r, sel


# --------------------------------------------------------------------------
# two-level colour map
# --------------------------------------------------------------------------

def compose_albedo(low, high):
    """V = V_high + V_low nearest-upsampled: low [H,L,L,3], high [H,th,tw,3]
    (th, tw multiples of L)."""
    low = np.asarray(low, np.float64)
    high = np.asarray(high, np.float64)
    L, th, tw = low.shape[1], high.shape[1], high.shape[2]
    up = np.repeat(np.repeat(low, th // L, axis=1), tw // L, axis=2)
    return high + up


def albedo_low_grad(grad_albedo, L):
    """dE/dV_low from dE/dV: the sum over each low texel's block."""
    g = np.asarray(grad_albedo, np.float64)
    Hh, th, tw = g.shape[0], g.shape[1], g.shape[2]
    return g.reshape(Hh, L, th // L, L, tw // L, 3).sum(axis=(2, 4))
