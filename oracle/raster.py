"""Reference hard rasteriser (TEST INFRASTRUCTURE ONLY: imported by tests/
and the benchmark's comparison study through the oracle, never by the product
path).

The paper compares its ray tracer with hard rasterisation (Section 4.2.2,
"Ray tracing vs rasterization": the hard variant of a widely used
rasteriser, equivalent to Neural Rendering, chosen because near the solution
soft rasterisation is scheduled down to it).  Hard rasterisation takes one
point per pixel, the pixel centre, and colours it by the nearest triangle
covering that point; its derivative flows through the covering triangle's
barycentric interpolation only: visibility (which triangle covers a pixel)
is piecewise constant and contributes nothing.

Readings (the paper fixes none of these details):
* pixel (i, j) is sampled at its centre (j + 1/2, i + 1/2); no anti-aliasing;
* a triangle covers the centre p when its three edge functions
  E(a, b, p) = (b.x - a.x)(p.y - a.y) - (b.y - a.y)(p.x - a.x), taken for the
  edges (v1, v2), (v2, v0), (v0, v1) of the projected vertices, are all >= 0
  or all <= 0 and their sum is not zero (no back-face culling; a centre on a
  shared edge is covered by both triangles);
* triangles with a vertex less than 1 mm in front of the camera are dropped;
* depth: 1/z at p interpolated with the screen-space barycentrics
  E_k / (E_0 + E_1 + E_2) (perspective-correct); the nearest triangle is the
  one with the largest 1/z rounded to float32, ties going to the smaller
  triangle index;
* projection, edge functions and 1/z in float64 from the float32 vertices
  with a fixed operation order (the device evaluates the same expressions);
* the covering triangle's surface point is where the ray through the pixel
  centre meets its plane (the perspective-correct barycentrics), shaded as by
  the ray tracer: albedo(uv) (bilinear, texel centres at (j + 1/2)/W, clamp to
  edge) times ka + kd max(0, n.l) with the interpolated, renormalised vertex
  normal; pixels no triangle covers take the background.
"""
from __future__ import annotations

import numpy as np
import torch

NEAR = 1e-3


def project(v32, R, o, fx, fy, cx, cy):
    """Screen coordinates and camera depth of float32 vertices [V,3], in
    float64: q = v - o, camera x = (R0 q0 + R1 q1) + R2 q2 (rows of R), then
    (fx x) / z + cx."""
    q = v32.astype(np.float64) - np.asarray(o, np.float32).astype(np.float64)
    Rm = np.asarray(R, np.float32).astype(np.float64).reshape(3, 3)
    cam = [(Rm[r, 0] * q[:, 0] + Rm[r, 1] * q[:, 1]) + Rm[r, 2] * q[:, 2] for r in range(3)]
    x, y, z = cam
    fx, fy, cx, cy = (float(np.float32(t)) for t in (fx, fy, cx, cy))
    return (fx * x) / z + cx, (fy * y) / z + cy, z


def edge(ax, ay, bx, by, px, py):
    """E(a, b, p) = (b.x - a.x)(p.y - a.y) - (b.y - a.y)(p.x - a.x)."""
    return (bx - ax) * (py - ay) - (by - ay) * (px - ax)


def raster_view(v32, faces, R, o, intr, W, H, want_zinv=False):
    """Covering triangle of every pixel centre of one view: face [H,W] int32
    (-1: none), and (optionally) the winning 1/z (float64; 0 where none)."""
    px, py, z = project(v32, R, o, *intr)
    kz = np.zeros((H, W), np.uint32)          # float32 bits of 1/z; 0 = empty
    face = np.full((H, W), -1, np.int32)
    zinv_out = np.zeros((H, W), np.float64)
    for f, (i0, i1, i2) in enumerate(np.asarray(faces)):
        if min(z[i0], z[i1], z[i2]) <= NEAR:
            continue
        xs, ys = (px[i0], px[i1], px[i2]), (py[i0], py[i1], py[i2])
        j0 = max(0, int(np.floor(min(xs) - 0.5)))
        j1 = min(W - 1, int(np.ceil(max(xs) - 0.5)))
        r0 = max(0, int(np.floor(min(ys) - 0.5)))
        r1 = min(H - 1, int(np.ceil(max(ys) - 0.5)))
        if j0 > j1 or r0 > r1:
            continue
        cx = np.arange(j0, j1 + 1, dtype=np.float64)[None, :] + 0.5
        cy = np.arange(r0, r1 + 1, dtype=np.float64)[:, None] + 0.5
        e0 = edge(px[i1], py[i1], px[i2], py[i2], cx, cy)
        e1 = edge(px[i2], py[i2], px[i0], py[i0], cx, cy)
        e2 = edge(px[i0], py[i0], px[i1], py[i1], cx, cy)
        area = (e0 + e1) + e2
        inside = (((e0 >= 0) & (e1 >= 0) & (e2 >= 0)) | ((e0 <= 0) & (e1 <= 0) & (e2 <= 0))) & (area != 0)
        if not inside.any():
            continue
        with np.errstate(divide="ignore", invalid="ignore"):
            zinv = ((e0 / z[i0] + e1 / z[i1]) + e2 / z[i2]) / area
        k = zinv.astype(np.float32).view(np.uint32)
        sub_k = kz[r0:r1 + 1, j0:j1 + 1]
        sub_f = face[r0:r1 + 1, j0:j1 + 1]
        better = inside & ((k > sub_k) | ((k == sub_k) & ((sub_f < 0) | (f < sub_f))))
        sub_k[better] = k[better]
        sub_f[better] = f
        zinv_out[r0:r1 + 1, j0:j1 + 1][better] = zinv[better]
    return (face, zinv_out) if want_zinv else face


def raster_faces(v32, faces, tab):
    """Covering triangle of every pixel of the packed views [P] int32 (-1:
    background).  v32 [n_hands,V,3] float32; tab: the camera arrays."""
    out = []
    for vi in range(len(tab["wh"])):
        W, H = (int(t) for t in tab["wh"][vi])
        h = int(tab["hand"][vi])
        out.append(raster_view(np.asarray(v32[h], np.float32), faces, tab["R"][vi], tab["o"][vi], tab["intr"][vi],
                               W, H).reshape(-1))
    return np.concatenate(out)


def _tex(albedo, u, v):
    """Bilinear lookup, texel centres at (j + 1/2)/W, clamp to edge; albedo
    [th,tw,3] torch, u, v torch [n]."""
    th, tw = albedo.shape[:2]
    x = u * tw - 0.5
    y = v * th - 0.5
    fx0, fy0 = torch.floor(x), torch.floor(y)
    ax, ay = (x - fx0)[:, None], (y - fy0)[:, None]
    j0, i0 = fx0.long(), fy0.long()
    j1, i1 = (j0 + 1).clamp(0, tw - 1), (i0 + 1).clamp(0, th - 1)
    j0, i0 = j0.clamp(0, tw - 1), i0.clamp(0, th - 1)
    a00, a01, a10, a11 = albedo[i0, j0], albedo[i0, j1], albedo[i1, j0], albedo[i1, j1]
    return (1 - ax) * (1 - ay) * a00 + ax * (1 - ay) * a01 + (1 - ax) * ay * a10 + ax * ay * a11


def raster_image(verts, normals, uv, albedo, background, faces, tab, shading, face_pp):
    """The image [P,3] (torch float64) of the given covering triangles
    face_pp [P]: differentiable in verts [n_hands,V,3], normals [n_hands,V,3]
    and albedo [n_hands,th,tw,3] (all torch float64) with the coverage held
    fixed."""
    ka, kd = float(np.float32(shading[0])), float(np.float32(shading[1]))
    light = torch.tensor([float(np.float32(c)) for c in shading[2:5]], dtype=torch.float64)
    uv = torch.as_tensor(np.asarray(uv, np.float64))
    fc = torch.as_tensor(np.asarray(faces, np.int64))
    bg = torch.as_tensor(np.asarray(background, np.float64))
    rows = []
    for vi in range(len(tab["wh"])):
        W, H = (int(t) for t in tab["wh"][vi])
        p0, p1 = int(tab["pix_off"][vi]), int(tab["pix_off"][vi + 1])
        h = int(tab["hand"][vi])
        f = torch.as_tensor(np.asarray(face_pp[p0:p1], np.int64))
        out = bg[p0:p1].clone()
        sel = torch.nonzero(f >= 0).squeeze(1)
        if len(sel):
            R = torch.as_tensor(np.asarray(tab["R"][vi], np.float32).astype(np.float64)).reshape(3, 3)
            o = torch.as_tensor(np.asarray(tab["o"][vi], np.float32).astype(np.float64))
            fx, fy, cx, cy = (float(np.float32(t)) for t in tab["intr"][vi])
            X = (sel % W).double() + 0.5
            Y = torch.div(sel, W, rounding_mode="floor").double() + 0.5
            # ray through the pixel centre: d = R^T ((X - cx)/fx, (Y - cy)/fy, 1)
            dc = torch.stack([(X - cx) / fx, (Y - cy) / fy, torch.ones_like(X)], 1)
            d = dc @ R
            tri = fc[f[sel]]
            v = verts[h]
            v0, v1, v2 = v[tri[:, 0]], v[tri[:, 1]], v[tri[:, 2]]
            e1, e2 = v1 - v0, v2 - v0
            pp = torch.cross(d, e2, dim=1)
            det = (e1 * pp).sum(1)
            s = o[None, :] - v0
            q = torch.cross(s, e1, dim=1)
            b1 = (s * pp).sum(1) / det
            b2 = (d * q).sum(1) / det
            b0 = 1.0 - b1 - b2
            bb = torch.stack([b0, b1, b2], 1)
            uvp = (bb[:, :, None] * uv[tri]).sum(1)
            n = (bb[:, :, None] * normals[h][tri]).sum(1)
            n = n / torch.sqrt((n * n).sum(1, keepdim=True))
            shade = ka + kd * torch.clamp((n * light).sum(1), min=0.0)
            col = _tex(albedo[h], uvp[:, 0], uvp[:, 1]) * shade[:, None]
            out = out.index_put((sel,), col)
        rows.append(out)
    return torch.cat(rows, 0)
