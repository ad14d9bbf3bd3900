"""Seeded synthetic inputs for multiview hand refinement.

Stands in for the MANO hand model, the InterHand2.6M camera rigs and the HTML
hand textures the paper works with (Section 3, "Geometry" and "Color mapping";
Section 4.2.1 for the synthetic setup).  None of those assets is available, so
this module builds, from a seed:

* a procedural linear-blend-skinned hand: one welded triangle surface with 778
  vertices, 1538 triangles and 2315 edges (a topological disk whose only
  boundary is a 16-edge wrist opening), a 16-joint tree (root + 5 fingers x 3),
  10 smooth shape directions, skinning weights, a joint regressor and per-vertex
  texture coordinates;
* calibrated pinhole cameras on a sphere or a spherical shell, looking at the hand;
* albedo maps made of Gaussian colour blobs, per-pixel uniform backgrounds;
* parameter draws (ground truth and the noisy initial estimate).

It holds none of the method's arithmetic: no skinning, projection, ray tracing or
shading happens here.  Everything is float64 NumPy; callers round to float32.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

N_JOINTS = 16
N_SHAPE = 10
N_PARAMS = 64
# Layout of the 64-float parameter block: 16 joint rotations (axis-angle, joint 0
# is the root), 10 shape coefficients, global rotation (axis-angle), translation.
POSE = slice(0, 48)
SHAPE = slice(48, 58)
ROT = slice(58, 61)
TRANS = slice(61, 64)
FINGER_POSE = slice(3, 48)

N_VERTS = 778
N_FACES = 1538
N_EDGES = 2315
WRIST_EDGES = 16


@dataclass
class HandModel:
    v_template: np.ndarray   # [V,3]
    shapedirs: np.ndarray    # [V,3,K]
    j_regressor: np.ndarray  # [J,V], rows sum to 1
    weights: np.ndarray      # [V,J], rows sum to 1, <=4 non-zeros
    parents: np.ndarray      # [J] int32, parents[0] = -1
    faces: np.ndarray        # [F,3] int32, outward (counter-clockwise) winding
    uv: np.ndarray           # [V,2] in [0,1]
    edges: np.ndarray        # [E,2] int32 (a,b) as directed in edge_faces[:,0]
    edge_faces: np.ndarray   # [E,2] int32, second entry -1 on the boundary
    vf_offsets: np.ndarray   # [V+1] int32 CSR vertex -> incident faces
    vf_faces: np.ndarray     # [3F] int32
    layout2d: np.ndarray = field(repr=False, default=None)  # [V,2] flat layout

    @property
    def n_verts(self):
        return self.v_template.shape[0]

    @property
    def n_faces(self):
        return self.faces.shape[0]

    @property
    def n_edges(self):
        return self.edges.shape[0]


# --------------------------------------------------------------------------
# procedural hand surface
# --------------------------------------------------------------------------

_CM = 0.01


def _seg_dist(p, a, b):
    ab = b - a
    t = np.clip(((p - a) @ ab) / max(ab @ ab, 1e-30), 0.0, 1.0)
    return np.linalg.norm(p - (a + t * ab))


def _build_layout():
    """Flat layout of the hand: palm grid + four finger strips + a thumb strip.

    Returns 2-D points, quads (as 4-tuples of point ids, counter-clockwise),
    per-point part labels and along-axis coordinates, and the ids of the
    wrist-opening points.
    """
    hx = 0.38 * _CM
    ncol = 23
    rows = np.array([0.0, 1.0, 1.8, 2.6, 3.4, 4.2, 6.5, 9.0]) * _CM
    nrow = len(rows)
    pts, part, along = [], [], []

    def add(p, prt, s):
        pts.append(np.asarray(p, dtype=np.float64))
        part.append(prt)
        along.append(s)
        return len(pts) - 1

    palm = np.zeros((ncol, nrow), dtype=np.int64)
    for i in range(ncol):
        for j in range(nrow):
            palm[i, j] = add((i * hx, rows[j]), 0, rows[j] - rows[-1])
    quads = []
    for i in range(ncol - 1):
        for j in range(nrow - 1):
            quads.append((palm[i, j], palm[i + 1, j], palm[i + 1, j + 1], palm[i, j + 1]))

    # fingers 1..4 = pinky, ring, middle, index (thumb is finger 0), attached to
    # 5-point segments of the palm's top row with 2-cell gaps between them.
    starts = [0, 6, 12, 18]
    lengths = np.array([6.2, 7.7, 8.2, 7.5]) * _CM
    nrows_f = [10, 12, 13, 12]
    finger_grids = []
    ytop = rows[-1]
    for k, (s0, L, nr) in enumerate(zip(starts, lengths, nrows_f)):
        g = np.zeros((5, nr + 1), dtype=np.int64)
        prt = 4 - k  # pinky -> 4 ... index -> 1
        for a in range(5):
            g[a, 0] = palm[s0 + a, nrow - 1]
            part[g[a, 0]] = prt
            along[g[a, 0]] = 0.0
        for r in range(1, nr + 1):
            s = L * r / nr
            taper = 1.0 - 0.15 * (r / nr)
            xc = (s0 + 2) * hx
            for a in range(5):
                g[a, r] = add((xc + (a - 2) * hx * taper, ytop + s), prt, s)
        for a in range(4):
            for r in range(nr):
                quads.append((g[a, r], g[a + 1, r], g[a + 1, r + 1], g[a, r + 1]))
        finger_grids.append((prt, g, L, nr))

    # thumb: attached to the palm's right column, rows 1..5, pointing out and up
    nr_t = 10
    L_t = 6.0 * _CM
    dt = np.array([1.0, 0.55])
    dt /= np.linalg.norm(dt)
    pt = np.array([-dt[1], dt[0]])
    gt = np.zeros((5, nr_t + 1), dtype=np.int64)
    for a in range(5):
        gt[a, 0] = palm[ncol - 1, 1 + a]
        part[gt[a, 0]] = 0
        along[gt[a, 0]] = 0.0
    base_c = pts[palm[ncol - 1, 3]]
    for r in range(1, nr_t + 1):
        s = L_t * r / nr_t
        blend = min(r / 3.0, 1.0)
        half = (1.6 + (0.95 - 1.6) * blend) * _CM
        across = (1 - blend) * np.array([0.0, 1.0]) + blend * pt
        across /= np.linalg.norm(across)
        c = base_c + s * dt
        for a in range(5):
            gt[a, r] = add(c + (a - 2) / 2.0 * half * across, 0, s)
    for a in range(4):
        for r in range(nr_t):
            quads.append((gt[a, r], gt[a + 1, r], gt[a + 1, r + 1], gt[a, r + 1]))
    finger_grids.append((0, gt, L_t, nr_t))

    pts = np.array(pts)
    wrist = [palm[i, 0] for i in range(7, 16)]  # 9 points, 8 edges
    return dict(pts=pts, quads=quads, part=np.array(part), along=np.array(along),
                palm=palm, fingers=finger_grids, wrist=wrist, rows=rows, hx=hx)


def _tri_area2(p, a, b, c):
    return (p[b, 0] - p[a, 0]) * (p[c, 1] - p[a, 1]) - (p[b, 1] - p[a, 1]) * (p[c, 0] - p[a, 0])


def _mesh_edges(faces):
    d = {}
    for f, (i0, i1, i2) in enumerate(faces):
        for a, b in ((i0, i1), (i1, i2), (i2, i0)):
            d.setdefault((a, b), []).append(f)
    return d


def build_hand_mesh():
    """Welded hand surface (rest pose, metres) with exactly 778 vertices."""
    L = _build_layout()
    p2 = L["pts"]
    # outline of the flat layout = quad sides used by a single quad
    side_count = {}
    for q in L["quads"]:
        for k in range(4):
            a, b = q[k], q[(k + 1) % 4]
            key = (min(a, b), max(a, b))
            side_count[key] = side_count.get(key, 0) + 1
    outline_pt = np.zeros(len(p2), dtype=bool)
    for (a, b), c in side_count.items():
        if c == 1:
            outline_pt[a] = outline_pt[b] = True
    tris2 = []
    for q in L["quads"]:
        a, b, c, d = q
        # split along the diagonal that does not join two outline points: such a
        # chord would be shared by the front and back sheets (non-manifold)
        if outline_pt[a] and outline_pt[c]:
            t1, t2 = (b, c, d), (b, d, a)
        else:
            t1, t2 = (a, b, c), (a, c, d)
        if _tri_area2(p2, *t1) < 0:
            t1, t2 = t1[::-1], t2[::-1]
        tris2.extend([t1, t2])
    tris2 = np.array(tris2, dtype=np.int64)
    for t in tris2:
        assert _tri_area2(p2, *t) > 0, "folded layout"
    # outline of the flat layout
    ecount = {}
    for t in tris2:
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            key = (min(a, b), max(a, b))
            ecount[key] = ecount.get(key, 0) + 1
    outline_edges = [k for k, c in ecount.items() if c == 1]
    wrist = L["wrist"]
    wrist_set = {(min(a, b), max(a, b)) for a, b in zip(wrist[:-1], wrist[1:])}
    closed_outline = [e for e in outline_edges if e not in wrist_set]
    on_outline = np.zeros(len(p2), dtype=bool)
    for a, b in outline_edges:
        on_outline[a] = on_outline[b] = True
    wrist_inner = set(wrist[1:-1])
    # distance of every layout point to the closed outline -> thickness
    seg_a = np.array([p2[a] for a, b in closed_outline])
    seg_b = np.array([p2[b] for a, b in closed_outline])
    radius = np.where(L["part"] == 0, 0.95, 0.78) * _CM
    radius = np.where(L["part"] == 4, 0.66 * _CM, radius)
    palm_pts = set(L["palm"].ravel().tolist())
    radius = np.array([
        1.15 * _CM if (i in palm_pts and L["along"][i] < -1e-9) else radius[i]
        for i in range(len(p2))])
    for i in wrist_inner:
        radius[i] = 1.15 * _CM

    def thickness(i):
        d = min(_seg_dist(p2[i], a, b) for a, b in zip(seg_a, seg_b))
        r = radius[i]
        x = min(d / r, 1.0)
        return r * np.sqrt(max(0.0, 1.0 - (1.0 - x) ** 2))

    single = on_outline.copy()
    for i in wrist_inner:
        single[i] = False
    front = np.full(len(p2), -1, dtype=np.int64)
    back = np.full(len(p2), -1, dtype=np.int64)
    verts, src = [], []
    for i in range(len(p2)):
        if single[i]:
            front[i] = back[i] = len(verts)
            verts.append((p2[i, 0], p2[i, 1], 0.0))
            src.append(i)
        else:
            t = thickness(i)
            front[i] = len(verts)
            verts.append((p2[i, 0], p2[i, 1], t))
            src.append(i)
            back[i] = len(verts)
            verts.append((p2[i, 0], p2[i, 1], -t))
            src.append(i)
    faces = [(front[a], front[b], front[c]) for a, b, c in tris2]
    faces += [(back[a], back[c], back[b]) for a, b, c in tris2]
    verts = np.array(verts, dtype=np.float64)
    faces = np.array(faces, dtype=np.int64)
    src = np.array(src, dtype=np.int64)

    # refine to exactly N_VERTS by splitting the longest interior edges
    while len(verts) < N_VERTS:
        emap = _mesh_edges(faces)
        best, best_len = None, -1.0
        for (a, b), fl in emap.items():
            if a < b and (b, a) in emap:
                ln = np.linalg.norm(verts[a] - verts[b])
                if ln > best_len:
                    best, best_len = (a, b), ln
        a, b = best
        f0 = emap[(a, b)][0]
        f1 = emap[(b, a)][0]
        m = len(verts)
        verts = np.vstack([verts, 0.5 * (verts[a] + verts[b])])
        src = np.append(src, -1)
        new = []
        for f in range(len(faces)):
            if f in (f0, f1):
                continue
            new.append(faces[f])
        for f, (u, v) in ((f0, (a, b)), (f1, (b, a))):
            tri = list(faces[f])
            k = tri.index(u)
            w = tri[(k + 2) % 3]
            assert tri[(k + 1) % 3] == v
            new.append((u, m, w))
            new.append((m, v, w))
        faces = np.array(new, dtype=np.int64)
    assert len(verts) == N_VERTS, len(verts)
    return verts, faces, src, L


def _edge_tables(faces, n_verts):
    emap = _mesh_edges(faces)
    edges, efaces = [], []
    for (a, b), fl in sorted(emap.items(), key=lambda kv: kv[1][0]):
        if (b, a) in emap and a > b:
            continue  # listed from the other direction
        f0 = fl[0]
        f1 = emap[(b, a)][0] if (b, a) in emap else -1
        edges.append((a, b))
        efaces.append((f0, f1))
    inc = [[] for _ in range(n_verts)]
    for f, tri in enumerate(faces):
        for v in tri:
            inc[v].append(f)
    offs = np.zeros(n_verts + 1, dtype=np.int32)
    offs[1:] = np.cumsum([len(x) for x in inc])
    flat = np.array([f for x in inc for f in x], dtype=np.int32)
    return (np.array(edges, dtype=np.int32), np.array(efaces, dtype=np.int32), offs, flat)


def _smoothstep(x):
    x = np.clip(x, 0.0, 1.0)
    return x * x * (3.0 - 2.0 * x)


def make_hand_model(seed: int = 0) -> HandModel:
    """The procedural hand.  The surface and rig are fixed; `seed` draws the
    10 shape directions."""
    verts, faces, src, L = build_hand_mesh()
    V = len(verts)
    p2 = L["pts"]
    # 2-D layout position of every vertex (split vertices: midpoint of their edge)
    lay = np.zeros((V, 2))
    for i in range(V):
        lay[i] = p2[src[i]] if src[i] >= 0 else verts[i, :2]
    part_v = np.full(V, -1, dtype=np.int64)
    along_v = np.zeros(V)
    for i in range(V):
        if src[i] >= 0:
            part_v[i] = L["part"][src[i]]
            along_v[i] = L["along"][src[i]]
    # split vertices inherit from the nearest original vertex
    for i in range(V):
        if src[i] < 0:
            d = np.linalg.norm(verts[: len(src)] - verts[i], axis=1)
            d[src < 0] = np.inf
            j = int(np.argmin(d))
            part_v[i], along_v[i] = part_v[j], along_v[j]

    # joints: 0 root; finger f in 0..4 (thumb..pinky) owns joints 1+3f..3+3f
    parents = np.full(N_JOINTS, -1, dtype=np.int32)
    for f in range(5):
        parents[1 + 3 * f] = 0
        parents[2 + 3 * f] = 1 + 3 * f
        parents[3 + 3 * f] = 2 + 3 * f
    joint_s = {}
    ring_of = {}
    palm = L["palm"]
    for prt, g, Lf, nr in L["fingers"]:
        r1 = int(round(0.45 * nr))
        r2 = int(round(0.75 * nr))
        joint_s[prt] = (0.0, Lf * r1 / nr, Lf * r2 / nr)
        ring_of[prt] = (g[:, 0], g[:, r1], g[:, r2])
    # regressor: each joint is the mean of a cross-section ring of vertices
    src_to_verts = {}
    for i in range(V):
        if src[i] >= 0:
            src_to_verts.setdefault(int(src[i]), []).append(i)
    jreg = np.zeros((N_JOINTS, V))
    root_ring = [v for p in palm[:, 1] for v in src_to_verts[int(p)]]
    jreg[0, root_ring] = 1.0 / len(root_ring)
    for prt in range(5):
        for k in range(3):
            ring = [v for p in ring_of[prt][k] for v in src_to_verts[int(p)]]
            jreg[1 + 3 * prt + k, ring] = 1.0 / len(ring)
    # skinning weights: rigid segments blended across +-band around each joint
    band = 0.45 * _CM
    W = np.zeros((V, N_JOINTS))
    for i in range(V):
        prt = part_v[i]
        s = along_v[i]
        if s < 0 or (prt == 0 and src[i] >= 0 and int(src[i]) in set(palm.ravel().tolist())
                     and s == 0 and False):
            W[i, 0] = 1.0
            continue
        js = joint_s[prt]
        chain = [0, 1 + 3 * prt, 2 + 3 * prt, 3 + 3 * prt]
        w = np.zeros(4)
        w[0] = 1.0
        for k in range(3):
            c = _smoothstep((s - js[k] + band) / (2 * band))
            # move weight c from the parent segment to the child segment
            w[k + 1] = c * w[k]
            w[k] = (1 - c) * w[k]
        for k in range(4):
            W[i, chain[k]] += w[k]
    # palm vertices that are not on a finger/thumb axis stay on the root
    for i in range(V):
        if part_v[i] >= 0 and along_v[i] < 0:
            W[i] = 0.0
            W[i, 0] = 1.0
    W /= W.sum(axis=1, keepdims=True)

    # centre the template on its bounding-box centre
    c = 0.5 * (verts.min(axis=0) + verts.max(axis=0))
    verts = verts - c
    # shape directions: smooth random fields, 2 mm RMS per unit coefficient
    rng = np.random.default_rng(np.random.SeedSequence([seed, 0x5EED]))
    sigma = 1.0 * _CM
    d2 = ((verts[:, None, :] - verts[None, :, :]) ** 2).sum(-1)
    K = np.exp(-d2 / (2 * sigma * sigma))
    K /= K.sum(axis=1, keepdims=True)
    raw = rng.standard_normal((N_SHAPE, V, 3))
    sd = np.einsum("ij,kjc->kic", K, raw)
    for k in range(N_SHAPE):
        sd[k] *= 0.002 / np.sqrt((sd[k] ** 2).sum(-1).mean())
    shapedirs = np.ascontiguousarray(np.transpose(sd, (1, 2, 0)))  # [V,3,K]

    # texture coordinates: the flat layout, scaled into the unit square
    lo = lay.min(axis=0)
    ext = (lay.max(axis=0) - lo).max() * 1.04
    uv = (lay - lo) / ext + 0.02
    uv = np.clip(uv, 0.0, 1.0)

    edges, efaces, offs, flat = _edge_tables(faces, V)
    # the model's real arrays hold float32 values (kept as float64 arrays), so
    # that every consumer, float32 or float64, reads exactly the same numbers
    f32v = lambda a: np.asarray(a, np.float32).astype(np.float64)
    return HandModel(v_template=f32v(verts), shapedirs=f32v(shapedirs), j_regressor=f32v(jreg), weights=f32v(W),
                     parents=parents, faces=faces.astype(np.int32), uv=f32v(uv), edges=edges,
                     edge_faces=efaces, vf_offsets=offs, vf_faces=flat, layout2d=lay)


# --------------------------------------------------------------------------
# cameras, appearance, parameters
# --------------------------------------------------------------------------

@dataclass
class Camera:
    R: np.ndarray    # [3,3] world -> camera rotation (rows: right, down, forward)
    o: np.ndarray    # [3] camera centre in world coordinates
    fx: float
    fy: float
    cx: float
    cy: float
    W: int
    H: int
    hand: int = 0


def look_at(o, target=(0.0, 0.0, 0.0)):
    """Rotation whose third row points from o to target, second row 'down'."""
    o = np.asarray(o, dtype=np.float64)
    z = np.asarray(target, dtype=np.float64) - o
    z /= np.linalg.norm(z)
    down = np.array([0.0, 1.0, 0.0])
    if abs(z @ down) > 0.95:
        down = np.array([0.0, 0.0, 1.0])
    y = down - (down @ z) * z
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    return np.stack([x, y, z])


def camera_rig(n_views, W, H, f, radius, rng, hand=0, target=(0.0, 0.0, 0.0)):
    """Cameras with uniformly random directions on a sphere (radius a float) or a
    shell (radius a (lo, hi) pair), all looking at `target`."""
    cams = []
    for _ in range(n_views):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = radius if np.isscalar(radius) else rng.uniform(radius[0], radius[1])
        o = np.asarray(target) + r * d
        cams.append(Camera(R=look_at(o, target), o=o, fx=float(f), fy=float(f),
                           cx=W / 2.0, cy=H / 2.0, W=int(W), H=int(H), hand=hand))
    return cams


def blob_albedo(th, tw, rng, n_blobs=20, base=(0.8, 0.6, 0.5)):
    """Skin-toned base colour plus Gaussian colour blobs, clamped to [0,1]; [th,tw,3]."""
    yy, xx = np.meshgrid((np.arange(th) + 0.5) / th, (np.arange(tw) + 0.5) / tw, indexing="ij")
    img = np.broadcast_to(np.asarray(base, dtype=np.float64), (th, tw, 3)).copy()
    for _ in range(n_blobs):
        cx, cy = rng.uniform(0, 1, 2)
        s = rng.uniform(0.03, 0.15)
        col = rng.uniform(0, 1, 3)
        g = np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))
        img += g[..., None] * (col - np.asarray(base)) * 0.8
    return np.clip(img, 0.0, 1.0)


def uniform_background(H, W, rng):
    return rng.uniform(0.0, 1.0, (H, W, 3))


def random_rotvec(rng):
    """Axis-angle of a uniformly distributed rotation."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    ang = 2 * np.arccos(np.clip(q[0], -1, 1))
    ax = q[1:]
    n = np.linalg.norm(ax)
    return np.zeros(3) if n < 1e-12 else ax / n * ang


def true_params(rng, pose_sigma=0.3, shape=True, global_rot=True):
    p = np.zeros(N_PARAMS)
    p[FINGER_POSE] = rng.normal(0.0, pose_sigma, 45)
    if shape:
        p[SHAPE] = rng.standard_normal(N_SHAPE)
    if global_rot:
        p[ROT] = random_rotvec(rng)
    return p


def perturb_params(p, rng, pose_sigma=0.1, trans_mm=5.0, shape_sigma=0.0):
    q = p.copy()
    q[FINGER_POSE] += rng.normal(0.0, pose_sigma, 45)
    d = rng.standard_normal(3)
    q[TRANS] += trans_mm * 1e-3 * d / np.linalg.norm(d)
    if shape_sigma > 0:
        q[SHAPE] += rng.normal(0.0, shape_sigma, N_SHAPE)
    return q


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    model: HandModel
    cams: list            # list[Camera]
    n_hands: int
    params_true: np.ndarray   # [n_hands,64]
    params_init: np.ndarray   # [n_hands,64]
    albedo_true: np.ndarray   # [n_hands,th,tw,3]
    albedo_init: np.ndarray   # [n_hands,th,tw,3]
    backgrounds: list         # per view [H,W,3]
    spp: int
    iters: int
    seed: int

    @property
    def n_pixels(self):
        return sum(c.W * c.H for c in self.cams)

    def pixel_offsets(self):
        off = np.zeros(len(self.cams) + 1, dtype=np.int64)
        off[1:] = np.cumsum([c.W * c.H for c in self.cams])
        return off

    def packed_background(self):
        return np.concatenate([b.reshape(-1, 3) for b in self.backgrounds], axis=0)


def _rng(seed, tag):
    return np.random.default_rng(np.random.SeedSequence([seed, tag]))


def workload_tiny(seed=0):
    """4 views 64x64, f=80 on a 0.6 m sphere, 64x64 albedo, 4 spp, 10 iterations."""
    model = make_hand_model(0)
    r = _rng(seed, 1)
    pt = true_params(r, 0.3, shape=False, global_rot=False)
    pi = perturb_params(pt, r, 0.1, 5.0)
    alb = blob_albedo(64, 64, _rng(seed, 2))
    cams = camera_rig(4, 64, 64, 80.0, 0.6, _rng(seed, 3))
    bgr = _rng(seed, 4)
    bgs = [uniform_background(c.H, c.W, bgr) for c in cams]
    return Workload("tiny 4x64x64 4spp", model, cams, 1, pt[None], pi[None], alb[None], alb[None].copy(),
                    bgs, 4, 10, seed)


def workload_realistic(seed=0, n_views=8, W=334, H=512, f=700.0, tex=512, spp=16, iters=200):
    """8 views 334x512, f=700 on a 0.6-0.9 m shell, 512x512 albedo, 16 spp."""
    model = make_hand_model(0)
    r = _rng(seed, 11)
    pt = true_params(r, 0.3, shape=True, global_rot=True)
    pi = perturb_params(pt, r, 0.1, 5.0)
    alb = blob_albedo(tex, tex, _rng(seed, 12))
    cams = camera_rig(n_views, W, H, f, (0.6, 0.9), _rng(seed, 13))
    bgr = _rng(seed, 14)
    bgs = [uniform_background(c.H, c.W, bgr) for c in cams]
    init_alb = np.full_like(alb, 0.5)
    return Workload(f"realistic {n_views}x{W}x{H} {spp}spp", model, cams, 1, pt[None], pi[None],
                    alb[None], init_alb[None], bgs, spp, iters, seed)


def workload_dense(seed=0):
    """40 views 334x512, 4 spp, 1024x1024 albedo."""
    w = workload_realistic(seed, n_views=40, tex=1024, spp=4, iters=200)
    w.name = "dense 40x334x512 4spp"
    return w


def workload_batched(seed=0, n_hands=64, spp=8):
    """64 hands, views per hand uniform in [4,40], resolutions from
    {128x128, 256x256, 334x512} (f scaled with the width)."""
    model = make_hand_model(0)
    r = _rng(seed, 21)
    res = [(128, 128), (256, 256), (334, 512)]
    cams, pts, pis, albs, bgs = [], [], [], [], []
    bgr = _rng(seed, 24)
    for h in range(n_hands):
        pt = true_params(r, 0.3, shape=True, global_rot=True)
        pts.append(pt)
        pis.append(perturb_params(pt, r, 0.1, 5.0))
        albs.append(blob_albedo(256, 256, _rng(seed * 1000 + h, 22)))
        nv = int(r.integers(4, 41))
        W, H = res[int(r.integers(0, 3))]
        hc = camera_rig(nv, W, H, 700.0 * W / 334.0, (0.6, 0.9), _rng(seed * 1000 + h, 23), hand=h)
        cams.extend(hc)
        bgs.extend(uniform_background(c.H, c.W, bgr) for c in hc)
    albs = np.array(albs)
    return Workload(f"batched {n_hands} hands {spp}spp", model, cams, n_hands, np.array(pts),
                    np.array(pis), albs, np.full_like(albs, 0.5), bgs, spp, 200, seed)


def workload_mixed(seed=0, spp=4):
    """A small batch for parity against the oracle: 3 hands with 3, 1 and 2
    views of 64x64, 48x32 and 96x64 pixels (f = 80 W / 64, 0.6 m sphere),
    the hands' views interleaved in the camera list, 64x64 albedo, 4 spp."""
    model = make_hand_model(0)
    r = _rng(seed, 31)
    layout = [(0, 64, 64), (2, 96, 64), (0, 64, 64), (1, 48, 32), (2, 96, 64), (0, 64, 64)]
    pts = [true_params(r, 0.3, shape=True, global_rot=True) for _ in range(3)]
    pis = [perturb_params(p, r, 0.1, 5.0) for p in pts]
    albs = np.array([blob_albedo(64, 64, _rng(seed * 1000 + h, 32)) for h in range(3)])
    cams = []
    for k, (h, W, H) in enumerate(layout):
        cams.extend(camera_rig(1, W, H, 80.0 * W / 64.0, 0.6, _rng(seed * 1000 + k, 33), hand=h))
    bgr = _rng(seed, 34)
    bgs = [uniform_background(c.H, c.W, bgr) for c in cams]
    return Workload(f"mixed 3 hands {spp}spp", model, cams, 3, np.array(pts), np.array(pis), albs,
                    albs.copy(), bgs, spp, 10, seed)


# --------------------------------------------------------------------------
# shading constants and float32 camera tables (inputs shared by every consumer)
# --------------------------------------------------------------------------

# Lambertian + ambient under one fixed world light; float32-representable.
KA = float(np.float32(0.3))
KD = float(np.float32(0.7))
LIGHT = tuple(float(x) for x in (np.array([1.0, -2.0, -3.0]) / np.sqrt(14.0)).astype(np.float32))
SHADING = (KA, KD) + LIGHT


def camera_arrays(cams):
    """float32/int tables describing a list of cameras (packed-view layout):
    R [n,9] f32 (world->camera, row-major), o [n,3] f32 (centre), intr [n,4] f32
    (fx, fy, cx, cy), wh [n,2] i32, hand [n] i32, pix_off [n+1] i64."""
    n = len(cams)
    R = np.stack([c.R.reshape(9) for c in cams]).astype(np.float32)
    o = np.stack([c.o for c in cams]).astype(np.float32)
    intr = np.array([[c.fx, c.fy, c.cx, c.cy] for c in cams], dtype=np.float32)
    wh = np.array([[c.W, c.H] for c in cams], dtype=np.int32)
    hand = np.array([c.hand for c in cams], dtype=np.int32)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum([c.W * c.H for c in cams])
    return dict(R=R, o=o, intr=intr, wh=wh, hand=hand, pix_off=off)


# --------------------------------------------------------------------------
# initial parameters of the edge-proposal network (seeded; zero output layer,
# so the initial proposal is the length-proportional one)
# --------------------------------------------------------------------------

def mlp_init(seed=0, n_in=16, n_hid=64, out_scale=0.0):
    """Float32 arrays W1 [16,64], b1 [64], W2 [64,64], b2 [64], w3 [64], b3 [1]:
    hidden weights N(0, 1/fan_in), zero biases, output weights N(0, out_scale^2)."""
    r = _rng(seed, 31)
    return {"W1": (r.normal(0, 1, (n_in, n_hid)) / np.sqrt(n_in)).astype(np.float32),
            "b1": np.zeros(n_hid, np.float32),
            "W2": (r.normal(0, 1, (n_hid, n_hid)) / np.sqrt(n_hid)).astype(np.float32),
            "b2": np.zeros(n_hid, np.float32),
            "w3": (r.normal(0, 1, n_hid) * out_scale).astype(np.float32),
            "b3": np.zeros(1, np.float32)}
