"""The procedural hand: exact sizes, a manifold disk with one 16-edge wrist
opening, consistent outward winding, valid skinning tables."""
import numpy as np

from paper_2107_05509_amd import scene


def test_counts(hand_model):
    m = hand_model
    assert m.n_verts == 778 and m.n_faces == 1538 and m.n_edges == 2315
    assert m.shapedirs.shape == (778, 3, 10)
    assert m.j_regressor.shape == (16, 778) and m.weights.shape == (778, 16)


def test_manifold_disk(hand_model):
    m = hand_model
    directed = {}
    for f, t in enumerate(m.faces):
        assert len(set(t.tolist())) == 3
        for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
            assert (a, b) not in directed, "directed edge used twice: inconsistent winding"
            directed[(a, b)] = f
    boundary = [(a, b) for (a, b) in directed if (b, a) not in directed]
    assert len(boundary) == 16
    # the boundary edges form a single closed loop
    nxt = dict(boundary)
    start = boundary[0][0]
    cur, n = start, 0
    while True:
        cur = nxt[cur]
        n += 1
        if cur == start:
            break
    assert n == 16
    # Euler characteristic of a disk
    assert m.n_verts - m.n_edges + m.n_faces == 1
    # every vertex is used and the surface is connected
    used = np.zeros(m.n_verts, bool)
    used[m.faces.ravel()] = True
    assert used.all()
    adj = [[] for _ in range(m.n_verts)]
    for a, b in m.edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    assert len(seen) == m.n_verts


def test_edge_tables(hand_model):
    m = hand_model
    for e, ((a, b), (f0, f1)) in enumerate(zip(m.edges, m.edge_faces)):
        t = m.faces[f0].tolist()
        k = t.index(a)
        assert t[(k + 1) % 3] == b  # (a,b) follows f0's winding
        if f1 >= 0:
            t = m.faces[f1].tolist()
            k = t.index(b)
            assert t[(k + 1) % 3] == a
    assert (m.edge_faces[:, 1] < 0).sum() == 16
    # CSR vertex -> faces
    for v in range(0, m.n_verts, 7):
        fs = m.vf_faces[m.vf_offsets[v]:m.vf_offsets[v + 1]]
        assert set(fs.tolist()) == set(np.nonzero((m.faces == v).any(1))[0].tolist())


def test_outward_winding(hand_model):
    m = hand_model
    v = m.v_template
    f = m.faces
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    # the signed volume enclosed (the wrist opening is small) is positive
    vol = np.einsum("ij,ij->i", v[f[:, 0]], n).sum() / 6.0
    assert vol > 0
    assert vol > 1e-4  # > 100 cm^3: a hand-sized solid


def test_rig_tables(hand_model):
    m = hand_model
    assert np.allclose(m.weights.sum(1), 1.0)
    assert ((m.weights > 0).sum(1) <= 4).all()
    assert (m.weights >= 0).all()
    assert np.allclose(m.j_regressor.sum(1), 1.0)
    assert m.parents[0] == -1 and all(0 <= m.parents[j] < j for j in range(1, 16))
    assert (m.uv >= 0).all() and (m.uv <= 1).all()
    # shape directions: 2 mm RMS per unit coefficient
    rms = np.sqrt((m.shapedirs ** 2).sum(1).mean(0))
    assert np.allclose(rms, 0.002)


def test_seeded_workloads_are_reproducible():
    a = scene.workload_tiny(3)
    b = scene.workload_tiny(3)
    assert np.array_equal(a.params_init, b.params_init)
    assert np.array_equal(a.backgrounds[0], b.backgrounds[0])
    c = scene.camera_arrays(a.cams)
    assert c["R"].dtype == np.float32 and c["pix_off"][-1] == 4 * 64 * 64
    for cam in a.cams:
        R = cam.R
        assert np.allclose(R @ R.T, np.eye(3)) and np.isclose(np.linalg.det(R), 1.0)
        # the camera looks at the origin
        assert np.allclose(R[2], -cam.o / np.linalg.norm(cam.o))
