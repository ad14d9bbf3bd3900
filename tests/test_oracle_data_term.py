"""Pins of the oracle's full data term (Eq. 3 with f1 = D_c + D_e of Eq. 4;
Section 3.1 "Rendering", "Colour mapping", "Render-and-compare").

- filters against an independent library routine (scipy.ndimage.correlate
  with clamped-to-edge borders) and the Gaussian's closed form;
- Canny on a vertical step edge against a one-dimensional closed form of the
  same smoothing and Sobel weights (magnitude and the selected columns), on
  constant images (nothing selected), under transposition (symmetry);
- the selection's threshold and one-step hysteresis rules on given maps;
- D_e's gradient against central differences at a frozen selection;
- the colour transform's linearity and its gradient by central differences;
- the two-level colour map against numpy's Kronecker product, and the low
  map's gradient as block sums (exact: the map is linear)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import data_term as dt


def test_gaussian_kernel_closed_form():
    for size, sigma in ((5, 1.0), (11, 5.0)):
        w = dt.gaussian_kernel(size, sigma)
        c = size // 2
        i = np.arange(size) - c
        g1 = np.exp(-i * i / (2 * sigma * sigma))
        ref = np.outer(g1, g1) / np.outer(g1, g1).sum()
        assert np.allclose(w, ref, rtol=1e-14, atol=0)
        assert abs(w.sum() - 1.0) < 1e-14 and np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])


@pytest.mark.parametrize("size", [3, 5, 11])
def test_correlate_matches_library(size):
    rng = np.random.default_rng(size)
    x = rng.normal(size=(17, 23))
    w = rng.normal(size=(size, size))
    ref = ndi.correlate(x, w, mode="nearest")
    assert np.allclose(dt.correlate(x, w), ref, rtol=1e-12, atol=1e-12)


def test_blur_of_constant_and_delta():
    K = dt.gaussian_kernel(11, 5.0)
    assert np.allclose(dt.correlate(np.full((30, 31), 0.7), K), 0.7, atol=1e-14)
    d = np.zeros((31, 31))
    d[15, 15] = 1.0
    out = dt.correlate(d, K)
    assert np.allclose(out[10:21, 10:21], K[::-1, ::-1], atol=1e-16)
    assert abs(out.sum() - 1.0) < 1e-13


def test_constant_image_has_no_edges():
    e, S = dt.canny(np.full((24, 20, 3), 0.4))
    assert not S.any() and np.abs(e).max() == 0.0


def _step(H, W, j0, a, b):
    img = np.full((H, W, 3), a)
    img[:, j0:] = b
    return img


@pytest.mark.parametrize("a,b", [(0.1, 0.9), (0.8, 0.05)])
def test_vertical_step_edge(a, b):
    H, W, j0 = 26, 30, 14
    img = _step(H, W, j0, a, b)
    gx, gy, M = dt.gradients(dt.grey(img))
    # 1-D closed form: the 5x5 Gaussian's column marginal smooths the step;
    # Sobel x / 8 is (sum of the column weights 4) / 8 times the central difference
    i = np.arange(5) - 2
    g1 = np.exp(-i * i / 2.0)
    g1 /= g1.sum()
    col = np.array([a if j < j0 else b for j in range(W)], float)
    colp = np.pad(col, 2, mode="edge")
    s = np.array([np.dot(g1, colp[j:j + 5]) for j in range(W)])
    sp = np.pad(s, 1, mode="edge")
    gx1 = 0.5 * (sp[2:] - sp[:-2])
    assert np.allclose(gx, gx1[None, :], atol=1e-13)
    assert np.abs(gy).max() < 1e-13
    assert np.allclose(M, np.sqrt(gx1 * gx1 + 1e-6)[None, :], atol=1e-13)
    e, S = dt.canny(img)
    # the two columns either side of the step carry the largest magnitude
    # (equal up to rounding, so either or both survive the suppression) and
    # are the only ones selected, over the whole height
    cols = np.nonzero(S.any(0))[0].tolist()
    assert cols and set(cols) <= {j0 - 1, j0} and all(S[:, j].all() for j in cols)
    assert np.array_equal(e[:, cols], M[:, cols])


def test_transposed_image_gives_transposed_edges():
    rng = np.random.default_rng(3)
    img = np.zeros((28, 28, 3))
    img[8:20, 6:22] = rng.uniform(0.5, 1.0, 3)
    img[12:16, 10:25] = rng.uniform(0.0, 0.3, 3)
    e, S = dt.canny(img)
    et, St = dt.canny(img.transpose(1, 0, 2))
    assert S.any() and np.array_equal(St, S.T) and np.allclose(et, e.T, atol=1e-14)


def test_selection_thresholds_and_one_step_hysteresis():
    H, W = 9, 9
    gx = np.zeros((H, W)); gy = np.zeros((H, W)); M = np.full((H, W), 0.01)
    # a horizontal-gradient ridge along column 4 (maximal across the row)
    gx[:, 4] = 1.0
    M[:, 4] = [0.25, 0.15, 0.15, 0.05, 0.25, 0.15, 0.12, 0.15, 0.15]
    S = dt.select(gx, gy, M)
    # strong rows 0 and 4 kept; weak rows 1 (next to 0), 3 (below threshold:
    # no), 5 (next to 4) kept; 6 and 7 weak with no strong neighbour: dropped
    assert S[:, 4].tolist() == [True, True, False, False, True, True, False, False, False]
    assert S[:, [0, 1, 2, 3, 5, 6, 7, 8]].sum() == 0
    # a larger neighbour across the gradient suppresses the pixel
    M2 = M.copy()
    M2[4, 5] = 0.3
    assert not dt.select(gx, gy, M2)[4, 4]
    # the hysteresis step counts diagonal neighbours: a weak pixel whose only
    # strong neighbour is diagonal is kept
    gx3 = np.zeros((H, W)); M3 = np.full((H, W), 0.01)
    gx3[2, 2] = gx3[3, 3] = 1.0
    M3[2, 2], M3[3, 3] = 0.25, 0.15
    S3 = dt.select(gx3, np.zeros((H, W)), M3)
    assert S3[2, 2] and S3[3, 3] and S3.sum() == 2


def _view_case(seed, H=22, W=26):
    rng = np.random.default_rng(seed)
    R = np.full((H, W, 3), 0.2) + rng.uniform(0, 0.05, (H, W, 3))
    R[5:16, 6:19] = rng.uniform(0.6, 0.9, 3)
    R[9:13, 3:12] = rng.uniform(0.0, 0.2, 3)
    O = R.copy()
    O[6:17, 7:20] = rng.uniform(0.5, 0.95, 3)
    return R, O


def test_edge_term_gradient_matches_central_differences():
    R, O = _view_case(1)
    H, W = R.shape[:2]
    wh, off = np.array([[W, H]]), np.array([0, H * W])
    Rp = R.reshape(-1, 3)
    Be = dt.edge_maps(O.reshape(-1, 3), wh, off)
    T = np.eye(3).reshape(1, 9)
    mask = np.ones(H * W, np.uint8)
    loss, gR, gT, rp, br, sel = dt.data_term(Rp, T, O.reshape(-1, 3), Be, mask, wh, off, [0], 1)
    assert sel.any()
    rng = np.random.default_rng(2)
    idx = rng.choice(H * W, 40, replace=False)
    h = 1e-6
    for p in idx:
        for ch in range(3):
            out = []
            for sgn in (1, -1):
                R2 = Rp.copy()
                R2[p, ch] += sgn * h
                l2, _, _, _, _, s2 = dt.data_term(R2, T, O.reshape(-1, 3), Be, mask, wh, off, [0], 1)
                assert np.array_equal(s2, sel)   # the selection stays frozen
                out.append(l2[0])
            fd = (out[0] - out[1]) / (2 * h)
            assert abs(fd - gR[p, ch]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gR).max()) + 1e-9, (p, ch, fd, gR[p, ch])


def test_colour_transform_linearity_and_gradient():
    R, O = _view_case(4)
    H, W = R.shape[:2]
    wh, off = np.array([[W, H]]), np.array([0, H * W])
    Rp = R.reshape(-1, 3)
    assert np.array_equal(dt.colour_transform(Rp, np.eye(3).reshape(1, 9), off), Rp)
    rng = np.random.default_rng(5)
    T1, T2 = rng.normal(size=(1, 9)), rng.normal(size=(1, 9))
    a = dt.colour_transform(Rp, T1 + T2, off)
    b = dt.colour_transform(Rp, T1, off) + dt.colour_transform(Rp, T2, off)
    assert np.allclose(a, b, atol=1e-14)
    Be = dt.edge_maps(O.reshape(-1, 3), wh, off)
    T = (np.eye(3) + 0.05 * rng.normal(size=(3, 3))).reshape(1, 9)
    loss, gR, gT, rp, br, sel = dt.data_term(Rp, T, O.reshape(-1, 3), Be, None, wh, off, [0], 1, w_e=0.5)
    # dE/dR through the transform (T not symmetric)
    for p, ch in [(30, 0), (250, 1), (401, 2), (77, 1)]:
        out = []
        for sgn in (1, -1):
            R2 = Rp.copy()
            R2[p, ch] += sgn * 1e-6
            l2, _, _, _, _, s2 = dt.data_term(R2, T, O.reshape(-1, 3), Be, None, wh, off, [0], 1, w_e=0.5)
            assert np.array_equal(s2, sel)
            out.append(l2[0])
        fd = (out[0] - out[1]) / 2e-6
        assert abs(fd - gR[p, ch]) <= 1e-5 * max(abs(fd), 1e-2 * np.abs(gR).max()), (p, ch, fd, gR[p, ch])
    h = 1e-7
    for k in range(9):
        out = []
        for sgn in (1, -1):
            T2_ = T.copy()
            T2_[0, k] += sgn * h
            l2, _, _, _, _, s2 = dt.data_term(Rp, T2_, O.reshape(-1, 3), Be, None, wh, off, [0], 1, w_e=0.5)
            assert np.array_equal(s2, sel)
            out.append(l2[0])
        fd = (out[0] - out[1]) / (2 * h)
        assert abs(fd - gT[0, k]) <= 1e-5 * max(abs(fd), 1e-2 * np.abs(gT).max()), (k, fd, gT[0, k])


def test_two_level_colour_map():
    rng = np.random.default_rng(6)
    low = rng.uniform(size=(2, 8, 8, 3))
    high = rng.normal(0, 0.1, size=(2, 64, 32, 3))
    V = dt.compose_albedo(low, high)
    ref = high + np.stack([np.stack([np.kron(low[h, :, :, c], np.ones((8, 4))) for c in range(3)], -1)
                           for h in range(2)])
    assert np.array_equal(V, ref)
    # L = sum w * V is linear in low: its gradient is exact and equals the block sums
    w = rng.normal(size=V.shape)
    g = dt.albedo_low_grad(w, 8)
    for (h, i, j, c) in [(0, 0, 0, 0), (1, 7, 7, 2), (0, 3, 5, 1)]:
        e = np.zeros_like(low)
        e[h, i, j, c] = 1.0
        d = (w * (dt.compose_albedo(low + e, high) - V)).sum()
        assert abs(d - g[h, i, j, c]) < 1e-12


@pytest.mark.parametrize("sgn", [1.0, -1.0])
def test_diagonal_suppression(sgn):
    # gradients along a diagonal: a ridge of magnitude across that direction
    # survives, its neighbours along the gradient do not
    # (a diagonal step moves i + j, or i - j, by 2: the even lines carry a
    # peak at line 8 and weak values that fall away from it, the odd lines
    # stay below the low threshold)
    H = W = 11
    gx = np.ones((H, W))
    gy = np.full((H, W), sgn)
    i, j = np.mgrid[0:H, 0:W]
    k = i + j if sgn > 0 else i - j + 8
    M = np.where(k % 2 == 1, 0.05, 0.15 - 0.005 * np.abs(k - 8))
    M = np.where(k == 8, 0.3, M)
    S = dt.select(gx, gy, M)
    assert np.array_equal(S[1:-1, 1:-1], (k == 8)[1:-1, 1:-1])
