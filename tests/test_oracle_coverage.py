"""Pins of the oracle's camera-coverage ordering (paper Section 4.2.3, camera
coverage, Eq. 6): a worked example, the tie rule, the coverage bound every
greedy maximum-coverage order meets against brute force over all subsets, and
visibility recounted from hit ids by plain loops."""
import itertools

import numpy as np

import oracle


def _sets(n_faces, sets):
    v = np.zeros((len(sets), n_faces), dtype=bool)
    for i, s in enumerate(sets):
        v[i, list(s)] = True
    return v


def test_worked_example():
    vis = _sets(12, [{0, 1, 2, 10}, {0, 1, 2, 3, 4, 5}, set(), {4, 5, 6, 7, 8, 9}])
    order, covered = oracle.camera_order(vis, [[0, 1, 2, 3]])
    # view 1 (6 faces; view 3 ties later in the list), then view 3 (+4: 6..9),
    # then view 0 (+1: face 10), then the empty view 2
    assert order.tolist() == [1, 3, 0, 2]
    assert covered.tolist() == [6, 10, 11, 11]


def test_ties_take_the_earlier_view_and_hands_are_separate():
    vis = _sets(6, [{0, 1}, {2, 3}, {4, 5}, {0, 1}])
    order, covered = oracle.camera_order(vis, [[2, 0], [3, 1]])
    assert order.tolist() == [2, 0, 3, 1]
    assert covered.tolist() == [2, 4, 2, 4]


def test_greedy_coverage_bound_against_brute_force():
    rng = np.random.default_rng(0)
    for trial in range(20):
        n, F = 7, 40
        vis = rng.uniform(size=(n, F)) < rng.uniform(0.1, 0.5)
        order, covered = oracle.camera_order(vis, [list(range(n))])
        assert sorted(order.tolist()) == list(range(n))
        assert np.all(np.diff(covered) >= 0)                       # Eq. 6: never decreases
        assert covered[-1] == int(vis.any(0).sum())
        for k in range(1, n + 1):
            best = max(int(vis[list(c)].any(0).sum()) for c in itertools.combinations(range(n), k))
            assert covered[k - 1] >= (1 - 1 / np.e) * best - 1e-9   # greedy maximum coverage
            if k == 1:
                assert covered[0] == best                           # the first step is optimal


def test_visibility_from_hits():
    rng = np.random.default_rng(1)
    pix_off = np.array([0, 5, 5, 12])
    hits = rng.integers(-1, 9, size=(12, 3)).astype(np.int32)
    vis = oracle.face_visibility(hits, pix_off, 9)
    for i in range(3):
        for f in range(9):
            seen = False
            for p in range(pix_off[i], pix_off[i + 1]):
                for s in range(3):
                    if hits[p, s] == f:
                        seen = True
            assert vis[i, f] == seen
