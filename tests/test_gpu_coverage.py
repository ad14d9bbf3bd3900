"""Camera coverage (paper Section 4.2.3, Eq. 6) on the HIP path, through the C ABI,
against the oracle: faces seen per view from the render's hit ids, and the
greedy camera order.  Bar: bit-exact (integer work)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, Case
from paper_2107_05509_amd import scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("case: 12 views 64x96, 4 spp, seed 0, camera coverage", flush=True)
    return Case(scene.workload_realistic(0, n_views=12, W=64, H=96, f=134.0, tex=64, spp=4))


def _hand_views(c):
    hands = np.asarray(c.tab["hand"])
    return [list(np.nonzero(hands == h)[0]) for h in range(c.w.n_hands)]


def _gpu_order(c, vis):
    order = torch.empty(len(c.cams), dtype=torch.int32, device=DEV)
    covered = torch.empty_like(order)
    c.gsc.camera_order(vis, order, covered)
    torch.cuda.synchronize()
    return order.cpu().numpy(), covered.cpu().numpy()


def test_visibility_and_order(case):
    c = case
    _, ghits = c.gpu_render(0, hits=True)
    _, ohits = c.oracle_render(0, hits=True)
    assert np.array_equal(ghits, ohits)
    vis = torch.empty(len(c.cams), c.model.n_faces, dtype=torch.int32, device=DEV)
    c.gsc.face_visibility(torch.as_tensor(ghits).to(DEV), vis)
    torch.cuda.synchronize()
    ovis = oracle.face_visibility(ohits, np.asarray(c.tab["pix_off"]), c.model.n_faces)
    assert np.array_equal(vis.cpu().numpy() != 0, ovis)
    order, covered = _gpu_order(c, vis)
    oorder, ocovered = oracle.camera_order(ovis, _hand_views(c))
    print("order", order.tolist(), "covered", covered.tolist(), flush=True)
    assert order.tolist() == oorder.tolist() and covered.tolist() == ocovered.tolist()
    assert covered[0] > 0 and np.all(np.diff(covered) >= 0)


def test_order_of_given_visibility(case):
    # sparse, dense and tied visibility sets (ties: the earlier view)
    c = case
    rng = np.random.default_rng(4)
    n, F = len(c.cams), c.model.n_faces
    for p in (0.002, 0.05, 0.5):
        v = rng.uniform(size=(n, F)) < p
        v[3] = v[1]   # an exact tie
        v[7] = False  # an empty view
        order, covered = _gpu_order(c, torch.as_tensor(v.astype(np.int32)).to(DEV))
        oorder, ocovered = oracle.camera_order(v, _hand_views(c))
        assert order.tolist() == oorder.tolist() and covered.tolist() == ocovered.tolist(), p
