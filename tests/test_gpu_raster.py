"""Hard rasterisation (hr_set_renderer(HR_RENDERER_RASTER); Section 4.2.2,
"Ray tracing vs rasterization") on the HIP path, through the C ABI, against
the oracle (oracle/raster.py) on identical float32 vertices: every pixel's
covering triangle bit-exact (screen bins and, with the hierarchy selected,
the all-triangle path), images 1e-5 relative, the gradients at fixed
coverage (colour map, unit vertex normals, vertices, parameters per block)
within 1e-4 per block and element-wise.  The edge term is ignored in raster
mode, a scene of more than one sample per pixel is refused, and
hr_iterate runs the loop."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import DEV, block_rel, check_grad, f32, rel_err
from oracle import raster
from paper_2107_05509_amd import binding, scene

pytestmark = pytest.mark.gpu


class RasterCase:
    def __init__(self, w, seed=5):
        self.w = w
        self.om = oracle.Model(w.model)
        self.tab = scene.camera_arrays(w.cams)
        self.th, self.tw = w.albedo_true.shape[1:3]
        self.g = binding.Scene(w.model, w.cams, w.n_hands, 1, self.th, self.tw, seed=seed)
        self.g.set_renderer(binding.HR_RENDERER_RASTER)
        self.P = int(self.tab["pix_off"][-1])
        self.bg = f32(w.packed_background())
        self.params = f32(w.params_init)
        self.albedo = f32(w.albedo_true)
        v, _ = oracle.skin(self.om, torch.as_tensor(self.params.astype(np.float64)))
        self.v32 = f32(v.numpy())
        self.fpp = raster.raster_faces(self.v32, w.model.faces, self.tab)

    def t(self, a, dt=torch.float32):
        return torch.as_tensor(np.ascontiguousarray(a)).to(DEV, dt)

    def gpu_render(self):
        img = torch.empty(self.P, 3, device=DEV)
        hf = torch.empty(self.P, 1, device=DEV, dtype=torch.int32)
        self.g.render(self.t(self.v32), self.t(self.albedo), self.t(self.bg), 0, img, hf)
        torch.cuda.synchronize()
        return img.cpu().numpy(), hf.cpu().numpy()[:, 0]

    def oracle_image(self, v64=None, nrm=None, alb=None):
        v64 = torch.as_tensor(self.v32.astype(np.float64)) if v64 is None else v64
        nrm = oracle.vertex_normals(v64, self.om.faces) if nrm is None else nrm
        alb = torch.as_tensor(self.albedo.astype(np.float64)) if alb is None else alb
        return raster.raster_image(v64, nrm, self.w.model.uv, alb, self.bg, self.w.model.faces, self.tab,
                                   scene.SHADING, self.fpp)

    def oracle_grads(self, d):
        v64 = torch.as_tensor(self.v32.astype(np.float64)).requires_grad_(True)
        nrm = oracle.vertex_normals(v64.detach(), self.om.faces).requires_grad_(True)
        alb = torch.as_tensor(self.albedo.astype(np.float64)).requires_grad_(True)
        (torch.as_tensor(d, dtype=torch.float64) * self.oracle_image(v64, nrm, alb)).sum().backward()
        gn = nrm.grad.numpy()
        p = torch.as_tensor(self.params.astype(np.float64)).requires_grad_(True)
        vs, _ = oracle.skin(self.om, p)
        vt = torch.as_tensor(self.v32.astype(np.float64)).requires_grad_(True)
        torch.autograd.backward([oracle.vertex_normals(vt, self.om.faces)], [torch.as_tensor(gn)])
        gv = v64.grad.numpy() + vt.grad.numpy()
        torch.autograd.backward([vs], [torch.as_tensor(gv)])
        return dict(ga=alb.grad.numpy(), gn=gn, gv=gv, gp=p.grad.numpy())

    def gpu_grads(self, d, flags=binding.HR_GRAD_ALL):
        H = self.w.n_hands
        gp = torch.empty(H, 64, device=DEV)
        ga = torch.empty(H, self.th, self.tw, 3, device=DEV)
        gv = torch.empty(H, self.w.model.n_verts, 3, device=DEV)
        gn = torch.empty_like(gv)
        self.g.backward(self.t(self.params), self.t(self.v32), self.t(self.albedo), self.t(self.bg), self.t(d), 0,
                        gp, ga, gv, gn, flags)
        torch.cuda.synchronize()
        return dict(ga=ga.cpu().numpy(), gn=gn.cpu().numpy(), gv=gv.cpu().numpy(), gp=gp.cpu().numpy())


@pytest.fixture(scope="module", params=["tiny", "mixed"])
def case(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"case: hard rasterisation, {request.param} workload, 1 sample per pixel", flush=True)
    w = scene.workload_tiny(0) if request.param == "tiny" else scene.workload_mixed(0)
    return RasterCase(w)


def test_covering_triangles_and_image(case):
    c = case
    img, hit = c.gpu_render()
    assert (c.fpp >= 0).mean() > 0.02
    assert np.array_equal(hit, c.fpp), f"{(hit != c.fpp).sum()} pixels differ"
    e = rel_err(img, c.oracle_image().numpy())
    print("image rel err max %.3g" % e.max(), flush=True)
    assert e.max() <= 1e-5
    # the all-triangle path (no screen bins) picks the same triangles
    c.g.set_accel(binding.HR_ACCEL_HIERARCHY)
    try:
        img2, hit2 = c.gpu_render()
    finally:
        c.g.set_accel(binding.HR_ACCEL_AUTO)
    assert np.array_equal(hit2, c.fpp)
    assert np.array_equal(img2, img)


def test_gradients_at_fixed_coverage(case):
    c = case
    d = f32(np.random.default_rng(7).normal(0, 1e-3, (c.P, 3)))
    g = c.gpu_grads(d)
    o = c.oracle_grads(d)
    for k in ("ga", "gn", "gv"):
        check_grad(k, g[k], o[k])
    for name, sl in {"pose": slice(0, 48), "shape": slice(48, 58), "global": slice(58, 64)}.items():
        check_grad(name, g["gp"][:, sl], o["gp"][:, sl])
    # no edge term: the interior term alone gives the same gradient
    gi = c.gpu_grads(d, binding.HR_GRAD_INTERIOR)
    for k in ("ga", "gv", "gp"):
        assert block_rel(gi[k], g[k]) <= 1e-6


def test_raster_needs_one_sample_per_pixel():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = scene.workload_tiny(0)
    th, tw = w.albedo_true.shape[1:3]
    g = binding.Scene(w.model, w.cams, w.n_hands, 4, th, tw, seed=5)
    with pytest.raises(binding.HRError):
        g.set_renderer(binding.HR_RENDERER_RASTER)
    with pytest.raises(binding.HRError):
        g.set_renderer(7)


def test_raster_refinement_loop(case):
    # hr_iterate in raster mode from the perturbed pose towards the oracle's
    # raster image of the true pose (true colour map, held fixed): the loss
    # falls, and the edge flag changes nothing (up to the order of the
    # adjoint's floating-point atomic sums)
    c = case
    vt, _ = oracle.skin(c.om, torch.as_tensor(np.asarray(c.w.params_true, np.float64)))
    vt32 = f32(vt.numpy())
    ft = raster.raster_faces(vt32, c.w.model.faces, c.tab)
    v64 = torch.as_tensor(vt32.astype(np.float64))
    tgt = raster.raster_image(v64, oracle.vertex_normals(v64, c.om.faces), c.w.model.uv,
                              torch.as_tensor(c.albedo.astype(np.float64)), c.bg, c.w.model.faces, c.tab,
                              scene.SHADING, ft).numpy()
    outs = []
    for flags in (binding.HR_GRAD_ALL, binding.HR_GRAD_ALL, binding.HR_GRAD_INTERIOR):
        st = c.g.make_state(c.t(c.params), c.t(c.albedo), c.t(c.bg), c.t(tgt))
        losses = []
        for _ in range(20):
            c.g.iterate(st, (0.0, 1e-2, 1e-2, 1e-2, 1e-3, 0.0), flags=flags)
            torch.cuda.synchronize()
            losses.append(st.loss.cpu().numpy().copy())
        outs.append((st.params.cpu().numpy(), np.array(losses)))
    print("raster loop losses", outs[0][1][[0, -1]].ravel(), flush=True)
    # Adam's normalised steps amplify the last-bit differences of the atomic
    # sums over 20 iterations (two runs with the same flags have differed by
    # up to 1.8e-3): the bar is that spread (times 3), and no tighter than
    # 5e-3 (the edge term, were it wrongly applied, moves the pose by far more)
    moved = outs[0][0] - c.params
    noise = block_rel(outs[1][0] - c.params, moved)
    err = block_rel(outs[2][0] - c.params, moved)
    print("moved: spread of two runs", noise, "edge flag off", err, flush=True)
    assert err <= max(3.0 * noise, 5e-3)
    # a pixel whose covering triangle flips in a later iteration moves the
    # loss by about one pixel's share
    lnoise = np.abs(outs[1][1] - outs[0][1]).max()
    assert np.abs(outs[2][1] - outs[0][1]).max() <= max(3.0 * lnoise, 1e-2 * np.abs(outs[0][1]).max())
    assert np.all(outs[0][1][-1] < outs[0][1][0])
