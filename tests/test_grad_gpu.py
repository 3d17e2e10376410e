"""GPU shading adjoint (orrb_shade_backward through the C ABI) against the oracle.

* analytic: for the same upstream gradient dL/drgb (seeded, or the squared error's
  2 (rgb - target) from the GPU's forward), the GPU adjoint equals the oracle's FP64
  analytic adjoint within 1e-4 relative on every parameter with |g| >= 1e-3 max|g| of
  its kind (near-tie pixels, whose visibility may resolve either way, carry weight 0
  on both sides);
* finite differences: on the full differentiable-shading workload (64 hand-like
  scenes x 3 cameras at 200x200, targets rendered with perturbed materials and
  lights), 16 random parameters match FP64 central differences (h = 1e-4) of the
  oracle's loss within 1e-4 relative, over the pixels whose loss is smooth within
  the step (see tests/fd.py);
* ShadeFn backward equals the direct call, and repeated calls are bit-identical.
"""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import fd

pytestmark = pytest.mark.gpu

KINDS = ("albedo", "roughness", "specular", "light_vec", "light_intensity", "exposure")


@pytest.fixture(scope="module")
def renderer():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    assert torch.cuda.is_available()
    return Renderer(0)


def _planar_weight(batch, weight):
    """Per-pixel weight [P] expanded to the planar rgb layout [3P]."""
    po = batch.pixel_offset
    return np.concatenate([np.tile(np.asarray(weight)[po[f]:po[f + 1]], 3) for f in range(batch.n_frames)])


def _gpu_backward(renderer, batch, grad_rgb_fn):
    """Forward on the GPU, then the adjoint of the upstream gradient grad_rgb_fn(rgb)
    (called twice to check determinism)."""
    import torch
    from paper_1906_11633_amd.renderer import shade_backward
    job = renderer.prepare(batch)
    out = renderer.render(job, vis=True)
    grad_rgb = grad_rgb_fn(out["rgb"]).contiguous()
    g = shade_backward(renderer.ctx, job.layout, job.state, out["vis"], grad_rgb)
    g2 = shade_backward(renderer.ctx, job.layout, job.state, out["vis"], grad_rgb)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy().astype(np.float64) for k, v in g.items()}
    for k in g:
        assert torch.equal(g[k], g2[k]), f"backward not deterministic: {k}"
    return res, job, out


def _gpu_grad(renderer, batch, target_rgb, weight):
    """GPU adjoint of the squared error: grad_rgb = 2 (rgb - target) * w."""
    import torch
    tgt = torch.from_numpy(np.asarray(target_rgb, np.float32)).cuda()
    w = torch.from_numpy(_planar_weight(batch, weight).astype(np.float32)).cuda()
    return _gpu_backward(renderer, batch, lambda rgb: 2.0 * (rgb - tgt) * w)


def _upstream(batch, weight, seed):
    """Seeded upstream gradient in [-1, 1], fp32-exact, zero on weight-0 pixels."""
    c = np.random.default_rng(seed).uniform(-1, 1, 3 * batch.total_pixels).astype(np.float32)
    return c * _planar_weight(batch, weight).astype(np.float32)


def _linear_pair(renderer, batch, weight, seed):
    """GPU and oracle adjoints of the same fixed upstream gradient.  The forward's
    fp32 rounding does not enter the upstream gradient here, so the comparison
    isolates the backward pass."""
    import torch
    c = _upstream(batch, weight, seed)
    ct = torch.from_numpy(c).cuda()
    gpu, _, _ = _gpu_backward(renderer, batch, lambda rgb: ct)
    _, ref = oracle.shade_grad(batch, dl_drgb=c.astype(np.float64), pixel_weight=np.asarray(weight, np.uint8))
    return gpu, ref


def _compare(gpu, ref, rtol=1e-4):
    worst = {}
    for k in KINDS:
        a, b = gpu[k].reshape(-1), ref[k].reshape(-1)
        scale = np.abs(b).max()
        assert scale > 0, k
        sel = np.abs(b) >= 1e-3 * scale
        rel = np.abs(a[sel] - b[sel]) / np.abs(b[sel])
        worst[k] = float(rel.max())
        assert rel.max() <= rtol, (k, worst[k], int(np.argmax(rel)))
    return worst


def test_adjoint_matches_oracle_small(renderer):
    """Point lights, hand-like scenes: same seeded upstream gradient on both sides."""
    base, _ = S.config4(4, 3, 72)
    w = (~oracle.near_tie(oracle.render(base))).astype(np.uint8)
    gpu, ref = _linear_pair(renderer, base, w, 11)
    print(_compare(gpu, ref))


def test_adjoint_directional_lights(renderer):
    """Config-1 scenes with materials: directional lights, whose direction vector
    gets a gradient through n.l and the half vector."""
    b = S.config1(materials=True)
    w = (~oracle.near_tie(oracle.render(b))).astype(np.uint8)
    gpu, ref = _linear_pair(renderer, b, w, 12)
    print(_compare(gpu, ref))


def test_adjoint_directional_and_point_rotated_camera(renderer):
    """A plane seen through a rotated LookAt camera, lit by a directional light near
    the mirror direction (a highlight) and a point light: the direction's gradient
    goes through R_V^T, which an identity view would not test."""
    from tests.test_oracle_edge_cases import MIRROR_U, directional_batch
    lights = ((1, MIRROR_U, 1.3), (0, (0.9, -1.1, 1.4), 2.5))
    b = directional_batch(0.6, 0.3, lights=lights)
    w = (~oracle.near_tie(oracle.render(b))).astype(np.uint8)
    gpu, ref = _linear_pair(renderer, b, w, 13)
    assert np.abs(ref["light_vec"][0]).max() > 0
    print(_compare(gpu, ref))


def test_adjoint_squared_error_small(renderer):
    """The squared-error adjoint: the upstream gradient 2 (rgb - target) is built from
    the GPU's own fp32 forward rgb and the same array is fed to the oracle's adjoint,
    so both sides differentiate the same loss at the same point: 1e-4 relative."""
    import torch
    base, target = S.config4(4, 3, 72)
    tgt = torch.from_numpy(oracle.render(target)["rgb"].astype(np.float32)).cuda()
    w = (~oracle.near_tie(oracle.render(base))).astype(np.uint8)
    wt = torch.from_numpy(_planar_weight(base, w).astype(np.float32)).cuda()
    held = {}

    def upstream(rgb):
        held["c"] = (2.0 * (rgb - tgt) * wt).contiguous()
        return held["c"]

    gpu, _, _ = _gpu_backward(renderer, base, upstream)
    c = held["c"].cpu().numpy().astype(np.float64)
    _, ref = oracle.shade_grad(base, dl_drgb=c, pixel_weight=w)
    print(_compare(gpu, ref))


def test_adjoint_vs_finite_differences_config4(renderer):
    """Differentiable-shading workload at full size: 16 parameters vs FP64 central
    differences (h = 1e-4)."""
    base, target = S.config4(4, 64, 200)
    tgt = oracle.render(target, threads=0)["rgb"]
    ref_out = oracle.render(base, threads=0)
    w = fd.smooth_mask(base, ref_out) & (~oracle.near_tie(ref_out)).astype(np.uint8)
    gpu, _, _ = _gpu_grad(renderer, base, tgt, w)
    rng = np.random.default_rng(16)
    po = ref_out["pixel_offset"]
    checked = []
    kinds = list(KINDS)
    while len(checked) < 16:
        k = kinds[len(checked) % len(kinds)]
        flat = gpu[k].reshape(-1)
        cand = np.nonzero(np.abs(flat) >= 1e-3 * np.abs(flat).max())[0]
        idx = int(rng.choice(cand))
        # the parameter's scene: only its frames' loss changes
        if k in ("albedo", "roughness", "specular"):
            o = idx // 3 if k == "albedo" else idx
            s = int(np.searchsorted(base.scene_object_begin, o, side="right") - 1)
        elif k in ("light_vec", "light_intensity"):
            l = idx // 3 if k == "light_vec" else idx
            s = int(np.searchsorted(base.scene_light_begin, l, side="right") - 1)
        else:
            s = int(base.frame_scene[idx])
        sub = base.select_scenes([s])
        frames = np.nonzero(base.frame_scene == s)[0]
        f0, f1 = int(frames[0]), int(frames[-1]) + 1
        sub_t = tgt[3 * po[f0]:3 * po[f1]]
        sub_w = w[po[f0]:po[f1]]
        # index of the parameter inside the one-scene batch
        if k == "albedo":
            sidx = idx - 3 * int(base.scene_object_begin[s])
        elif k in ("roughness", "specular"):
            sidx = idx - int(base.scene_object_begin[s])
        elif k == "light_vec":
            sidx = idx - 3 * int(base.scene_light_begin[s])
        elif k == "light_intensity":
            sidx = idx - int(base.scene_light_begin[s])
        else:
            sidx = idx - f0
        d = fd.central_difference(sub, sub_t, k, sidx, 1e-4, sub_w)
        rel = abs(flat[idx] - d) / abs(d)
        checked.append((k, idx, float(flat[idx]), d, rel))
        assert rel <= 1e-4, checked[-1]
    print("fd checks:", checked)


def test_shadefn_autograd(renderer):
    import torch
    from paper_1906_11633_amd.autograd import shade
    from paper_1906_11633_amd.renderer import shade_backward
    base, target = S.config4(4, 2, 64)
    tgt = torch.from_numpy(oracle.render(target)["rgb"].astype(np.float32)).cuda()
    job = renderer.prepare(base)
    params = [job.state[k].clone().requires_grad_(True) for k in
              ("albedo", "roughness", "specular", "light_vec", "light_intensity", "exposure")]
    rgb = shade(renderer, job, *params)
    loss = ((rgb - tgt) ** 2).sum()
    loss.backward()
    out = renderer.render(job, vis=True)
    g = shade_backward(renderer.ctx, job.layout, job.state, out["vis"], (2.0 * (out["rgb"] - tgt)).contiguous())
    torch.cuda.synchronize()
    for p, k in zip(params, ("albedo", "roughness", "specular", "light_vec", "light_intensity", "exposure")):
        assert torch.equal(p.grad, g[k]), k
