"""Pins of the oracle's shading adjoint (CPU only).

The adjoint is the exact derivative of the forward shading over the fixed
visibility, so it must match FP64 central finite differences of the oracle's own
loss (the forward being pinned separately), and the closed forms that linearity
gives for exposure, intensity and albedo."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import fd

PARAMS = ("albedo", "roughness", "specular", "light_vec", "light_intensity", "exposure")


def _small_problem(res=40, n_scenes=2, seed=4):
    base, target = S.config4(seed, n_scenes, res)
    tgt = oracle.render(target)["rgb"]
    return base, tgt


def test_adjoint_matches_central_differences():
    """Analytic gradient vs FP64 central differences (h = 1e-4) on every parameter
    kind, several entries each, over the pixels whose loss is smooth within the step
    (kink pixels of max(0, n.l) and max(0, n.h) held out, 0.1 % here)."""
    b, tgt = _small_problem()
    mask = fd.smooth_mask(b, oracle.render(b))
    assert mask.mean() > 0.99
    L0, g = oracle.shade_grad(b, tgt, mask)
    assert L0 > 0
    rng = np.random.default_rng(0)
    checked = 0
    for name in PARAMS:
        flat = g[name].reshape(-1)
        scale = np.abs(flat).max()
        assert scale > 0, name
        cand = np.nonzero(np.abs(flat) >= 1e-3 * scale)[0]
        for idx in rng.choice(cand, size=min(4, cand.size), replace=False):
            d = fd.central_difference(b, tgt, name, idx, 1e-4, mask)
            assert abs(flat[idx] - d) <= 1e-6 * abs(d) + 1e-9 * scale, (name, idx, flat[idx], d)
            checked += 1
    assert checked >= 20


def test_light_vecition_adjoint_converges_without_mask():
    """Over all pixels the light-position difference converges to the analytic
    gradient as h shrinks (the h = 1e-4 gap is the terminator kink, not the adjoint)."""
    b, tgt = _small_problem()
    _, g = oracle.shade_grad(b, tgt)
    for idx in range(3):
        d = fd.central_difference(b, tgt, "light_vec", idx, 1e-6)
        a = g["light_vec"].reshape(-1)[idx]
        assert abs(a - d) <= 1e-7 * abs(a), (idx, a, d)


def test_exposure_and_intensity_gradients_by_linearity():
    """rgb = e * U and (one light) rgb = I * U', so dL/de = sum g . rgb / e and
    dL/dI = sum g . rgb / I, from the forward render alone."""
    b, tgt = _small_problem()
    # keep one light per scene so each scene's rgb is linear in its single intensity
    lb = b.scene_light_begin
    keep = np.concatenate([np.arange(lb[s], lb[s] + 1) for s in range(b.n_scenes)])
    b1 = b.replace(scene_light_begin=np.arange(b.n_scenes + 1, dtype=np.int32), light_type=b.light_type[keep],
                   light_vec=b.light_vec[keep], light_intensity=b.light_intensity[keep])
    out = oracle.render(b1)
    _, g = oracle.shade_grad(b1, tgt)
    gpx = 2 * (out["rgb"] - tgt)
    po = out["pixel_offset"]
    for f in range(b1.n_frames):
        sl = slice(3 * po[f], 3 * po[f + 1])
        e = float(b1.exposure[f])
        np.testing.assert_allclose(g["exposure"][f], (gpx[sl] * out["rgb"][sl]).sum() / e, rtol=1e-10)
    for s in range(b1.n_scenes):
        frames = np.nonzero(b1.frame_scene == s)[0]
        tot = sum((gpx[3 * po[f]:3 * po[f + 1]] * out["rgb"][3 * po[f]:3 * po[f + 1]]).sum() for f in frames)
        np.testing.assert_allclose(g["light_intensity"][s], tot / float(b1.light_intensity[s]), rtol=1e-10)


def test_albedo_gradient_by_linearity_lambert():
    """With k_s = 0, rgb_c of object o's pixels is albedo_c * (e sum A ndl), so
    dL/da_{o,c} = sum over o's pixels of g_c * rgb_c / a_{o,c}."""
    b, tgt = _small_problem()
    b0 = b.replace(specular=np.zeros(b.n_objects))
    out = oracle.render(b0)
    _, g = oracle.shade_grad(b0, tgt)
    po = out["pixel_offset"]
    acc = np.zeros((b0.n_objects, 3))
    for f in range(b0.n_frames):
        s = int(b0.frame_scene[f])
        ob, oe = b0.scene_object_begin[s], b0.scene_object_begin[s + 1]
        tb = np.concatenate([[0], np.cumsum([b0.meshes[m].n_tris for m in b0.object_mesh[ob:oe]])])
        t = out["tri_id"][po[f]:po[f + 1]]
        n = po[f + 1] - po[f]
        rgb = out["rgb"][3 * po[f]:3 * po[f + 1]].reshape(3, n)
        gp = 2 * (rgb - tgt[3 * po[f]:3 * po[f + 1]].reshape(3, n))
        cov = t >= 0
        obj = ob + np.searchsorted(tb, t[cov], side="right") - 1
        for c in range(3):
            np.add.at(acc[:, c], obj, gp[c, cov] * rgb[c, cov])
    alb = b0.albedo.astype(np.float64)
    ok = alb > 1e-3
    np.testing.assert_allclose(g["albedo"][ok], acc[ok] / alb[ok], rtol=1e-9, atol=1e-12)


def test_pixel_weight_mask_and_determinism():
    b, tgt = _small_problem(res=32)
    L1, g1 = oracle.shade_grad(b, tgt, threads=1)
    L2, g2 = oracle.shade_grad(b, tgt, threads=4)
    assert L1 == L2
    for k in PARAMS:
        assert np.array_equal(g1[k], g2[k])
    z = np.zeros(b.total_pixels, np.uint8)
    L0, g0 = oracle.shade_grad(b, tgt, pixel_weight=z)
    assert L0 == 0 and all(np.all(g0[k] == 0) for k in PARAMS)
    # the loss is the plain sum of squared errors over all pixels and channels
    out = oracle.render(b)
    np.testing.assert_allclose(L1, ((out["rgb"] - tgt) ** 2).sum(), rtol=1e-12)


def _linear_fd(b, c, mask, name, idx, h):
    """Central difference of L = sum w c . rgb from two forward renders (no adjoint
    code involved)."""
    w3 = np.concatenate([np.tile(mask[b.pixel_offset[f]:b.pixel_offset[f + 1]], 3)
                         for f in range(b.n_frames)]).astype(np.float64)
    lp = (c * w3 * oracle.render(fd.perturbed(b, name, idx, h))["rgb"]).sum()
    lm = (c * w3 * oracle.render(fd.perturbed(b, name, idx, -h))["rgb"]).sum()
    return (lp - lm) / (2 * h)


def test_upstream_gradient_mode():
    """With a fixed upstream gradient c the loss is sum w c . rgb: its value is that
    sum over the forward render, and its gradient matches central differences of
    that sum; with c = 2 (rgb - target) it equals the squared-error gradient."""
    b, tgt = _small_problem(res=32)
    out = oracle.render(b)
    mask = fd.smooth_mask(b, out)
    c = np.random.default_rng(7).uniform(-1, 1, 3 * b.total_pixels)
    L, g = oracle.shade_grad(b, dl_drgb=c, pixel_weight=mask)
    w3 = np.concatenate([np.tile(mask[b.pixel_offset[f]:b.pixel_offset[f + 1]], 3)
                         for f in range(b.n_frames)]).astype(np.float64)
    np.testing.assert_allclose(L, (c * w3 * out["rgb"]).sum(), rtol=1e-12)
    rng = np.random.default_rng(1)
    for name in PARAMS:
        flat = g[name].reshape(-1)
        cand = np.nonzero(np.abs(flat) >= 1e-3 * np.abs(flat).max())[0]
        for idx in rng.choice(cand, size=min(2, cand.size), replace=False):
            d = _linear_fd(b, c, mask, name, idx, 1e-4)
            assert abs(flat[idx] - d) <= 1e-6 * abs(d) + 1e-9 * np.abs(flat).max(), (name, idx, flat[idx], d)
    _, gq = oracle.shade_grad(b, tgt)
    _, gl = oracle.shade_grad(b, dl_drgb=2.0 * (out["rgb"] - tgt))
    for k in PARAMS:
        np.testing.assert_allclose(gl[k], gq[k], rtol=1e-12, atol=1e-15 * np.abs(gq[k]).max())
