"""Finite-difference helpers for the shading-gradient checks (test helper).

The shading has kinks: max(0, n.l) at a light's terminator and max(0, n.h) where the
highlight vanishes.  A central difference whose +-h interval straddles a kink
measures the mean of the two one-sided slopes, not the derivative, and at h = 1e-4 m
the terminator pixels of point lights alone move a light-position difference by a
few 1e-4 relative.  ``smooth_mask`` therefore holds out, for the whole check, the
covered pixels where some light has |n.l| or |n.h| below ``tau``; on the remaining
pixels the loss is smooth over the step and the difference converges.
"""
import numpy as np

import oracle
from tests import brute

FIELD = dict(albedo="albedo", roughness="roughness", specular="specular", light_vec="light_vec",
             light_intensity="light_intensity", exposure="exposure")


def smooth_mask(batch, out, tau=2e-3):
    """uint8 [P]: 1 where the pixel's loss is smooth in every shading parameter."""
    mask = np.ones(int(out["pixel_offset"][-1]), np.uint8)
    po = out["pixel_offset"]
    for f in range(batch.n_frames):
        W, H = int(batch.width[f]), int(batch.height[f])
        n = oracle.frame_view(out["normal"], po, f, W, H, 3).reshape(3, -1).T
        z = out["depth"][po[f]:po[f + 1]]
        p = brute.pixel_rays(batch, f) * z[:, None]
        v = -p / np.maximum(np.linalg.norm(p, axis=1, keepdims=True), 1e-300)
        s = int(batch.frame_scene[f])
        V = batch.view[f].astype(np.float64)
        bad = np.zeros(W * H, bool)
        for l in range(batch.scene_light_begin[s], batch.scene_light_begin[s + 1]):
            u = np.asarray(batch.light_vec[l], np.float64)
            if batch.light_type[l] == 0:
                d = (V[:, :3] @ u + V[:, 3]) - p
            else:
                d = np.broadcast_to(-(V[:, :3] @ u), p.shape)
            d = d / np.linalg.norm(d, axis=1, keepdims=True)
            hh = d + v
            hh = hh / np.maximum(np.linalg.norm(hh, axis=1, keepdims=True), 1e-300)
            bad |= (np.abs((n * d).sum(1)) < tau) | (np.abs((n * hh).sum(1)) < tau)
        mask[po[f]:po[f + 1]] = ~(bad & (z > 0))
    return mask


def perturbed(batch, name, index, delta):
    arr = np.array(getattr(batch, FIELD[name]), np.float64)
    arr.reshape(-1)[index] += delta
    return batch.replace(**{FIELD[name]: arr})


def central_difference(batch, target, name, index, h=1e-4, mask=None):
    lp = oracle.loss(perturbed(batch, name, index, h), target, mask)
    lm = oracle.loss(perturbed(batch, name, index, -h), target, mask)
    return (lp - lm) / (2 * h)
