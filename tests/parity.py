"""GPU-vs-oracle comparison at the stated tolerances (test helper).

Bar (per frame, every pixel):
  * coverage, triangle ID and segmentation bit-exact on every pixel that is not a
    near-tie (the oracle's two nearest fragments within 1e-5 relative depth);
  * depth within 1e-5 relative, RGB and normal within 1e-4 absolute on those pixels;
  * background pixels exactly 0 / -1.
Near-tie pixels may legitimately resolve to either fragment; their fraction of
covered pixels is reported.
"""
from __future__ import annotations

import numpy as np

import oracle

DEPTH_RTOL = 1e-5
RGB_ATOL = 1e-4
NORMAL_ATOL = 1e-4


def to_numpy(out: dict) -> dict:
    return {k: v.detach().cpu().numpy() for k, v in out.items()}


def compare(batch, gpu: dict, ref: dict, strict: bool = True) -> dict:
    """Compare planar GPU outputs (numpy) with oracle outputs; returns statistics and,
    if strict, asserts the bar.  With spot lights, the RGB of pixels the oracle reports
    as shadow-ambiguous (a shadow-map texel choice or depth comparison inside its
    reporting band, where FP64 and fp32 may legitimately decide differently) is not
    compared; their fraction is reported."""
    tie = oracle.near_tie(ref)
    cov_ref = ref["tri_id"] >= 0
    ok = ~tie
    stats = dict(pixels=int(cov_ref.size), covered=int(cov_ref.sum()), near_tie=int(tie.sum()))
    stats["near_tie_frac"] = stats["near_tie"] / max(stats["covered"], 1)
    tri = gpu.get("tri_id")
    seg = gpu["seg"]
    stats["seg_mismatch"] = int((seg[ok] != ref["seg"][ok]).sum())
    if tri is not None:
        stats["tri_mismatch"] = int((tri[ok] != ref["tri_id"][ok]).sum())
    cov_gpu = seg >= 0
    stats["coverage_mismatch"] = int((cov_gpu[ok] != cov_ref[ok]).sum())
    both = ok & cov_ref & cov_gpu
    d_err = np.abs(gpu["depth"][both] - ref["depth"][both]) / ref["depth"][both]
    stats["depth_max_rel"] = float(d_err.max()) if d_err.size else 0.0
    P = cov_ref.size
    rgb_g = gpu["rgb"].reshape(-1)
    nrm_g = gpu["normal"].reshape(-1)
    # planar channel c of frame f sits at 3*off_f + c*HW_f + p; build the per-pixel index
    po = ref["pixel_offset"]
    idx3 = np.empty((3, P), np.int64)
    for f in range(len(po) - 1):
        n = po[f + 1] - po[f]
        base = 3 * po[f] + np.arange(n)
        for c in range(3):
            idx3[c, po[f]:po[f + 1]] = base + c * n
    amb = ref.get("shadow_amb")
    ok_rgb = ok if amb is None else ok & (amb == 0)
    stats["shadow_amb_frac"] = 0.0 if amb is None else float(amb[cov_ref].mean()) if cov_ref.any() else 0.0
    rgb_err = np.abs(rgb_g[idx3] - ref["rgb"][idx3])[:, ok_rgb]
    nrm_err = np.abs(nrm_g[idx3] - ref["normal"][idx3])[:, ok]
    stats["rgb_max_abs"] = float(rgb_err.max()) if rgb_err.size else 0.0
    stats["normal_max_abs"] = float(nrm_err.max()) if nrm_err.size else 0.0
    stats["rgb_fail"] = int((rgb_err > RGB_ATOL).any(0).sum())
    stats["normal_fail"] = int((nrm_err > NORMAL_ATOL).any(0).sum())
    bg = ~cov_ref & ok
    stats["background_nonzero"] = int((gpu["depth"][bg] != 0).sum() + (rgb_g[idx3][:, bg] != 0).sum()
                                      + (nrm_g[idx3][:, bg] != 0).sum() + (seg[bg] != -1).sum())
    if strict:
        assert stats["coverage_mismatch"] == 0, stats
        assert stats["seg_mismatch"] == 0, stats
        assert stats.get("tri_mismatch", 0) == 0, stats
        assert stats["depth_max_rel"] <= DEPTH_RTOL, stats
        assert stats["rgb_fail"] == 0, stats
        assert stats["normal_fail"] == 0, stats
        assert stats["background_nonzero"] == 0, stats
    return stats
