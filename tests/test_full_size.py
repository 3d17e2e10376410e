"""Parity at the benchmark's full sizes, in the launch configuration the benchmark
times: the 768-frame batch of 256 hand-like scenes x 3 cameras at 200x200 (one
frame-kernel launch, four channels) and the 3,072-frame uneven batch (autotuned tiling,
HIP-graph replay; its frames are claimed at run time, heaviest first).  The oracle renders a seeded sample of whole scenes (always the first
and the last, so the first and last work items of the persistent grid are covered); the
GPU frames of those scenes are cut out of the full-size outputs and compared at the
parity bar."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    assert torch.cuda.is_available()
    return Renderer(0)


def _cut(batch, out: dict, scenes) -> dict:
    """The planar outputs of the given scenes' frames, in the sub-batch's layout."""
    po = np.asarray(batch.pixel_offset, np.int64)
    frames = [f for s in scenes for f in np.nonzero(batch.frame_scene == s)[0]]
    res = {}
    for k, v in out.items():
        flat = v.detach().cpu().numpy().reshape(-1)
        ch = 3 if k in ("rgb", "normal") else 1
        res[k] = np.concatenate([flat[ch * po[f]:ch * po[f + 1]] for f in frames])
    return res


def _sample(n_scenes, k, seed):
    rng = np.random.default_rng(seed)
    mid = rng.choice(np.arange(1, n_scenes - 1), size=k, replace=False)
    return [0, *sorted(int(s) for s in mid), n_scenes - 1]


def _check(batch, out, scenes):
    sub = batch.select_scenes(scenes)
    stats = parity.compare(sub, _cut(batch, out, scenes), oracle.render(sub))
    print(batch.name, scenes, stats, flush=True)
    return stats


def test_config2_full_size_sampled(renderer):
    import torch
    b = S.config2(2, 256, 200)
    job = renderer.prepare(b)
    assert job.layout.info.frame_path_frames == b.n_frames  # the timed kernel
    assert job.layout.info.render_kernels == 1  # a uniform batch: static schedule, no counter
    out = renderer.alloc_outputs(job)
    for _ in range(2):  # a second launch over the same buffers, as in the timed loop
        renderer.render(job, out)
    torch.cuda.synchronize()
    st = _check(b, out, _sample(256, 4, 11))
    assert st["covered"] > 10000
    assert renderer.ctx.wait_timeouts() == 0  # no frame-kernel wait reached its bound


def test_uneven_full_size_sampled(renderer):
    import torch
    from paper_1906_11633_amd.renderer import Graph, autotune
    b = S.config3(3, 1024)
    job = renderer.prepare(b)
    out = renderer.alloc_outputs(job)
    autotune(renderer.ctx, job.layout, job.state, out, job.workspace)
    stream = torch.cuda.Stream()
    g = Graph(renderer.ctx, job.layout, job.state, out, job.workspace, stream)
    for _ in range(2):
        g.replay(stream)
    stream.synchronize()
    g.close()
    tris = np.array([b.scene_triangles(s) for s in range(b.n_scenes)])
    scenes = sorted(set(_sample(1024, 3, 12)) | {int(tris.argmax())})
    st = _check(b, out, scenes)
    assert st["covered"] > 1000
    assert renderer.ctx.wait_timeouts() == 0


def test_uneven_full_size_every_frame_once(renderer):
    """The frame kernel's run-time schedule at full size: all 3,072 frames of the uneven
    batch in one frame-kernel launch (tuning path 2), replayed from a graph (the claim
    counter is cleared inside it), are bit-identical to the tiled path's frames, so no
    frame is skipped or rendered twice over another."""
    import torch
    from paper_1906_11633_amd.renderer import Graph
    b = S.config3(3, 1024)
    job = renderer.prepare(b)
    job.layout.set_tuning(32, 32, 512, 0, 2)
    assert job.layout.info.frame_path_frames == b.n_frames and job.layout.info.tile_items == 0
    assert job.layout.info.render_kernels == 2  # counter clear + frame kernel
    out = renderer.alloc_outputs(job, tri_id=True)
    for v in out.values():
        v.fill_(7)  # a frame left out would keep this
    stream = torch.cuda.Stream()
    g = Graph(renderer.ctx, job.layout, job.state, out, job.workspace, stream)
    for _ in range(3):
        g.replay(stream)
        stream.synchronize()
    g.close()
    job.layout.set_tuning(32, 32, 256, 1, 1)
    ref = renderer.render(job, tri_id=True)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "normal", "seg", "tri_id"):
        assert torch.equal(out[k], ref[k]), k
    assert renderer.ctx.wait_timeouts() == 0


def test_config2_full_size_every_frame(renderer):
    """Every frame of the 768-frame batch, in the timed launch configuration, against
    properties that hold at any size: bit-identical to the tiled path (a separate kernel
    with its own binning and schedule, so a frame skipped, rendered twice or written
    into another's pixels shows up); background pixels exactly zero with seg -1; covered
    pixels with finite positive depth, unit normals, non-negative rgb and the seg id of
    one of the frame's scene's objects; and every frame with covered pixels (each camera
    looks at the hand)."""
    import torch
    b = S.config2(2, 256, 200)
    job = renderer.prepare(b)
    assert job.layout.info.frame_path_frames == b.n_frames and job.layout.info.render_kernels == 1
    out = renderer.alloc_outputs(job, tri_id=True)
    for v in out.values():
        v.fill_(7)  # a pixel left unwritten would keep this
    for _ in range(2):
        renderer.render(job, out)
    torch.cuda.synchronize()
    assert renderer.ctx.wait_timeouts() == 0
    job.layout.set_tuning(32, 32, 256, 1, 1)  # the tiled path
    assert job.layout.info.tile_items > 0 and job.layout.info.frame_path_frames == 0
    ref = renderer.render(job, tri_id=True)
    torch.cuda.synchronize()
    for k in ("rgb", "depth", "normal", "seg", "tri_id"):
        assert torch.equal(out[k], ref[k]), k

    po = np.asarray(b.pixel_offset, np.int64)
    depth = out["depth"].cpu().numpy().reshape(-1)
    seg = out["seg"].cpu().numpy().reshape(-1)
    rgb = out["rgb"].cpu().numpy().reshape(-1)
    nrm = out["normal"].cpu().numpy().reshape(-1)
    sob = np.asarray(b.scene_object_begin, np.int64)
    for f in range(b.n_frames):
        n = po[f + 1] - po[f]
        s, d = seg[po[f]:po[f + 1]], depth[po[f]:po[f + 1]]
        c3 = rgb[3 * po[f]:3 * po[f + 1]].reshape(3, n)
        n3 = nrm[3 * po[f]:3 * po[f + 1]].reshape(3, n)
        cov = s >= 0
        assert cov.any(), f
        sc = b.frame_scene[f]
        assert (s >= -1).all() and np.isin(s[cov], b.object_seg[sob[sc]:sob[sc + 1]]).all(), f
        assert (d[~cov] == 0).all() and (c3[:, ~cov] == 0).all() and (n3[:, ~cov] == 0).all(), f
        assert np.isfinite(d[cov]).all() and (d[cov] > 0).all(), f
        assert (c3[:, cov] >= 0).all() and np.isfinite(c3[:, cov]).all(), f
        assert np.abs(np.sqrt((n3[:, cov].astype(np.float64) ** 2).sum(0)) - 1.0).max() < 1e-5, f
