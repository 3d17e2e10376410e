"""GPU parity on the edge cases the oracle's own pins cover: directional lights seen
through a rotated camera, triangles discarded by the near plane and by the guard
band, and the per-call counters the kernels report; plus the graph-after-retune rule
of the boundary.  Every case runs through the C ABI and is compared with the FP64
oracle at the parity bar."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import scenes as S
from tests import parity
from tests.test_oracle_edge_cases import GUARD, MIRROR_U, directional_batch, guard_batch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def renderer():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    assert torch.cuda.is_available()
    return Renderer(0)


def _render(renderer, batch, tuning=None):
    import torch
    from paper_1906_11633_amd.renderer import read_stats
    job = renderer.prepare(batch)
    if tuning is not None:
        job.layout.set_tuning(*tuning)
    out = renderer.render(job, tri_id=True, vis=True, stats=True)
    torch.cuda.synchronize()
    stats = read_stats(out.pop("stats"))
    return parity.to_numpy(out), job, stats


def _check(renderer, batch, tuning=None):
    gpu, job, st = _render(renderer, batch, tuning)
    res = parity.compare(batch, gpu, oracle.render(batch))
    print(batch.name, tuning, res, st, flush=True)
    assert st["wait_timeouts"] == 0
    return res, st


def _cull_counts(batch):
    """FP64 count of the vertex instances nearer than the near plane and of those whose
    snapped coordinate leaves the +-2^24 guard band (visible objects only), written
    from the rule's definition."""
    near = guard = 0
    for f in range(batch.n_frames):
        s = batch.frame_scene[f]
        V = batch.view[f].astype(np.float64)
        fx, fy, cx, cy = batch.intr[f].astype(np.float64)
        for o in range(batch.scene_object_begin[s], batch.scene_object_begin[s + 1]):
            if not batch.object_visible[o]:
                continue
            P = batch.object_pose[o].astype(np.float64)
            p = batch.meshes[batch.object_mesh[o]].pos.astype(np.float64)
            world = p @ P[:, :3].T + P[:, 3]
            e = world @ V[:, :3].T + V[:, 3]
            w = -e[:, 2]
            is_near = w < float(batch.near[f])
            ok = ~is_near
            X = np.rint(256 * (fx * (e[ok, 0] / w[ok]) + cx))
            Y = np.rint(256 * (-fy * (e[ok, 1] / w[ok]) + cy))
            near += int(is_near.sum())
            guard += int(((np.abs(X) > GUARD) | (np.abs(Y) > GUARD)).sum())
    return near, guard


# ---------------------------------------------------------------------------------
# directional lights through a rotated LookAt camera
# ---------------------------------------------------------------------------------


@pytest.mark.parametrize("k_s,rough,u", [(0.0, 1.0, (0.9, 1.8, -1.3)), (0.6, 0.3, MIRROR_U)])
def test_directional_light_rotated_camera(renderer, k_s, rough, u):
    """The plane of the oracle's world-space closed-form pins, on both paths."""
    b = directional_batch(k_s, rough, u=u)
    for tuning in (None, (16, 16, 256, 0, 1)):
        res, _ = _check(renderer, b, tuning)
        assert res["covered"] > 1000


def test_config1_rotated_cameras(renderer):
    """Config-1 scenes (directional lights, materials) seen from four LookAt cameras
    off the z axis: a transposed view rotation on the light would move every shade."""
    b = S.config1(materials=True)
    rng = np.random.default_rng(41)
    views = []
    for f in range(b.n_frames):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        C = S.look_at_c2w(0.6 * d, np.zeros(3), (0.3, 0.2, 1.0))
        views.append(S.view_from_c2w(C))
    b = b.replace(view=np.asarray(views, np.float32))
    res, _ = _check(renderer, b)
    assert res["covered"] > 1000


# ---------------------------------------------------------------------------------
# near plane and guard band
# ---------------------------------------------------------------------------------


def near_batch():
    """A tessellated floor receding from 4 mm in front of the eye to 1.2 m, plus a
    capsule straddling the near plane: triangles with any vertex nearer than 1 cm are
    discarded whole (no clipping)."""
    floor = S.plane_mesh(24, 24, 0.6, 1.2)
    R = S.rot_axis("x", -1.35)
    pose = S.make_pose(R, (0.0, -0.05, -0.6))
    cap = S.capsule_mesh(0.02, 0.05)
    extra = [(cap, S.make_pose(S.rot_axis("y", 0.4), (0.01, 0.0, -0.012)))]
    return S.single_object_batch(floor, pose, res=(96, 80), extra_objects=extra,
                                 lights=((0, (0.1, 0.3, -0.2), 1.2), (1, (0.3, 0.8, 0.4), 0.6)), spec=0.3, rough=0.4)


def test_near_cull(renderer):
    b = near_batch()
    near, guard = _cull_counts(b)
    assert near > 20  # the cull does fire
    for tuning in (None, (32, 32, 256, 0, 1)):
        res, st = _check(renderer, b, tuning)
        assert res["covered"] > 2000
        assert st["near_vertices"] == near and st["guard_vertices"] == guard


@pytest.mark.parametrize("axis,far_sub,kept", [("x", GUARD, True), ("x", GUARD + 1, False), ("y", GUARD, True),
                                               ("y", GUARD + 1, False), ("x", -70000 * 256, False),
                                               ("y", -60000 * 256, True)])
def test_guard_band_exact_boundary(renderer, axis, far_sub, kept):
    """The oracle's exact guard-band fixtures: a vertex snapped exactly to 2^24 keeps
    its triangle, one sub-pixel beyond discards it."""
    b = guard_batch(axis, far_sub)
    for tuning in (None, (16, 16, 256, 0, 1)):
        gpu, _, st = _render(renderer, b, tuning)
        ref = oracle.render(b)
        parity.compare(b, gpu, ref)
        assert (gpu["tri_id"] >= 0).any() == kept
        assert st["guard_vertices"] == (0 if kept else 1)


def test_guard_band_scene(renderer):
    """Two 40 m strips across the view: the one 3 cm from the eye has its end vertices
    at about 77,000 px (beyond the guard band), so its triangles, which would cover a
    band across the screen centre, are discarded and the cube behind shows; the one at
    6 cm (ends at about 38,000 px) is kept.  Everything matches the oracle."""
    strip = S.plane_mesh(2, 1, 40.0, 0.01)
    extra = [(strip, S.make_pose(np.eye(3), (0.0, 0.015, -0.06))),
             (S.box_mesh(4), S.make_pose(np.eye(3), (0.0, 0.0, -0.4), 0.05))]
    b = S.single_object_batch(strip, S.make_pose(np.eye(3), (0.0, 0.0, -0.03)), res=(128, 96), extra_objects=extra,
                              lights=((0, (0.0, 0.3, -0.3), 1.5),), spec=0.2, rough=0.6)
    near, guard = _cull_counts(b)
    assert guard == 4 and near == 0
    for tuning in (None, (16, 16, 256, 0, 1)):
        res, st = _check(renderer, b, tuning)
        assert st["guard_vertices"] == guard and st["near_vertices"] == near
        gpu, _, _ = _render(renderer, b, tuning)
        segs = set(np.unique(gpu["seg"]).tolist())
        assert segs == {-1, 8, 9}, segs  # the far strip (7) is gone, the near one and the cube remain


# ---------------------------------------------------------------------------------
# per-call counters and the graph rule
# ---------------------------------------------------------------------------------


def test_stats_zero_on_benchmark_scenes(renderer):
    b = S.config2(2, 4, 200)
    _, _, st = _render(renderer, b)
    assert all(v == 0 for v in st.values()), st
    _, _, st = _render(renderer, b, (32, 32, 256, 0, 1))
    assert st["wait_timeouts"] == 0 and st["near_vertices"] == 0 and st["guard_vertices"] == 0


def test_stats_count_frame_path_fallbacks(renderer):
    """The bin-overflow and survivor-overflow scenes of the parity tests are counted."""
    mesh = S.plane_mesh(47, 47, 3.2, 3.2)
    R = S.rot_axis("x", 0.2)
    extra = [(mesh, S.make_pose(R, (0.02, -0.03, -2.2), 1.0)), (mesh, S.make_pose(R.T, (-0.01, 0.02, -2.4), 1.0))]
    b = S.single_object_batch(mesh, S.make_pose(np.eye(3), (0.0, 0.0, -2.0), 1.0), res=(256, 256), extra_objects=extra,
                              lights=((0, (0.3, 0.4, 0.5), 1.5),), spec=0.4, rough=0.5)
    _, _, st = _render(renderer, b)
    assert st["bin_overflow_frames"] == 1 and st["wait_timeouts"] == 0
    mesh = S.plane_mesh(57, 57, 0.7, 0.7)
    b = S.single_object_batch(mesh, S.make_pose(np.eye(3), (0.0, 0.0, -2.0), 1.0), res=(200, 200),
                              lights=((0, (0.3, 0.4, 0.5), 1.5),), spec=0.4, rough=0.5)
    _, _, st = _render(renderer, b)
    assert st["survivor_resetup_frames"] == 1 and st["bin_overflow_frames"] == 0


def test_graph_refused_after_retune_and_mesh_growth(renderer):
    """A captured graph holds the layout's tables and tuning: after set_tuning (which
    rebuilds and may move the tables) or a new mesh in the pool, replay returns
    ORRB_ERR_INVALID_ARGUMENT and launches nothing; a graph captured afterwards
    replays and matches a direct render bit for bit."""
    import torch
    from paper_1906_11633_amd import _lib
    from paper_1906_11633_amd.renderer import Graph
    b = S.config3(3, 4)
    job = renderer.prepare(b)
    out = renderer.alloc_outputs(job)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = Graph(renderer.ctx, job.layout, job.state, out, job.workspace, s)
    with torch.cuda.stream(s):
        g.replay(s)
    s.synchronize()
    job.layout.set_tuning(16, 16, 512, 1, 1)
    for k in out:
        out[k].fill_(7)
    with pytest.raises(_lib.OrrbError) as ei:
        g.replay(s)
    assert ei.value.status == 1
    s.synchronize()
    assert bool((out["seg"] == 7).all())  # nothing was launched
    g.close()
    g2 = Graph(renderer.ctx, job.layout, job.state, out, job.workspace, s)
    g2.replay(s)
    s.synchronize()
    ref = renderer.render(job)
    torch.cuda.synchronize()
    for k in ref:
        assert torch.equal(ref[k], out[k]), k
    renderer.ctx.add_mesh(S.box_mesh(1))
    with pytest.raises(_lib.OrrbError) as ei:
        g2.replay(s)
    assert ei.value.status == 1
    g2.close()
