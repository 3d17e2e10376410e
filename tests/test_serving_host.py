"""Host-side logic of the serving loop (CPU only): merged batch descriptions and the
Poisson request trace."""
import numpy as np

from paper_1906_11633_amd import scenes as S
from paper_1906_11633_amd.serving import CAMS_PER_SCENE, LIGHTS_PER_SCENE, Request, ScenePool, poisson_trace


def test_merged_batch_description():
    pool = ScenePool(None, 8, device="cpu")
    r1 = Request(0, np.array([3, 1]), 64, 0.0)
    r2 = Request(1, np.array([5]), 200, 0.0)
    desc, oi, li, fi, intr = pool.batch_desc([r1, r2])
    ops = pool.objs_per_scene
    assert desc["n_scenes"] == 3
    assert list(desc["width"]) == [64] * 6 + [200] * 3
    assert np.array_equal(oi[:ops], 3 * ops + np.arange(ops))
    assert np.array_equal(oi[2 * ops:], 5 * ops + np.arange(ops))
    assert np.array_equal(li[:LIGHTS_PER_SCENE], 3 * LIGHTS_PER_SCENE + np.arange(LIGHTS_PER_SCENE))
    assert np.array_equal(fi, np.array([9, 10, 11, 3, 4, 5, 15, 16, 17]))
    np.testing.assert_allclose(intr[0], S.intrinsics(64, 64))
    np.testing.assert_allclose(intr[-1], S.intrinsics(200, 200))
    assert r1.n_frames == 2 * CAMS_PER_SCENE and r1.pixels == 6 * 64 * 64


def test_padded_lights_are_dark():
    """Lights beyond a scene's own are zero-intensity, so they add exactly nothing."""
    pool = ScenePool(None, 8, device="cpu")
    b = S.config2(5, 8, 200)
    li = pool.dev["light_intensity"].numpy().reshape(8, LIGHTS_PER_SCENE)
    for s in range(8):
        n = b.scene_light_begin[s + 1] - b.scene_light_begin[s]
        assert np.all(li[s, n:] == 0) and np.all(li[s, :n] > 0)


def test_poisson_trace_statistics():
    pool = ScenePool(None, 16, device="cpu")
    tr = poisson_trace(pool, rate=2000.0, duration=2.0)
    gaps = np.diff([r.arrival for r in tr])
    assert abs(len(tr) / 2.0 - 2000) < 150
    assert abs(gaps.mean() - 1 / 2000) < 1e-4
    sizes = np.array([len(r.scene_ids) for r in tr])
    assert sizes.min() >= 1 and sizes.max() <= 32
    assert set(r.res for r in tr) <= set(S.C5_RES)
