"""GPU parity of spot lights with shadow maps (Sec. 5: the benchmark scene's spot lights
with soft shadows; Sec. 4.3.1: spotlight angles): the shadow frames are rendered by the
same kernels (depth only) before the frames, and shading filters them 3 x 3.  Compared
with the oracle at the parity bar on every pixel whose shadow decisions are not inside
the oracle's reporting band; bit-identical across tunings and through a graph."""
import numpy as np
import pytest

import oracle
from paper_1906_11633_amd import _lib as L
from paper_1906_11633_amd import scenes as S
from tests import parity
from tests.test_oracle_shadows import _scene

pytestmark = pytest.mark.gpu

TUNINGS = [None, (32, 32, 256, 0, 1), (32, 32, 512, 0, 2)]
IDS = ["frame-path", "tiled", "one-launch"]


@pytest.fixture(scope="module")
def renderer():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    assert torch.cuda.is_available()
    return Renderer(0)


def _render(renderer, batch, tuning=None):
    import torch
    job = renderer.prepare(batch)
    if tuning is not None:
        job.layout.set_tuning(*tuning)
    print(f"[shadows] {batch.name} frames={batch.n_frames} tuning={job.layout.info.tuning.as_tuple()}", flush=True)
    out = renderer.render(job, tri_id=True, stats=True)
    torch.cuda.synchronize()
    return parity.to_numpy(out), job


@pytest.mark.parametrize("tuning", TUNINGS, ids=IDS)
def test_occluder_under_spot_light(renderer, tuning):
    b = _scene(occluder=True)
    gpu, _ = _render(renderer, b, tuning)
    st = parity.compare(b, gpu, oracle.render(b))
    print(st, flush=True)
    assert st["covered"] > 5000 and st["shadow_amb_frac"] < 0.05
    assert int(gpu["stats"][0]) == 0


@pytest.mark.parametrize("tuning", TUNINGS, ids=IDS)
def test_hand_scenes_three_spot_lights(renderer, tuning):
    """Hand scenes lit by three shadow-casting spot lights each (LightSetup placement,
    randomized angles and intensities)."""
    b = S.with_spot_lights(S.config2(2, 3, 200), seed=7)
    gpu, _ = _render(renderer, b, tuning)
    ref = oracle.render(b)
    st = parity.compare(b, gpu, ref)
    print(st, flush=True)
    assert st["covered"] > 10000
    # the shadows matter: rendering the same lights as unshadowed point lights differs
    free = oracle.render(b.replace(light_type=np.zeros_like(b.light_type)))
    assert np.abs(free["rgb"] - ref["rgb"]).max() > 0.05


def test_spot_lights_bit_identical_across_tunings_and_graph(renderer):
    import torch
    from paper_1906_11633_amd.renderer import Graph
    b = S.with_spot_lights(S.config3(3, 6, max_tris=20000), seed=3, target=(0.0, 0.0, 0.0))
    base, _ = _render(renderer, b)
    for t in TUNINGS[1:]:
        o, _ = _render(renderer, b, t)
        for k in ("rgb", "depth", "normal", "seg", "tri_id"):
            assert np.array_equal(o[k], base[k]), (t, k)
    job = renderer.prepare(b)
    out = renderer.alloc_outputs(job)
    stream = torch.cuda.Stream()
    g = Graph(renderer.ctx, job.layout, job.state, out, job.workspace, stream)
    for _ in range(3):
        g.replay(stream)
        stream.synchronize()
        _ = torch.randn(1000, device="cuda").sum().item()
        assert np.array_equal(out["rgb"].cpu().numpy(), base["rgb"])
    g.close()
    parity.compare(b, base, oracle.render(b))


def test_backward_refuses_spot_lights(renderer):
    import torch
    from paper_1906_11633_amd.renderer import shade_backward
    b = _scene(occluder=False)
    job = renderer.prepare(b)
    out = renderer.render(job, vis=True)
    torch.cuda.synchronize()
    with pytest.raises(L.OrrbError) as e:
        shade_backward(renderer.ctx, job.layout, job.state, out["vis"], torch.zeros_like(out["rgb"]))
    assert e.value.status == 5
