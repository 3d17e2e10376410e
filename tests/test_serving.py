"""Continuous-batching server (GPU): results are identical alone and in the mix,
admission by memory queues requests without losing any, and a Poisson run reports
latency percentiles."""
import numpy as np
import pytest

import oracle
from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_1906_11633_amd.renderer import Renderer
    from paper_1906_11633_amd.serving import ScenePool
    assert torch.cuda.is_available()
    r = Renderer(0)
    return r, ScenePool(r.ctx, 24)


def _requests(pool, n, seed=0, max_scenes=8, res=(64, 128, 200)):
    from paper_1906_11633_amd.serving import Request
    rng = np.random.default_rng(seed)
    return [Request(k, rng.integers(0, pool.n_scenes, int(rng.integers(1, max_scenes + 1))), int(rng.choice(res)),
                    0.0) for k in range(n)]


def test_result_alone_equals_in_the_mix(setup):
    import torch
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    reqs = _requests(pool, 10)
    srv = Server(r.ctx, pool, keep_results=True, n_streams=3, max_batch_frames=48)
    st = srv.run(reqs)
    assert st["requests"] == len(reqs)
    assert st["launches"] < len(reqs)  # requests were merged
    torch.cuda.synchronize()
    for q in reqs:
        job = r.prepare(pool.standalone_batch(q))
        alone = r.render(job)
        torch.cuda.synchronize()
        for k in ("rgb", "depth", "normal", "seg"):
            assert torch.equal(alone[k], q.result[k]), (q.rid, k)


def test_served_request_matches_oracle(setup):
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    reqs = _requests(pool, 3, seed=3, max_scenes=2, res=(64,))
    srv = Server(r.ctx, pool, keep_results=True)
    srv.run(reqs)
    for q in reqs:
        b = pool.standalone_batch(q)
        gpu = {k: v.cpu().numpy() for k, v in q.result.items()}
        parity.compare(b, gpu, oracle.render(b))


def test_tiny_budget_queues_and_completes(setup):
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    reqs = _requests(pool, 12, seed=1)
    biggest = max(Server(r.ctx, pool).need_bytes(q) for q in reqs)
    srv = Server(r.ctx, pool, budget_bytes=biggest + 1)
    st = srv.run(reqs)
    assert st["requests"] == len(reqs)
    assert srv.used == 0
    assert st["max_inflight"] >= 1
    # with room for one request at a time, admissions follow arrival order
    assert [q.rid for q in sorted(srv.done, key=lambda q: q.t_admit)] == [q.rid for q in reqs]
    with pytest.raises(ValueError):
        Server(r.ctx, pool, budget_bytes=biggest - 1).submit(max(reqs, key=lambda q: Server(r.ctx, pool).need_bytes(q)))


def test_poisson_run_reports_latency(setup):
    from paper_1906_11633_amd.serving import Server, poisson_trace
    r, pool = setup
    trace = poisson_trace(pool, rate=2000.0, duration=0.5, warmup=0.1)
    srv = Server(r.ctx, pool)
    st = srv.run(trace, warmup=0.1)
    print(st)
    assert st["requests"] > 100
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    assert st["frames_per_s"] > 0
