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


def test_large_merged_launches_on_several_streams(setup):
    """Merged launches of more frames than the frame kernel has workgroups, with mixed
    sizes (frames claimed at run time), in flight on several streams at once: every
    request's result equals its render alone."""
    import torch
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    reqs = _requests(pool, 60, seed=7)
    srv = Server(r.ctx, pool, keep_results=True, n_streams=3, max_batch_frames=400)
    st = srv.run(reqs)
    assert st["requests"] == len(reqs)
    assert srv.launches >= 2 and srv.launch_frames / srv.launches > 256
    torch.cuda.synchronize()
    for q in reqs:
        job = r.prepare(pool.standalone_batch(q))
        alone = r.render(job)
        torch.cuda.synchronize()
        for k in ("rgb", "depth", "normal", "seg"):
            assert torch.equal(alone[k], q.result[k]), (q.rid, k)


@pytest.mark.parametrize("res", [64, 128, 200])
def test_served_request_matches_oracle(setup, res):
    """Requests served in a merged launch match the oracle at every config-5 size."""
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    reqs = _requests(pool, 3, seed=3 + res, max_scenes=2, res=(res,))
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
    srv = Server(r.ctx, pool)
    needs = [srv.need_bytes(q) for q in reqs]  # also caches each request's own layout
    srv.budget = max(needs) + srv.table_bytes + (64 << 10)
    st = srv.run(reqs)
    assert st["requests"] == len(reqs)
    assert srv.used == 0
    assert st["max_inflight"] >= 1 and st["wait_timeouts"] == 0
    # admissions follow arrival order
    assert [q.rid for q in sorted(srv.done, key=lambda q: (q.t_admit, q.rid))] == [q.rid for q in reqs]
    big = max(reqs, key=srv.need_bytes)
    with pytest.raises(ValueError):
        Server(r.ctx, pool, budget_bytes=srv.need_bytes(big) - 1).submit(big)


def test_budget_binds_on_workspace(setup):
    """On the tiled path a launch needs 16 B of workspace per vertex instance: the
    budget counts it, so a budget that holds every request's outputs and state but not
    its workspace refuses the request, and one that holds a single request with its
    workspace runs the requests one launch at a time, with the same results as the
    frame path."""
    import torch
    from paper_1906_11633_amd.serving import Server
    r, pool = setup
    from paper_1906_11633_amd.serving import Request
    tiled = (32, 32, 256, 0, 1)
    rng = np.random.default_rng(4)
    reqs = [Request(k, rng.integers(0, pool.n_scenes, 2), 64, 0.0) for k in range(6)]  # equal sizes
    srv = Server(r.ctx, pool, tuning=tiled, keep_results=True)
    needs = [srv.need_bytes(q) for q in reqs]
    data = [srv.data_bytes(q) for q in reqs]
    assert all(n - d >= 3 * 6936 * 16 for n, d in zip(needs, data))  # the workspace is counted
    big = reqs[int(np.argmax(needs))]
    with pytest.raises(ValueError):
        Server(r.ctx, pool, budget_bytes=max(data) + (64 << 10), tuning=tiled).submit(big)
    srv.budget = max(needs) + srv.table_bytes + (64 << 10)
    smallest_pair = sorted(needs)[0] + sorted(needs)[1]
    assert srv.budget < smallest_pair  # no two requests fit together
    st = srv.run(reqs)
    assert st["requests"] == len(reqs) and st["max_inflight"] == 1 and srv.used == 0
    assert st["launches"] == len(reqs) and st["wait_timeouts"] == 0
    torch.cuda.synchronize()
    for q in reqs:
        job = r.prepare(pool.standalone_batch(q))
        alone = r.render(job)
        torch.cuda.synchronize()
        for k in ("rgb", "depth", "normal", "seg"):
            assert torch.equal(alone[k], q.result[k]), (q.rid, k)


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
