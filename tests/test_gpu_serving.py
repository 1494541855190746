"""Serving: a Poisson trace of mixed-size requests through the continuous-
batching server. Every request's diagram must be the one it has alone, the
server must have formed several batches with more than one request, and
batches of the two workers must have overlapped in time."""
import numpy as np
import pytest

import oracle
import synthfields as sf


@pytest.mark.gpu
@pytest.mark.parametrize("workers,use_graph", [(2, False), (1, True)])
def test_served_results_equal_alone(workers, use_graph):
    import torch
    from paper_2206_13932_amd import dms, serving
    specs = sf.serving_requests(96, seed=7, side_range=(6, 40), rate=3000.0)
    fields = [sf.gaussians(shape, seed, 4, 0.01) for _, shape, seed in specs]
    reqs = serving.make_requests(specs, fields)
    cfg = serving.ServerConfig(workers=workers, budget_vertices=1 << 18, use_graph=use_graph)
    server = serving.Server(cfg)
    stats = server.run_trace(reqs)
    server.close()
    print(f"[serving] {len(stats.batches)} batches, {stats.req_per_s:.0f} req/s, "
          f"p50 {stats.pct(50):.2f} ms, p99 {stats.pct(99):.2f} ms", flush=True)
    assert len(stats.batches) >= 3
    assert max(b[1] for b in stats.batches) > 1
    assert {b[0] for b in stats.batches} == set(range(workers))
    assert np.isfinite(stats.latencies_ms).all() and (stats.latencies_ms > 0).all()
    if workers > 1:
        # batches of different workers ran at the same time (their calls
        # overlapped on the host while both were in flight on the device)
        spans = [(b[0], b[5], b[6]) for b in stats.batches]
        assert any(wa != wb and sa < eb and sb < ea for wa, sa, ea in spans for wb, sb, eb in spans), spans
    ctx = dms.Context(0)
    for r in reqs:
        alone = ctx.diagram(r.host_field.cuda())
        for d in range(3):
            assert torch.equal(r.result[d], alone[d]), (r.rid, d)
    ctx.close()
    # and a sample of the served results against the oracle
    for r in reqs[::8]:
        res = oracle.run(r.host_field.numpy())
        for d in range(3):
            assert np.array_equal(r.result[d].cpu().numpy(), res.pairs[d]), (r.rid, d)
