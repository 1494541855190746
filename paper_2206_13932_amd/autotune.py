"""Autotuner of the batched launch: picks the batch tile shape -- the
super-grid cross-section the boxes are packed into, the per-batch vertex
budget and the depth quantum -- and whether the order + gradient kernels are
replayed from a captured graph, by timing a calibration sample of requests
(all arriving at once, so the measured rate is the server's capacity)."""
from __future__ import annotations

import itertools

from . import serving

DEFAULT_SPACE = {
    "cross": [(0, 0), (256, 256)],
    "budget_vertices": [1 << 23, 1 << 25, 1 << 26],
    "z_quantum": [16],
    # graph replay with one worker, or two overlapping workers without it
    "workers_graph": [(1, True), (2, False), (3, False)],
}


def autotune(requests, space=None, device: int = 0, repeats: int = 1, rate: float | None = None,
             headroom: float = 1.5):
    """requests: serving.Request list (their arrival times are ignored).
    Without a rate, picks the configuration of highest capacity. With the
    expected arrival rate (requests/s), picks the smallest per-batch vertex
    budget -- the shortest batches, hence the lowest latency -- among the
    configurations whose capacity is at least headroom x rate (the highest
    capacity if none is), ties broken by capacity.
    Returns (chosen ServerConfig, [(config dict, requests/s)])."""
    space = space or DEFAULT_SPACE
    keys = list(space)
    table = []
    configs = []
    for values in itertools.product(*(space[k] for k in keys)):
        kw = dict(zip(keys, values))
        workers, use_graph = kw.pop("workers_graph")
        cfg = serving.ServerConfig(workers=workers, use_graph=use_graph, **kw)
        server = serving.Server(cfg, device)
        try:
            server_rate = 0.0
            for _ in range(repeats + 1):  # the first run warms the context up
                reqs = [serving.Request(r.rid, 0.0, r.host_field) for r in requests]
                server_rate = server.run_trace(reqs).req_per_s
        finally:
            server.close()
        table.append((dict(zip(keys, values)), server_rate))
        configs.append((cfg, server_rate))
    best = max(configs, key=lambda cc: cc[1])
    if rate is not None:
        ok = [cc for cc in configs if cc[1] >= headroom * rate]
        if ok:
            best = min(ok, key=lambda cc: (cc[0].budget_vertices, -cc[1]))
    return best[0], table
