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


def autotune(requests, space=None, device: int = 0, repeats: int = 1):
    """requests: serving.Request list (their arrival times are ignored).
    Returns (best ServerConfig, [(config dict, requests/s)])."""
    space = space or DEFAULT_SPACE
    keys = list(space)
    table = []
    best = None
    for values in itertools.product(*(space[k] for k in keys)):
        kw = dict(zip(keys, values))
        workers, use_graph = kw.pop("workers_graph")
        cfg = serving.ServerConfig(workers=workers, use_graph=use_graph, **kw)
        server = serving.Server(cfg, device)
        try:
            rate = 0.0
            for _ in range(repeats + 1):  # the first run warms the context up
                reqs = [serving.Request(r.rid, 0.0, r.host_field) for r in requests]
                rate = server.run_trace(reqs).req_per_s
        finally:
            server.close()
        table.append((dict(zip(keys, values)), rate))
        if best is None or rate > best[1]:
            best = (cfg, rate)
    return best[0], table
