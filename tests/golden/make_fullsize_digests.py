"""Writes fullsize_digests.json: digests of the diagrams of the full-size
workloads, computed once on the CPU with oracle/ only (the oracle pipeline
and the brute-force union-find checkers) on fields from synthfields.

For each workload it stores the sha256 of the generated float32 field (so a
test can tell that it regenerated the same input) and, as counts plus sha256
digests of little-endian int64 arrays:

* ``oracle``: the oracle's pair lists D0, D1, D2 (simplex ids, the canonical
  order dms_diagram returns), where the sequential oracle finishes in
  minutes;
* ``kruskal_d0``: D0 of the whole lexicographic filtration in vertex-order
  space (rank of the birth's highest vertex, rank of the death's highest
  vertex), pairs of positive persistence, sorted -- Kruskal's union-find over
  every edge (Sec. 5.1; PairSimplices in dimension 0, Sec. 2.5);
* ``dual_d2``: D2 in the same space from the dual union-find over every
  triangle and tetrahedron with an outside node (Sec. 5.2).

Usage: python tests/golden/make_fullsize_digests.py [--jobs N]
Takes about half an hour on 8 cores and needs about 40 GB of memory.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# name -> (generator, grid shape [nz, ny, nx], generator arguments, which digests)
WORKLOADS = {
    "smooth256": ("gaussians", (256, 256, 256), dict(seed=0, k=32, noise_frac=0.01), ("oracle", "kruskal_d0", "dual_d2")),
    "noise128": ("noise", (128, 128, 128), dict(seed=0), ("oracle", "kruskal_d0", "dual_d2")),
    "noise256": ("noise", (256, 256, 256), dict(seed=0), ("oracle",)),
    "smooth512": ("gaussians", (512, 512, 512), dict(seed=0, k=64, noise_frac=0.005), ("kruskal_d0", "dual_d2")),
    "noise512": ("noise", (512, 512, 512), dict(seed=0), ("kruskal_d0", "dual_d2")),
}


def digest(a: np.ndarray) -> dict:
    a = np.ascontiguousarray(a, dtype="<i8")
    return {"n": int(a.shape[0]), "sha256": hashlib.sha256(a.tobytes()).hexdigest()}


def field_of(name):
    import synthfields as sf
    kind, shape, kw, _ = WORKLOADS[name]
    return getattr(sf, kind)(shape, **kw)


def task(args):
    name, what = args
    import oracle
    t = time.time()
    f = field_of(name)
    out = {}
    if what == "field":
        kind, shape, kw, _ = WORKLOADS[name]
        out = {"sha256": hashlib.sha256(np.ascontiguousarray(f).tobytes()).hexdigest(), "shape": list(f.shape),
               "generator": f"synthfields.{kind}{tuple(shape)}, {kw}"}
    elif what == "oracle":
        res = oracle.run(f)
        out = {f"d{d}": digest(res.pairs[d]) for d in range(3)}
        out["n_crit"] = [int(len(c)) for c in res.crit]
    else:
        rank = oracle.vertex_order(f)
        del f
        shape = WORKLOADS[name][1]
        pairs = oracle.bf_d0_kruskal(shape, rank) if what == "kruskal_d0" else oracle.bf_d2_dual(shape, rank)
        out = digest(pairs)
    print(f"[golden] {name} {what} done in {time.time() - t:.0f} s", flush=True)
    return name, what, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("--only", default="", help="comma-separated workload names")
    args = ap.parse_args()
    import oracle
    oracle.build(force=False)
    names = [n for n in WORKLOADS if not args.only or n in args.only.split(",")]
    tasks = [(n, "field") for n in names] + [(n, w) for n in names for w in WORKLOADS[n][3]]
    # the longest first
    cost = {"oracle": 3, "dual_d2": 2, "kruskal_d0": 1, "field": 0}
    tasks.sort(key=lambda t: (-("512" in t[0]), -cost[t[1]]))
    path = os.path.join(HERE, "fullsize_digests.json")
    result = json.load(open(path)) if os.path.exists(path) else {}
    with ProcessPoolExecutor(max_workers=args.jobs) as pool:
        for name, what, out in pool.map(task, tasks):
            result.setdefault(name, {})[what] = out
    with open(path, "w") as fh:
        json.dump(result, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
