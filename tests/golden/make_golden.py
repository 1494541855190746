"""Writes the derived golden fixtures of this folder (closed forms only)."""
import itertools
import json
import os


def counts(nx, ny, nz):
    n = (nx, ny, nz)
    E = sum(
        (n[0] - d[0]) * (n[1] - d[1]) * (n[2] - d[2])
        for d in itertools.product((0, 1), repeat=3) if any(d)
    )
    cubes = (nx - 1) * (ny - 1) * (nz - 1)
    T = 2 * ((nx - 1) * (ny - 1) * nz + (nx - 1) * ny * (nz - 1) + nx * (ny - 1) * (nz - 1)) + 6 * cubes
    return [nx * ny * nz, E, T, 6 * cubes]


if __name__ == "__main__":
    grids = [(2, 2, 2), (3, 3, 3), (16, 16, 16), (7, 9, 11), (96, 96, 96), (256, 256, 256), (512, 512, 512)]
    out = {f"{g[0]}x{g[1]}x{g[2]}": counts(*g) for g in grids}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "simplex_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
