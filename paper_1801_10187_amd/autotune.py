"""Tile-shape tuning by measurement.

The paper tunes its kernels' launch parameters by timing them on the
hardware (sec. 3.5: the threads per cell and block sizes of each kernel,
chosen from short timed runs). The step kernel here has one such parameter,
the tile shape (the cells a block collides together: 4x4x2, 4x4x4, 8x4x4 or
8x8x4), which the library chooses from the mean density unless told
otherwise. `tune` times every shape on a box of the given density and
settings and returns the fastest, caching the answer per device and
settings in a JSON file; `sweep` tabulates all shapes against the density
rule's choice. Run `python -m paper_1801_10187_amd.autotune` for the table.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import binding

SHAPES = list(binding.TILE_SHAPES)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mpcd_tiles.json")


def rule_shape(density, single=True, collision=binding.SRD, precision=binding.FP32):
    """The library's own choice (MPCD_TILE_* 0) for a mean density: a box
    alone or a box of a batch, SRD or AT rule, FP32 or FP64 form."""
    if density >= 12.0:
        return "4x4x2"
    if not single:
        return "4x4x4" if density >= 3.5 else ("8x4x4" if density >= 1.75 else "8x8x4")
    if collision == binding.AT and precision == binding.FP64:
        return "4x4x4" if density >= 2.5 else "8x8x4"
    return "4x4x4" if density >= 7.5 else ("8x4x4" if density >= 3.75 else "8x8x4")


def _fluid(n_cells, density, kT, seed):
    rng = np.random.default_rng(seed)
    L = np.array(n_cells, dtype=np.float64)
    n = int(round(density * np.prod(n_cells)))
    pos = rng.random((n, 3)) * L
    pos = np.where(pos >= L, 0.0, pos)
    vel = rng.normal(size=(n, 3)) * np.sqrt(kT)
    return pos, vel - vel.mean(axis=0)


def measure(shape, density, precision=binding.FP32, thermostat=True, collision=binding.SRD,
            n_cells=(64, 64, 64), steps=100, warmup=10, seed=1, inp=None):
    """Milliseconds per step of one `steps`-step call on a box of `n_cells`
    at `density`, tiles of `shape` (None: the density rule)."""
    import torch
    pos, vel = inp if inp is not None else _fluid(n_cells, density, 1.0, seed)
    with binding.Sim(pos, vel, n_cells, seed=seed, precision=precision, thermostat=thermostat,
                     collision=collision, tile=shape) as s:
        s.step(warmup)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.sync()
        t1 = time.perf_counter()
    return 1e3 * (t1 - t0) / steps


def _key(density, precision, thermostat, collision):
    import torch
    dev = torch.cuda.get_device_name(0)
    return f"{dev}|rho={density:g}|prec={precision}|thermo={int(bool(thermostat))}|rule={collision}"


def tune(density, precision=binding.FP32, thermostat=True, collision=binding.SRD,
         cache=DEFAULT_CACHE, repeats=2, **kw):
    """The fastest tile shape for boxes of this mean density and settings:
    from the cache if present, else timed (each shape `repeats` times, the
    best time counts) and stored."""
    key = _key(density, precision, thermostat, collision)
    table = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if key in table:
        return table[key]["best"]
    pos_vel = _fluid(kw.get("n_cells", (64, 64, 64)), density, 1.0, kw.get("seed", 1))
    times = {sh: min(measure(sh, density, precision, thermostat, collision, inp=pos_vel, **kw)
                     for _ in range(repeats)) for sh in SHAPES}
    best = min(times, key=times.get)
    table[key] = {"best": best, "ms_per_step": times}
    if cache:
        os.makedirs(os.path.dirname(cache) or ".", exist_ok=True)
        with open(cache, "w") as f:
            json.dump(table, f, indent=1)
    return best


def sweep(densities, precision=binding.FP32, thermostat=True, collision=binding.SRD,
          repeats=2, **kw):
    """Rows (density, {shape: ms/step}, best shape, rule's shape, rule's
    time / best time), every shape timed `repeats` times (best counts)."""
    rows = []
    for rho in densities:
        inp = _fluid(kw.get("n_cells", (64, 64, 64)), rho, 1.0, kw.get("seed", 1))
        t = {sh: min(measure(sh, rho, precision, thermostat, collision, inp=inp, **kw)
                     for _ in range(repeats)) for sh in SHAPES}
        best = min(t, key=t.get)
        rule = rule_shape(rho, True, collision, precision)
        rows.append((rho, t, best, rule, t[rule] / t[best]))
        print(f"[autotune] density {rho:g}: fastest {best}", file=sys.stderr, flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--densities", default="1.5,2.5,3.5,5,7,10,12,15")
    ap.add_argument("--form", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--rule", default="srd", choices=["srd", "at"])
    ap.add_argument("--no-thermostat", action="store_true")
    ap.add_argument("--cells", type=int, default=64, help="box edge in cells")
    ap.add_argument("--steps", type=int, default=100)
    args = ap.parse_args()
    prec = binding.FP32 if args.form == "fp32" else binding.FP64
    coll = binding.AT if args.rule == "at" else binding.SRD
    thermo = not args.no_thermostat and coll == binding.SRD
    rows = sweep([float(x) for x in args.densities.split(",")], prec, thermo, coll,
                 n_cells=(args.cells,) * 3, steps=args.steps)
    print(f"# {args.form} {args.rule} thermostat={thermo} box {args.cells}^3, "
          f"{args.steps}-step calls, ms per step (best of 2)")
    print("| density | " + " | ".join(SHAPES) + " | fastest | rule | rule / fastest |")
    print("|---" * (len(SHAPES) + 4) + "|")
    for rho, t, best, rule, ratio in rows:
        print(f"| {rho:g} | " + " | ".join(f"{t[s]:.4f}" for s in SHAPES) +
              f" | {best} | {rule} | {ratio:.3f} |")
    print(json.dumps({"rows": [{"density": r[0], "ms_per_step": r[1], "fastest": r[2], "rule": r[3],
                                "rule_over_fastest": r[4]} for r in rows]}))


if __name__ == "__main__":
    main()
