"""Leaf-size autotuner for the sweeping solver.

For a problem size and precision, every leaf size b that has compiled
kernels is timed on the device (factorization plus one GMRES solve, or the
solve alone), and the fastest is kept.  Results are cached in a JSON file
keyed by (n, precision, rank, objective); timings come from the library's
HIP events.  The medium, frequency and source of the trial are the caller's,
so the choice reflects the GMRES iteration count of that problem too.
"""
import json
import os
import time

import torch

from . import _lib
from .solver import Solver

DEFAULT_LEAVES = (16, 32, 64)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hsweep_autotune.json")


def _key(n, precision, rank, objective):
    return f"n={n}|{precision}|r={rank}|{objective}"


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path, table):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tune_leaf(c, omega, pml, f, precision="c64", rank=8, rank_tol=1e-6, tol=1e-6,
              leaves=DEFAULT_LEAVES, objective="end_to_end", repeats=2, cache=DEFAULT_CACHE,
              use_cache=True):
    """Return (best leaf, {leaf: ms}) for this problem.

    objective: "end_to_end" (factor + solve) or "solve" (solve only).
    f: complex128 CUDA tensor of right-hand sides.
    """
    n = int(c.shape[0])
    key = _key(n, precision, rank, objective)
    table = _load(cache) if (use_cache and cache) else {}
    if key in table:
        return int(table[key]["leaf"]), {int(k): v for k, v in table[key]["ms"].items()}
    results = {}
    for b in leaves:
        try:
            s = Solver(c, omega, pml, leaf=b, rank=rank, rank_tol=rank_tol, precision=precision)
        except _lib.HsweepError:
            continue                      # no kernels for this (leaf, rank, levels)
        best = None
        for rep in range(repeats + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.factor()
            t1 = time.perf_counter()
            s.solve(f, tol=tol, allow_noconv=True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ms = 1e3 * ((t2 - t0) if objective == "end_to_end" else (t2 - t1))
            if rep > 0:                   # the first run includes one-time set-up
                best = ms if best is None else min(best, ms)
        results[b] = best
        s.close()
    if not results:
        raise RuntimeError("no leaf size has compiled kernels for this problem")
    leaf = min(results, key=results.get)
    if use_cache and cache:
        table[key] = {"leaf": leaf, "ms": {str(k): v for k, v in results.items()}}
        _save(cache, table)
    return leaf, results
