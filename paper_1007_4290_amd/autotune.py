"""Autotuner of the sweeping solver's tile shapes: the dense leaf size b
and the number of right-hand sides per sweep workgroup (rhs_group).

For one problem (medium, frequency, absorbing layer, right-hand sides and
tolerance), every candidate with compiled kernels is timed on the device,
factorization plus one GMRES solve (or the solve alone), and the fastest is
kept.  The medium, frequency and sources of the trial are the caller's, so
the choice reflects that problem's GMRES iteration count as well as the
kernel times.  Results are cached in a JSON file under a key that holds
everything the timing depends on: n, omega, the PML width, precision, rank,
rank tolerance, GMRES tolerance, the number of right-hand sides, the
objective and a hash of the velocity field.
"""
import hashlib
import json
import os
import time

import numpy as np
import torch

from . import _lib
from .solver import Solver

DEFAULT_LEAVES = (16, 32, 64)
DEFAULT_GROUPS = (1,)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hsweep_autotune.json")


def _key(c, omega, pml, precision, rank, rank_tol, tol, nrhs, objective):
    arr = c.detach().cpu().numpy() if isinstance(c, torch.Tensor) else np.asarray(c)
    h = hashlib.sha1(np.ascontiguousarray(arr, dtype=np.float64).tobytes()).hexdigest()[:16]
    return (f"n={arr.shape[0]}|omega={float(omega):.12g}|pml={int(pml)}|{precision}|r={rank}|rtol={rank_tol:g}"
            f"|tol={tol:g}|nrhs={nrhs}|{objective}|c={h}")


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


def tune(c, omega, pml, f, precision="c64", rank=8, rank_tol=1e-6, tol=1e-6, leaves=DEFAULT_LEAVES,
         groups=DEFAULT_GROUPS, objective="end_to_end", repeats=2, cache=DEFAULT_CACHE, use_cache=True):
    """Return ((leaf, rhs_group), {(leaf, rhs_group): ms}) for this problem.

    objective: "end_to_end" (factor + solve) or "solve" (solve only).
    f: complex128 CUDA tensor of right-hand sides, (nrhs, n*n).
    """
    nrhs = int(f.shape[0]) if f.dim() == 2 else 1
    key = _key(c, omega, pml, precision, rank, rank_tol, tol, nrhs, objective) + \
        f"|leaves={list(leaves)}|groups={list(groups)}"
    table = _load(cache) if (use_cache and cache) else {}
    if key in table:
        ent = table[key]
        return (int(ent["leaf"]), int(ent["rhs_group"])), \
            {tuple(int(x) for x in k.split(",")): v for k, v in ent["ms"].items()}
    results = {}
    for b in leaves:
        for g in groups:
            try:
                s = Solver(c, omega, pml, leaf=b, rank=rank, rank_tol=rank_tol, precision=precision, rhs_group=g)
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
            results[(b, g)] = best
            s.close()
    if not results:
        raise RuntimeError("no leaf size has compiled kernels for this problem")
    choice = min(results, key=results.get)
    if use_cache and cache:
        table[key] = {"leaf": choice[0], "rhs_group": choice[1],
                      "ms": {f"{k[0]},{k[1]}": v for k, v in results.items()}}
        _save(cache, table)
    return choice, results


def tune_leaf(c, omega, pml, f, precision="c64", rank=8, rank_tol=1e-6, tol=1e-6, leaves=DEFAULT_LEAVES,
              objective="end_to_end", repeats=2, cache=DEFAULT_CACHE, use_cache=True):
    """Return (best leaf, {leaf: ms}) for this problem (one right-hand side per workgroup)."""
    (leaf, _), res = tune(c, omega, pml, f, precision, rank, rank_tol, tol, leaves, (1,), objective, repeats,
                          cache, use_cache)
    return leaf, {k[0]: v for k, v in res.items()}


def tune_batch_leaves(problems, precision="c64", rank=8, rank_tol=1e-6, tol=1e-6, leaves=DEFAULT_LEAVES,
                      objective="end_to_end", repeats=1, cache=DEFAULT_CACHE, use_cache=True):
    """Leaf size per grid size for a batch of instances.

    problems: list of (c, omega, pml, f) with f a complex128 CUDA tensor.
    The first instance of each grid size is the trial problem of its size;
    returns ({n: leaf}, {n: {leaf: ms}})."""
    first = {}
    for c, omega, pml, f in problems:
        n = int(np.asarray(c.shape)[0])
        first.setdefault(n, (c, omega, pml, f))
    choice, timings = {}, {}
    for n, (c, omega, pml, f) in sorted(first.items()):
        leaf, ms = tune_leaf(c, omega, pml, f, precision, rank, rank_tol, tol, leaves, objective, repeats,
                             cache, use_cache)
        choice[n] = leaf
        timings[n] = ms
    return choice, timings
