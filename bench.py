"""Benchmark: 2D Helmholtz solves/s at relative residual 1e-6, complex64 sweep
(FP64 residual and Arnoldi) beside the complex128 sweep, on one MI355X.

Headline workload (n=255): omega = 2 pi 32 (8 points per wavelength),
velocity c = 1 + 0.3 * smooth Gaussian random field (correlation 0.1, seed 1),
PML 16 points, centre Gaussian source, H-matrix Schur complements with leaf 16
and rank <= 8 at relative tolerance 1e-6.

One step is the whole hot path for one right-hand side with the inputs
already in device memory: stencil coefficients, the layer-by-layer
factorization with H-matrix Schur complements, and flexible GMRES with the
sweep as preconditioner until ||f - A u|| <= 1e-6 ||f||.  `value` is that
end-to-end rate; `solve_phase_solves_per_s` (factorization built once, then
solves only) is reported beside it.

Prints one JSON line.  `roofline` covers the dominant kernel of a step, the
layer kernel of the factorization (one launch per layer: the recompressions of
the off-diagonal blocks and the dense leaves), whose average launch time is
measured with HIP events around each launch on the stream it runs on.  It is
latency bound (chains of small dependent steps on single wavefronts), so it is
reported against the vector FP32 peak ("alu") with its algorithmic flops.
`kernels` gives the fraction of the other kernels of the step (Woodbury,
sweep, stencil, Krylov vector work).  `workloads` measures the other problem
sizes: the n=1023 lens, 64 sources at n=511 (complex64 against complex128
sweeps), a batch of 24 instances of three sizes, and the misfit gradient at
n=511.  `cpu_baseline` times the CPU oracle (sparse LU, the plain definition
u = A^{-1} f) on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3      # MI355X FP32, vector and matrix (256 CUs at 2.4 GHz)
FP64_PEAK_TFLOPS = 78.6
METRIC = "2D Helmholtz solves/s at rel. residual 1e-6: complex64 vs FP64 sweep"
# HBM bytes per launch of layer_kernel<float, 16, 8> on this workload: FETCH_SIZE
# + WRITE_SIZE from two rocprofv3 counter passes, each scaled by what the counter
# reads for a 1 GiB device-to-device copy (profiles/factor_kernels_pmc.md).
# Counters cannot be read inside a timed run; a change to the kernel voids this.
LAYER_KERNEL_HBM_BYTES = 913175 + 98784
# The same passes for the sweep launches (profiles/sweep_kernel_pmc.md), keyed
# by workload; None where not measured for the current kernel.
SWEEP_HBM_BYTES = {"helm255_grf": 64644540 + 1562656, "helm511_grf_64src": 1005177426 + 401348213,
                   "helm511_grf_64src_group4": 703650680 + 401475733}


def e_layer(plan):
    np_, b, L, r = plan["n_p"], plan["b"], plan["levels"], plan["r"]
    return np_ * b + L * r * np_ + ((1 << L) - 1) * 4 * r * r


def sweep_bytes(plan, n, elem, nrhs=1):
    """Algorithmic bytes of one application of M to nrhs fields: every layer's
    factor data read once per layer step (2n-1 steps), the couplings twice,
    the complex128 input and output fields and the forward work vector
    (written, then read) of each right-hand side."""
    np_ = plan["n_p"]
    fac = (2 * n - 1) * e_layer(plan) * elem
    coup = 2 * (n - 1) * np_ * elem
    vec = nrhs * (2 * n * n * 16 + 2 * n * np_ * elem)
    return fac + coup + vec


def sweep_flops(plan, n, nrhs=1):
    """Real flops of one application of M: one complex multiply-add (8 flops)
    per stored factor entry, layer step and right-hand side."""
    return 8.0 * (2 * n - 1) * e_layer(plan) * nrhs


def stencil_bytes(n, nrhs, residual=False):
    """FP64 5-point operator over n^2 points: read x (16 B), write y (16 B),
    read c (8 B); the residual form also reads f (16 B)."""
    return n * n * nrhs * (56 if residual else 40)


def krylov_bytes(n, its_per_cycle, nrhs=1):
    """FP64 vector traffic of the flexible GMRES steps: in step j, two
    Gram-Schmidt passes (inner products over j+1 basis vectors and w, then
    the update reading them and writing w), the norm of w and the scaling
    into the next basis vector."""
    N = n * n
    tot = 0
    for its in its_per_cycle:
        for j in range(its):
            tot += 2 * ((j + 2) + (j + 3)) + 1 + 2
    return 16 * N * nrhs * tot


def layer_kernel_flops(plan, b, r):
    """Algorithmic real flops of one layer-kernel launch (a layer m > 0).

    Per off-diagonal block of a level-lam node pair (2^(lam-1) blocks, s = n_p
    >> lam rows, k = 1 + r*lam stacked columns, kk = min(s, k)): the stacked
    factor D P X (8 lam s r^2), two complex QR factorizations (8 (s k^2 -
    k^3/3) each), the core product (8 kk^2 k), an SVD of the kk x kk core
    (48 kk^3) and the application of both Q factors to r columns (2 * 8 s kk r).
    Per leaf (2^L of them): the update by the ancestors' low-rank terms
    (8 L (b r^2 + b^2 r)) and the Gauss-Jordan inverse (8 b^3)."""
    np_, L = plan["n_p"], plan["levels"]
    total = 0.0
    for lam in range(1, L + 1):
        s = np_ >> lam
        k = 1 + r * lam
        kk = min(s, k)
        blk = 8 * lam * s * r * r + 2 * 8 * (s * k * k - k ** 3 / 3) + 8 * kk * kk * k + 48 * kk ** 3 \
            + 2 * 8 * s * kk * r
        total += (1 << (lam - 1)) * blk
    total += (1 << L) * (8 * L * (b * r * r + b * b * r) + 8 * b ** 3)
    return total


def woodbury_flops(plan, b, r):
    """Algorithmic real flops of the Woodbury launches of one layer: per level
    lam (2^lam nodes of s = n_p >> lam rows) the 2r x 2r core through one r x r
    inverse and five r x r products (48 r^3), P_c = T_c Q_c by the leaves
    (8 s b r) and by each inner level's low-rank correction (16 s r^2 each),
    and G_c = Q_c^t P_c (8 s r^2)."""
    np_, L = plan["n_p"], plan["levels"]
    total = 0.0
    for lam in range(1, L + 1):
        s = np_ >> lam
        total += (1 << lam) * (48 * r ** 3 + 8 * s * b * r + 16 * (L - lam) * s * r * r + 8 * s * r * r)
    return total + 48 * r ** 3


def _frac(achieved, peak):
    return achieved / peak if peak else None


def run_gpu(wl, precision, steps, warmup, tol):
    import torch
    from paper_1007_4290_amd.solver import Solver

    c = wl.velocity()
    f = torch.as_tensor(wl.sources(), device="cuda:0")
    s = Solver(c, wl.omega, wl.pml, leaf=wl.leaf, rank=wl.rank, rank_tol=wl.rank_tol, precision=precision)
    for _ in range(warmup):
        s.factor()
        s.solve(f, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sweep_ms, applies, factor_ms, iters, res, sten_ms, kry_ms = 0.0, 0, 0.0, [], [], 0.0, 0.0
    for _ in range(steps):
        s.factor()
        factor_ms += s.timings()["factor_ms"]
        u, it, rr = s.solve(f, tol=tol)
        tm = s.timings()
        sweep_ms += tm["sweep_ms"]
        sten_ms += tm["stencil_ms"]
        kry_ms += tm["krylov_ms"]
        applies += tm["applies"]
        iters.append(it[0])
        res.append(rr[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel timing of the factorization (plain launches, HIP events)
    s.profile_factor()
    prof = [s.profile_factor() for _ in range(max(1, min(steps, 3)))]
    layer_ms = sum(p["layer_ms"] for p in prof) / sum(p["layers"] for p in prof)
    wood_ms = sum(p["wood_ms"] for p in prof) / len(prof)
    # solve phase alone (factorization reused)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        s.solve(f, tol=tol)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    info = s.plan_info()
    info.update({"b": wl.leaf, "r": wl.rank})
    return {
        "ms_per_step": 1e3 * (t1 - t0) / steps,
        "solve_ms": 1e3 * (t3 - t2) / steps,
        "factor_ms": factor_ms / steps,
        "sweep_ms_avg": sweep_ms / max(applies, 1),
        "stencil_ms_per_solve": sten_ms / steps,
        "krylov_ms_per_solve": kry_ms / steps,
        "layer_kernel_ms_avg": layer_ms,
        "wood_ms_per_factor": wood_ms,
        "iters": iters,
        "relres": max(res),
        "plan": info,
        "u": u.cpu().numpy(),
    }


def _timed_solve(s, F, tol, reps, torch):
    """Median wall time (ms) of `reps` solves, with the library's per-phase
    device times of the last one."""
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, its, res = s.solve(F, tol=tol, maxit=200)
        torch.cuda.synchronize()
        ts.append(1e3 * (time.perf_counter() - t0))
    return float(np.median(ts)), U, its, res, s.timings()


def bench_workloads(tol):
    """The other problem sizes: one warm-up, then medians of timed runs."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver, factor_batch, solve_batch, helmholtz_solve
    from paper_1007_4290_amd import autotune

    out = {}
    # n = 1023 lens, complex64 (one right-hand side)
    wl = W.get("helm1023_lens")
    F = torch.as_tensor(wl.sources(), device="cuda:0")
    s = Solver(wl.velocity(), wl.omega, wl.pml, leaf=wl.leaf, rank=wl.rank, rank_tol=wl.rank_tol, precision="c64")
    s.factor()
    s.solve(F, tol=tol)
    fms = []
    for _ in range(2):
        s.factor()
        fms.append(s.timings()["factor_ms"])
    ms, U, its, res, tm = _timed_solve(s, F, tol, 3, torch)
    plan = dict(s.plan_info(), b=wl.leaf, r=wl.rank)
    sw = tm["sweep_ms"] / max(tm["applies"], 1)
    nb = sweep_bytes(plan, wl.n, 8)
    out["helm1023_lens"] = {
        "n": wl.n, "precision": "c64", "factor_ms": float(np.median(fms)), "solve_ms": ms,
        "solve_phase_solves_per_s": 1e3 / ms, "end_to_end_solves_per_s": 1e3 / (ms + float(np.median(fms))),
        "gmres_iters": its[0], "relres": res[0],
        "sweep": {"avg_launch_ms": sw, "bytes_per_launch": nb, "bound": "hbm",
                  "achieved": nb / (sw * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": _frac(nb / (sw * 1e-3) / 1e9, HBM_PEAK_GBS)},
    }
    print(f"[bench] helm1023: factor {out['helm1023_lens']['factor_ms']:.1f} ms, solve {ms:.1f} ms", file=sys.stderr,
          flush=True)
    del s

    # 64 sources on one n = 511 medium: complex64 (one and four right-hand sides
    # per workgroup) against complex128 sweeps, solve phase
    wl = W.get("helm511_grf_64src")
    F = torch.as_tensor(wl.sources(), device="cuda:0")
    rows = {}
    for prec, grp in (("c64", 1), ("c64", 4), ("c128", 1)):
        s = Solver(wl.velocity(), wl.omega, wl.pml, leaf=wl.leaf, rank=wl.rank, rank_tol=wl.rank_tol,
                   precision=prec, rhs_group=grp)
        s.factor()
        fms = s.timings()["factor_ms"]
        s.solve(F, tol=tol)
        ms, U, its, res, tm = _timed_solve(s, F, tol, 2, torch)
        plan = dict(s.plan_info(), b=wl.leaf, r=wl.rank)
        elem = 8 if prec == "c64" else 16
        sw = tm["sweep_ms"] / max(tm["applies"], 1)
        nb = sweep_bytes(plan, wl.n, elem, nrhs=F.shape[0])
        fl = sweep_flops(plan, wl.n, nrhs=F.shape[0])
        peak_fl = FP32_PEAK_TFLOPS if prec == "c64" else FP64_PEAK_TFLOPS
        rows[f"{prec}_group{grp}"] = {
            "factor_ms": fms, "solve_ms": ms, "solve_phase_solves_per_s": F.shape[0] * 1e3 / ms,
            "gmres_iters_max": max(its), "relres_max": max(res),
            "sweep": {"avg_launch_ms": sw, "bytes_per_launch": nb, "flops_per_launch": fl,
                      "hbm_achieved_GBs": nb / (sw * 1e-3) / 1e9,
                      "hbm_frac": _frac(nb / (sw * 1e-3) / 1e9, HBM_PEAK_GBS),
                      "flop_achieved_TFLOPs": fl / (sw * 1e-3) / 1e12,
                      "flop_frac": _frac(fl / (sw * 1e-3) / 1e12, peak_fl),
                      "traffic": {("c64", 1): SWEEP_HBM_BYTES["helm511_grf_64src"],
                                  ("c64", 4): SWEEP_HBM_BYTES["helm511_grf_64src_group4"]}.get((prec, grp)),
                      "matrix_cores": prec == "c64" and grp == 4},
        }
        print(f"[bench] helm511 64 src {prec} group {grp}: solve {ms:.1f} ms", file=sys.stderr, flush=True)
        del s
    out["helm511_grf_64src"] = {"n": wl.n, "nrhs": int(F.shape[0]), **rows,
                                "c64_over_c128_solve_phase": rows["c64_group1"]["solve_phase_solves_per_s"]
                                / rows["c128_group1"]["solve_phase_solves_per_s"]}

    # mixed batch: 24 instances of n = 127, 255, 511, leaves from the tuner,
    # one factorization batch and one batched FGMRES
    wls = W.configs.mixed_batch()
    trial = [(wl.velocity(), wl.omega, wl.pml, torch.as_tensor(wl.sources(), device="cuda:0")) for wl in wls]
    leaves, tune_ms = autotune.tune_batch_leaves(trial, leaves=(16, 32), repeats=1, use_cache=False)
    solvers = [Solver(wl.velocity(), wl.omega, wl.pml, leaf=leaves[wl.n], rank=8, rank_tol=1e-6, precision="c64")
               for wl in wls]
    fs = [torch.as_tensor(wl.sources()[0], device="cuda:0") for wl in wls]
    factor_batch(solvers)
    solve_batch(solvers, fs, tol=tol)
    fts, sts = [], []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        factor_batch(solvers)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        us, its, res = solve_batch(solvers, fs, tol=tol)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fts.append(1e3 * (t1 - t0))
        sts.append(1e3 * (t2 - t1))
    fm, sm = float(np.median(fts)), float(np.median(sts))
    out["mixed_batch_24"] = {
        "instances": len(wls), "sizes": [127, 255, 511], "leaves": {str(k): v for k, v in leaves.items()},
        "factor_batch_ms": fm, "solve_batch_ms": sm, "solve_phase_solves_per_s": len(wls) * 1e3 / sm,
        "end_to_end_solves_per_s": len(wls) * 1e3 / (fm + sm), "gmres_iters_max": max(its),
        "relres_max": max(res), "tuner_ms": {str(k): v for k, v in tune_ms.items()},
    }
    print(f"[bench] mixed batch: factor {fm:.1f} ms, solve {sm:.1f} ms", file=sys.stderr, flush=True)
    del solvers

    # misfit gradient at n = 511: 32 sources, 256 receivers, adjoint sweep
    wl = W.get("grad511")
    F = torch.as_tensor(wl.sources(), device="cuda:0")
    rec = torch.as_tensor(wl.receivers, device="cuda:0")
    c0 = torch.as_tensor(wl.velocity(), device="cuda:0")
    data = torch.zeros((F.shape[0], rec.numel()), dtype=torch.complex128, device="cuda:0")

    def grad_once():
        c_t = c0.clone().requires_grad_(True)
        u = helmholtz_solve(c_t, F, wl.omega, wl.pml, tol=tol, leaf=32, rank=8, rank_tol=1e-6, precision="c64")
        r = u[:, rec] - data
        J = 0.5 * (r.abs() ** 2).sum()
        J.backward()
        return c_t.grad

    grad_once()
    gts = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grad_once()
        torch.cuda.synchronize()
        gts.append(1e3 * (time.perf_counter() - t0))
    gm = float(np.median(gts))
    out["grad511"] = {"n": wl.n, "sources": int(F.shape[0]), "receivers": int(rec.numel()),
                      "gradient_ms": gm, "gradients_per_s": 1e3 / gm,
                      "note": "setup, factorization, 32 forward and 32 adjoint solves, gradient kernel"}
    print(f"[bench] gradient: {gm:.1f} ms", file=sys.stderr, flush=True)
    out["strong_rank2_127"] = strong_workload(tol)
    out["strong_rank2_lens"] = strong_lens_workload()
    out["threed_strong_rank2_15"] = threed_workload(tol)
    return out


def threed_workload(tol, n=15):
    """The 3D face-by-face sweep (Sec. 4) with rank-2 strongly admissible
    face factors: n = 15 cube, random medium 1 + 0.3 U(0, 1) (seed 13),
    omega = 2 pi 2, layers of 3 points, leaf boxes of 16 face points, a
    centre Gaussian source, complex128."""
    import torch
    from paper_1007_4290_amd.solver import Solver3
    c = 1 + 0.3 * np.random.default_rng(13).random((n, n, n))
    om = 2 * np.pi * 2
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    sg = 1.5 * h
    src = np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2) / (2 * sg * sg)) / (2 * np.pi * sg * sg) ** 1.5
    f = torch.as_tensor(src.ravel().astype(complex), device="cuda:0")
    s = Solver3(c, om, 3, leaf=16, rank=2, rank_tol=1e-6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.factor()
    torch.cuda.synchronize()
    fm = 1e3 * (time.perf_counter() - t0)
    s.solve(f, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, its, res = s.solve(f, tol=tol)
    torch.cuda.synchronize()
    sm = 1e3 * (time.perf_counter() - t0)
    print(f"[bench] 3D n = {n}: factor {fm:.0f} ms, solve {sm:.1f} ms, its {its}", file=sys.stderr, flush=True)
    return {"n": n, "omega": "2pi*2", "pml": 3, "leaf": 16, "rank": 2, "precision": "c128", "factor_ms": fm,
            "solve_ms": sm, "gmres_iters": its, "relres": res, "factor_bytes": s.plan_info()["factor_bytes"],
            "note": "face factorization walks the block recursion from the host (the strong-format kernels of "
                    "the 2D layers on quadtree face clusters; latency bound)"}


def strong_workload(tol, n=127):
    """Strongly admissible rank-2 factors (the paper's setting) on the n = 127
    random medium (omega = 2 pi 16, 8 points per wavelength, layers of 12
    points, leaf 16, complex128), beside the weak rank-8 complex128 factors
    of the same problem."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver
    leaf, q = (16, n // 8 + 1) if n >= 127 else (8, 8)
    c = W.random_field_medium(n, 1)
    om = 2 * np.pi * q
    pml = 12
    f = torch.as_tensor(W.gaussian_source(n, (0.5, 0.5)).reshape(1, -1).astype(complex), device="cuda:0")
    row = {"n": n, "omega": f"2pi*{q}", "leaf": leaf, "precision": "c128"}
    for adm, rank in (("strong", 2), ("weak", 8)):
        s = Solver(c, om, pml, leaf=leaf, rank=rank, rank_tol=1e-6, precision="c128", admissibility=adm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factor()
        torch.cuda.synchronize()
        fm = 1e3 * (time.perf_counter() - t0)
        s.solve(f, tol=tol)
        ms, U, its, res, tm = _timed_solve(s, f, tol, 2, torch)
        _, its10, _ = s.solve(f, tol=1e-10)
        row[f"{adm}_rank{rank}"] = {"factor_ms": fm, "solve_ms": ms, "gmres_iters": its[0],
                                    "gmres_iters_at_1e-10": its10[0], "relres": res[0],
                                    "factor_bytes": s.plan_info()["factor_bytes"],
                                    "end_to_end_solves_per_s": 1e3 / (fm + ms)}
        print(f"[bench] {adm} rank {rank}, n = {n}: factor {fm:.0f} ms, solve {ms:.1f} ms, its {its[0]}",
              file=sys.stderr, flush=True)
        del s
    row["note"] = ("strong factorization: the host walks the block recursion; each recompression is one "
                   "wavefront (two QRs, core SVD, kept columns; a walk's recompressions in one launch), "
                   "H-matrix products one launch per class of leaf blocks with disjoint rows; bound by the "
                   "latency of that dependent chain")
    return row


# The paper's lens rows with strongly admissible rank-2 factors (T_setup,
# GMRES iterations and T_solve of its first right-hand side at tolerance
# 1e-3, on its 2010 CPU): context only, the media and hardware differ.
PAPER_LENS_STRONG = {255: (5.05, 2, 0.25), 511: (34.4, 3, 1.45)}


def strong_lens_factor(n):
    """One strongly admissible rank-2 factorization of the lens workload of
    strong_lens_workload at size n, timed."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver
    s = Solver(W.lens_medium(n), 2 * np.pi * ((n + 1) // 8), 16, leaf=16, rank=2, rank_tol=1e-6, precision="c128",
               admissibility="strong")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.factor()
    torch.cuda.synchronize()
    print(f"[bench] strong rank 2 lens, n = {n}: factor {1e3 * (time.perf_counter() - t0):.0f} ms", file=sys.stderr,
          flush=True)


def strong_lens_workload(sizes=(255, 511)):
    """Strongly admissible rank-2 factors at the paper's lens sizes: the lens
    medium, 8 points per wavelength (omega = 2 pi (n + 1) / 8), layers of 16
    points, leaf 16, complex128, a Gaussian point source at (0.5, 0.125);
    GMRES to 1e-3 (the paper's tolerance) and to 1e-6."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver
    rows = {}
    for n in sizes:
        q = (n + 1) // 8
        c = W.lens_medium(n)
        om = 2 * np.pi * q
        f = torch.as_tensor(W.gaussian_source(n, (0.5, 0.125)).reshape(1, -1).astype(complex), device="cuda:0")
        s = Solver(c, om, 16, leaf=16, rank=2, rank_tol=1e-6, precision="c128", admissibility="strong")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.factor()
        torch.cuda.synchronize()
        fm = 1e3 * (time.perf_counter() - t0)
        s.solve(f, tol=1e-3)
        ms3, _, its3, _, _ = _timed_solve(s, f, 1e-3, 2, torch)
        ms6, _, its6, res6, _ = _timed_solve(s, f, 1e-6, 2, torch)
        ps, pit, pso = PAPER_LENS_STRONG[n]
        rows[str(n)] = {"omega": f"2pi*{q}", "factor_ms": fm, "solve_ms_at_1e-3": ms3, "gmres_iters_at_1e-3": its3[0],
                        "solve_ms_at_1e-6": ms6, "gmres_iters_at_1e-6": its6[0], "relres": res6[0],
                        "factor_bytes": s.plan_info()["factor_bytes"],
                        "paper_2010_cpu": {"T_setup_s": ps, "gmres_iters": pit, "T_solve_s": pso}}
        print(f"[bench] strong rank 2 lens, n = {n}: factor {fm:.0f} ms, solve {ms3:.1f} ms ({its3[0]} its at 1e-3), "
              f"{ms6:.1f} ms ({its6[0]} its at 1e-6)", file=sys.stderr, flush=True)
        del s
    rows["note"] = ("the paper's lens sizes with its rank-2 strong format; its T_setup/T_solve (2010 CPU, its own "
                    "lens) are context, not a target")
    return rows


def cpu_baseline(wl, budget_s=10.0):
    """The oracle's direct solve (assembly + SuperLU factor + solve), timed on
    the host, and the same split into factorization and per-solve times."""
    from oracle import assemble, direct
    c = wl.velocity()
    f = wl.sources()[0]
    t0 = time.perf_counter()
    count = 0
    u = None
    while True:
        st = assemble.stencil(c, wl.omega, wl.pml)
        u = direct.solve_sparse(st, f)
        count += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    # factorization and solve separately (median of 3)
    st = assemble.stencil(c, wl.omega, wl.pml)
    fac, sol = [], []
    for _ in range(3):
        a = time.perf_counter()
        lu = direct.SparseLU(st)
        b = time.perf_counter()
        lu.solve(f)
        d = time.perf_counter()
        fac.append(b - a)
        sol.append(d - b)
    blas = None
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = max((x.get("num_threads", 0) for x in info if x.get("user_api") == "blas"), default=None)
    except Exception:
        pass
    return {"value": count / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{count} complete oracle solves (assembly + SuperLU factor + solve) of the "
                      f"n={wl.n} workload in {dt:.1f} s on one host core",
            "host_cpu_count": os.cpu_count(), "blas_threads": blas,
            "note": "SuperLU is single-threaded: the factor and solve use one core whatever the BLAS thread count",
            "factor_s": float(np.median(fac)), "solve_s": float(np.median(sol)),
            "solve_phase_solves_per_s": 1.0 / float(np.median(sol))}, u


def kernel_probe(name):
    """Factor one workload (complex64) and apply its sweep three times to all
    its sources, with one and then four right-hand sides per workgroup."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver
    wl = W.get(name)
    F = torch.as_tensor(wl.sources(), device="cuda:0")
    for grp in (1, 4):
        s = Solver(wl.velocity(), wl.omega, wl.pml, leaf=wl.leaf, rank=wl.rank, rank_tol=wl.rank_tol,
                   precision="c64", rhs_group=grp).factor()
        for _ in range(3):
            s.apply(F)
        torch.cuda.synchronize()
        print(f"[probe] {name}: factor and 3 applies of {F.shape[0]} fields, rhs_group {grp}", file=sys.stderr,
              flush=True)
        del s


def iteration_tables():
    """GMRES iterations at a fixed 8 points per wavelength as omega grows (the
    shape of the paper's 2D PML tables, Sec. 3): lens, waveguide and random
    media at n = 127, 255, 511, 1023 (omega = 2 pi (n+1)/8, layers of 16
    points), a point source at (0.5, 0.125) and a wave packet at
    (0.125, 0.125) towards (1, 1), complex64 factors (leaf 16 up to n = 255,
    32 above, rank 8, tolerance 1e-6), GMRES to 1e-3 (the paper's tolerance)
    and to 1e-6.  Prints one JSON line; not part of the default run."""
    import torch
    import workloads as W
    from paper_1007_4290_amd.solver import Solver
    media = {"lens": W.lens_medium, "waveguide": W.waveguide_medium,
             "random": lambda n: W.random_field_medium(n, seed=1, amplitude=0.3)}
    out = {}
    for name, med in media.items():
        for n in (127, 255, 511, 1023):
            om = 2 * np.pi * (n + 1) / 8
            c = med(n)
            F = np.stack([W.gaussian_source(n, (0.5, 0.125)).ravel(),
                          W.wave_packet(n, (0.125, 0.125), (1.0, 1.0), om).ravel()])
            s = Solver(c, om, 16, leaf=16 if n <= 255 else 32, rank=8, rank_tol=1e-6, precision="c64").factor()
            f = torch.as_tensor(F, device="cuda:0")
            _, it3, _ = s.solve(f, tol=1e-3, maxit=300)
            _, it6, r6 = s.solve(f, tol=1e-6, maxit=300)
            out[f"{name}_{n}"] = {"omega_over_2pi": (n + 1) / 8, "iters_tol1e-3": list(it3), "iters_tol1e-6": list(it6),
                                  "relres_tol1e-6": [float(x) for x in r6]}
            print(f"[tables] {name} n={n}: iterations {list(it3)} at 1e-3, {list(it6)} at 1e-6",
                  file=sys.stderr, flush=True)
            del s
    print(json.dumps({"iteration_tables": out}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-workloads", action="store_true", help="skip the other problem sizes")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (the "
                         "calibration kernel for the HBM byte counters); not part of the timing")
    ap.add_argument("--kernel-probe", choices=["helm255_grf", "helm511_grf_64src"], default=None,
                    help="only factor the workload and apply its sweep 3 times with one and with four "
                         "right-hand sides per workgroup (a short run for the hardware counters); no JSON line")
    ap.add_argument("--strong-probe", action="store_true",
                    help="only the strongly admissible rank-2 factorization and solve at n = 63 (a short run "
                         "for the kernel trace); no JSON line")
    ap.add_argument("--strong-lens-probe", action="store_true",
                    help="only one strongly admissible rank-2 factorization of the n = 255 lens (the first row of "
                         "the strong_rank2_lens workload; a run for the kernel trace); no JSON line")
    ap.add_argument("--iteration-tables", action="store_true",
                    help="only the GMRES iteration counts of three media at 8 points per wavelength, "
                         "n = 127..1023 (one JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import workloads as W

    if args.copy_probe_mib > 0:
        import torch
        n4 = (args.copy_probe_mib << 20) // 4
        src = torch.ones(n4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print(f"[bench] copy probe: {args.copy_probe_mib} MiB read, {args.copy_probe_mib} MiB written",
              file=sys.stderr, flush=True)

    if args.kernel_probe:
        kernel_probe(args.kernel_probe)
        return
    if args.iteration_tables:
        iteration_tables()
        return
    if args.strong_probe:
        print(json.dumps(strong_workload(1e-6, n=63)), file=sys.stderr, flush=True)
        return
    if args.strong_lens_probe:
        strong_lens_factor(255)
        return
    tol = 1e-6
    wl = W.get("helm255_grf", precision="c64")
    r64 = run_gpu(wl, "c64", args.steps, args.warmup, tol)
    print(f"[bench] c64: {r64['ms_per_step']:.2f} ms/step, iters {r64['iters'][0]}", file=sys.stderr, flush=True)
    r128 = run_gpu(wl, "c128", args.steps, args.warmup, tol)
    print(f"[bench] c128: {r128['ms_per_step']:.2f} ms/step, iters {r128['iters'][0]}", file=sys.stderr, flush=True)

    plan = r64["plan"]
    n = wl.n
    nbytes = sweep_bytes(plan, n, 8)
    achieved = nbytes / (r64["sweep_ms_avg"] * 1e-3) / 1e9
    lflops = layer_kernel_flops(plan, wl.leaf, wl.rank)
    l_ach = lflops / (r64["layer_kernel_ms_avg"] * 1e-3) / 1e12
    wflops = woodbury_flops(plan, wl.leaf, wl.rank) * n
    w_ach = wflops / (r64["wood_ms_per_factor"] * 1e-3) / 1e12
    its = r64["iters"][0]
    sb = stencil_bytes(n, 1) * its + stencil_bytes(n, 1, residual=True) * (1 + (its - 1) // 40)
    s_ach = sb / (r64["stencil_ms_per_solve"] * 1e-3) / 1e9
    kb = krylov_bytes(n, [its])
    k_ach = kb / (r64["krylov_ms_per_solve"] * 1e-3) / 1e9
    line = {
        "metric": METRIC,
        "value": 1e3 / r64["ms_per_step"],
        "unit": "solves/s",
        "value_kind": "end to end: factorization + GMRES solve per step (one right-hand side)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "helm255_grf", "n": n, "omega": "2pi*32", "pml": wl.pml,
                   "medium": "1+0.3*GRF(l=0.1,seed=1)", "source": "centre Gaussian", "leaf": wl.leaf,
                   "rank": wl.rank, "rank_tol": wl.rank_tol, "gmres_tol": tol, "n_p": plan["n_p"],
                   "levels": plan["levels"]},
        "solve_phase_solves_per_s": 1e3 / r64["solve_ms"],
        "c64": {"solves_per_s": 1e3 / r64["ms_per_step"], "factor_ms": r64["factor_ms"],
                "solve_ms": r64["solve_ms"], "solve_phase_solves_per_s": 1e3 / r64["solve_ms"],
                "gmres_iters": r64["iters"][0], "relres": r64["relres"]},
        "c128": {"solves_per_s": 1e3 / r128["ms_per_step"], "factor_ms": r128["factor_ms"],
                 "solve_ms": r128["solve_ms"], "solve_phase_solves_per_s": 1e3 / r128["solve_ms"],
                 "gmres_iters": r128["iters"][0], "relres": r128["relres"]},
        "roofline": {"kernel": f"layer_kernel<float, {wl.leaf}, {wl.rank}>", "bound": "alu",
                     "achieved": l_ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": l_ach / FP32_PEAK_TFLOPS, "traffic": LAYER_KERNEL_HBM_BYTES,
                     "flops_per_launch": lflops,
                     "avg_launch_ms": r64["layer_kernel_ms_avg"],
                     "factor_share": r64["layer_kernel_ms_avg"] * n / r64["factor_ms"],
                     "note": "latency bound: dependent steps on single wavefronts"},
        "kernels": {
            "woodbury": {"bound": "alu", "ms_per_factor": r64["wood_ms_per_factor"], "flops_per_factor": wflops,
                         "achieved": w_ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": w_ach / FP32_PEAK_TFLOPS},
            "sweep": {"kernel": "sweep_kernel<float>", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": SWEEP_HBM_BYTES["helm255_grf"],
                      "bytes_per_launch": nbytes, "avg_launch_ms": r64["sweep_ms_avg"]},
            "stencil": {"bound": "hbm", "ms_per_solve": r64["stencil_ms_per_solve"], "bytes_per_solve": sb,
                        "achieved": s_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": s_ach / HBM_PEAK_GBS},
            "krylov": {"bound": "hbm", "ms_per_solve": r64["krylov_ms_per_solve"], "bytes_per_solve": kb,
                       "achieved": k_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": k_ach / HBM_PEAK_GBS},
        },
    }
    if not args.no_workloads:
        line["workloads"] = bench_workloads(tol)
    if not args.no_cpu:
        cb, u_ref = cpu_baseline(wl)
        line["cpu_baseline"] = cb
        err64 = float(np.linalg.norm(r64["u"][0] - u_ref) / np.linalg.norm(u_ref))
        err128 = float(np.linalg.norm(r128["u"][0] - u_ref) / np.linalg.norm(u_ref))
        line["c64"]["err_vs_oracle"] = err64
        line["c128"]["err_vs_oracle"] = err128
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
