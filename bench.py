"""Benchmark: 2D Helmholtz solves/s at relative residual 1e-6, complex64 sweep
(FP64 residual and Arnoldi) beside the complex128 sweep, on one MI355X.

Workload (n=255): omega = 2 pi 32 (8 points per wavelength), velocity
c = 1 + 0.3 * smooth Gaussian random field (correlation 0.1, seed 1), PML 16
points, centre Gaussian source, H-matrix Schur complements with leaf 16 and
rank <= 8 at relative tolerance 1e-6.

One step is the whole hot path for one right-hand side with the inputs
already in device memory: stencil coefficients, the layer-by-layer
factorization with H-matrix Schur complements, and flexible GMRES with the
sweep as preconditioner until ||f - A u|| <= 1e-6 ||f||.

Prints one JSON line.  `roofline` covers the dominant kernel, the layer
kernel of the factorization (one launch per layer: the recompressions of the
off-diagonal blocks and the dense leaves), whose average launch time is
measured with HIP events around each launch on the stream it runs on.  It is
latency bound (chains of small dependent steps on single wavefronts), so it is
reported against the vector FP32 peak ("alu") with its algorithmic flops.
`roofline_sweep` covers the preconditioner sweep against HBM.  `cpu_baseline`
times the CPU oracle (sparse LU, the plain definition u = A^{-1} f).
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
FP32_PEAK_TFLOPS = 157.3      # MI355X vector FP32 (256 CUs at 2.4 GHz)
FP64_PEAK_TFLOPS = 78.6
METRIC = "2D Helmholtz solves/s at rel. residual 1e-6: complex64 vs FP64 sweep"
# HBM bytes per launch of layer_kernel<float, 16, 8> on this workload: FETCH_SIZE
# + WRITE_SIZE from two rocprofv3 counter passes, each scaled by what the counter
# reads for a 1 GiB device-to-device copy (profiles/layer_kernel_pmc_helm255.md).
# Counters cannot be read inside a timed run; a change to the kernel voids this.
LAYER_KERNEL_HBM_BYTES = 981244
# The same two passes for one complex64 sweep launch (one right-hand side).
SWEEP_KERNEL_HBM_BYTES = 66189250


def sweep_bytes(plan, n, elem, nrhs=1):
    """Algorithmic bytes of one sweep launch: every layer's factor data is
    read once per layer step (2n-1 steps), plus the couplings, the input and
    output fields (complex128) and the forward work vector (written, then read)."""
    np_, b, L, r = plan["n_p"], plan["b"], plan["levels"], plan["r"]
    e_layer = np_ * b + L * r * np_ + ((1 << L) - 1) * 4 * r * r
    fac = (2 * n - 1) * e_layer * elem
    coup = 2 * (n - 1) * np_ * elem
    vec = nrhs * (2 * n * n * 16 + 2 * n * np_ * elem)
    return fac + coup * nrhs + vec


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
    sweep_ms, applies, factor_ms, iters, res = 0.0, 0, 0.0, [], []
    for _ in range(steps):
        s.factor()
        factor_ms += s.timings()["factor_ms"]
        u, it, rr = s.solve(f, tol=tol)
        tm = s.timings()
        sweep_ms += tm["sweep_ms"]
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
        "layer_kernel_ms_avg": layer_ms,
        "wood_ms_per_factor": wood_ms,
        "iters": iters,
        "relres": max(res),
        "plan": info,
        "u": u.cpu().numpy(),
    }


def cpu_baseline(wl, budget_s=10.0):
    """The oracle's direct solve (SuperLU factor + solve), timed on the host."""
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
    return {"value": count / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{count} complete oracle solves (assembly + SuperLU factor + solve) of the "
                      f"n={wl.n} workload in {dt:.1f} s on one host core"}, u


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (the "
                         "calibration kernel for the HBM byte counters); not part of the timing")
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

    tol = 1e-6
    wl = W.get("helm255_grf", precision="c64")
    r64 = run_gpu(wl, "c64", args.steps, args.warmup, tol)
    print(f"[bench] c64: {r64['ms_per_step']:.2f} ms/step, iters {r64['iters'][0]}", file=sys.stderr, flush=True)
    r128 = run_gpu(wl, "c128", args.steps, args.warmup, tol)
    print(f"[bench] c128: {r128['ms_per_step']:.2f} ms/step, iters {r128['iters'][0]}", file=sys.stderr, flush=True)

    plan = r64["plan"]
    nbytes = sweep_bytes(plan, wl.n, 8)
    achieved = nbytes / (r64["sweep_ms_avg"] * 1e-3) / 1e9
    lflops = layer_kernel_flops(plan, wl.leaf, wl.rank)
    l_ach = lflops / (r64["layer_kernel_ms_avg"] * 1e-3) / 1e12
    line = {
        "metric": METRIC,
        "value": 1e3 / r64["ms_per_step"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "helm255_grf", "n": wl.n, "omega": "2pi*32", "pml": wl.pml,
                   "medium": "1+0.3*GRF(l=0.1,seed=1)", "source": "centre Gaussian", "leaf": wl.leaf,
                   "rank": wl.rank, "rank_tol": wl.rank_tol, "gmres_tol": tol, "n_p": plan["n_p"],
                   "levels": plan["levels"]},
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
                     "factor_share": r64["layer_kernel_ms_avg"] * wl.n / r64["factor_ms"],
                     "note": "latency bound: dependent steps on single wavefronts; Woodbury kernels "
                             f"{r64['wood_ms_per_factor']:.1f} ms per factorization"},
        "roofline_sweep": {"kernel": "sweep_kernel<float>", "bound": "hbm", "achieved": achieved,
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": SWEEP_KERNEL_HBM_BYTES, "bytes_per_launch": nbytes,
                           "avg_launch_ms": r64["sweep_ms_avg"]},
    }
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
