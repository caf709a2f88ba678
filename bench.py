"""Benchmark: time to 1e-8 relative residual for the 2D fractional Laplacian
elliptic problem on a 1024 x 1024 grid, alpha = 1 (Omega = (-1,1)^2, f a seeded
sum of 32 Gaussian bumps), on one MI355X.

One "step" is one complete solve of that system (operator already built, inputs
resident in HBM): every kernel of the hot path (FFT application, sine-transform
preconditioner, fused Krylov updates, FP64 refinement) runs inside it.

Solver configurations timed (each must reach ||f - M u||/||f|| <= 1e-8, the
residual recomputed in FP64 on the GPU at the end of every solve):
  fp64_pcg       FP64 PCG, finite-difference Laplacian preconditioner (the paper's method)
  fp64_cg        FP64 CG without preconditioner
  f32_pcg        FP32 inner PCG + FP64 iterative refinement
  f32_cg         FP32 inner CG  + FP64 iterative refinement
  fp64_spectral  FP64 PCG, sine-basis diagonal of M as preconditioner
  f32_spectral   FP32 inner PCG (sine-basis diagonal) + FP64 refinement
  learned_f32    FP32 inner flexible CG with the learned preconditioner + FP64 refinement
  learned_fp64   FP64 flexible CG with the learned preconditioner
The learned preconditioner is trained first (outside the timed region) on
solver-generated pairs at 256^2, alpha ~ U[0.2, 1.9]: 100 problems x (10
iterate errors + 10 random-field errors) = 2000 pairs, then 4000 Adam steps of
batch 16 (the length that needed the fewest iterations on held-out 1024^2
right-hand sides at alpha = 0.5, 1.0, 1.5, among 1500 to 6000).  `value` is the time of
learned_f32; the plain-FP64 baseline is the faster of fp64_pcg and fp64_cg.

Reported beside it (not part of `value`): per-pass timings of the 1024^2
application and preconditioner and of every pass at 256^3 (`passes_3d`);
`roofline`, the kernel with the largest time per solve among those the timed
solver launches once per inner iteration (FP32 FFT and sine passes, network
layers), with its HBM traffic from a committed rocprofv3 counter summary when
one exists, and `roofline_next`, the runner-up; `learned_vs_spectral`, the
timed solver against the same refinement loop with the sine-basis diagonal
alone; the batched workloads (16 x 256^3 right-hand sides, 32 uneven 2D
backward-Euler problems x 200 steps, each with the FD preconditioner and the
sine-basis diagonal); the learned preconditioner in 3D (trained at 32^3,
evaluated at 128^3, alpha = 1.5, and at 256^3, alpha = 1.2, against FP64 PCG);
the oracle's FP64 PCG timed on the host for a bounded number of its
iterations, and the paper's method with scipy.fft solved in full.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--alpha A] [--no-cpu]
                       [--no-batched] [--no-learned-3d] [--passes-3d N] [--only a,b]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="comma list of configurations to time")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 3D and uneven-batch workloads")
    ap.add_argument("--uneven-steps", type=int, default=200)
    ap.add_argument("--train-problems", type=int, default=100)
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--train-batch", type=int, default=16)
    ap.add_argument("--no-learned-3d", action="store_true", help="skip the 3D learned-preconditioner workload")
    ap.add_argument("--train3d-problems", type=int, default=40)
    ap.add_argument("--train3d-n", type=int, default=32)
    ap.add_argument("--train3d-steps", type=int, default=600)
    ap.add_argument("--passes-3d", type=int, default=256,
                    help="also time every pass of the 3D application and preconditioner at this n^3 (0: skip)")
    ap.add_argument("--pass-reps", type=int, default=50)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "independent right-hand sides shard across GPUs without communication, "
              "so per-GPU throughput is the figure that transfers.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1802_03770_amd as fl
    from workloads import bump_field

    n, alpha, tol = args.n, args.alpha, args.tol
    log(f"[bench] workload 2D n={n} alpha={alpha} tol={tol}")
    f_np, h = bump_field(n, 2, 32, 2000, width=(0.05, 0.2))
    f = torch.from_numpy(f_np).cuda()
    t0 = time.perf_counter()
    op = fl.Op(2, alpha, h, (n, n))
    torch.cuda.synchronize()
    t_make = (time.perf_counter() - t0) * 1e3
    log(f"[bench] make_weights {t_make:.1f} ms (sine-transform plans, autotuned: {op.plan()})")

    # learned preconditioner: training set and training (not timed as a solve)
    net, train_info = None, None
    want_learned = not args.only or any(k.startswith("learned") for k in args.only.split(","))
    if want_learned:
        from paper_1802_03770_amd import learned as L
        from workloads import learned_training_plan
        t0 = time.perf_counter()
        plan = learned_training_plan(nalpha=args.train_problems, n=256, seed=5000)
        R, T, A = L.make_pairs(plan, iters=10, fields=10, stream=op.stream, log=log)
        t_pairs = time.perf_counter() - t0
        t0 = time.perf_counter()
        net, losses = L.train(R, T, A, steps=args.train_steps, batch=args.train_batch, lr=1e-3, seed=1,
                              stream=op.stream)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        l0 = float(np.mean(losses[:50]))
        l1 = float(np.mean(losses[-50:]))
        ms_step = t_train * 1e3 / max(1, len(losses))
        log(f"[bench] learned: {R.shape[0]} pairs at 256^2 in {t_pairs:.1f} s, {len(losses)} Adam steps "
            f"(batch {args.train_batch}) in {t_train:.1f} s ({ms_step:.2f} ms/step), loss {l0:.3e} -> {l1:.3e}")
        train_info = {"pairs": int(R.shape[0]), "grid": 256, "pairs_s": round(t_pairs, 2), "steps": len(losses),
                      "batch": args.train_batch, "train_s": round(t_train, 2), "ms_per_adam_step": round(ms_step, 3),
                      "loss_first": l0, "loss_last": l1}
        del R, T, A

    configs = {
        "fp64_pcg": fl.solve_opts(pc=fl.FL_PC_FD, mixed=0),
        "fp64_cg": fl.solve_opts(pc=fl.FL_PC_NONE, mixed=0),
        "f32_pcg": fl.solve_opts(pc=fl.FL_PC_FD, mixed=1),
        "f32_cg": fl.solve_opts(pc=fl.FL_PC_NONE, mixed=1),
        "fp64_spectral": fl.solve_opts(pc=fl.FL_PC_SPECTRAL, mixed=0),
        "f32_spectral": fl.solve_opts(pc=fl.FL_PC_SPECTRAL, mixed=1),
    }
    if net is not None:
        configs["learned_f32"] = fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=1, net=net)
        configs["learned_fp64"] = fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=0, net=net)
    if args.only:
        configs = {k: v for k, v in configs.items() if k in args.only.split(",")}
    results = {}
    for name, opts in configs.items():
        for _ in range(args.warmup):
            u, info = op.solve(f, tol=tol, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for _ in range(args.steps):
            u, info = op.solve(f, tol=tol, opts=opts)
            infos.append(info)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        worst = max(i["rel_res_true"] for i in infos)
        ok = worst <= tol and all(i["status"] == 0 for i in infos)
        results[name] = {"ms": ms, "iters": infos[-1]["iters"], "outer": infos[-1]["outer_iters"],
                         "rel_res_true": worst, "ok": ok, "fell_back": infos[-1]["fell_back"]}
        log(f"[bench] {name}: {ms:.2f} ms/solve iters={infos[-1]['iters']} outer={infos[-1]['outer_iters']} "
            f"true_res={worst:.2e} ok={ok}")
    good = {k: v for k, v in results.items() if v["ok"]}
    if not good:
        log("[bench] no configuration reached the tolerance")
        sys.exit(1)
    best = "learned_f32" if "learned_f32" in good else min(good, key=lambda k: good[k]["ms"])
    base = [k for k in ("fp64_pcg", "fp64_cg") if k in good]
    base_ms = min(good[k]["ms"] for k in base) if base else None

    # roofline of the dominant pass, timed live with HIP events on the op stream
    H = n // 1 + 1
    passes = {
        # name: (dtype, pass id, algorithmic bytes per launch)
        "f32_sine_col_scale": (torch.float32, 4, 2 * n * n * 4),
        "f32_fft_col_conv": (torch.float32, 1, 2 * n * (n + 1) * 8 + (n + 1) * (n + 1) * 4),
        "f32_fft_row_fwd": (torch.float32, 0, n * n * 4 + n * (n + 1) * 8),
        "f32_fft_row_inv": (torch.float32, 2, n * (n + 1) * 8 + n * n * 4),
        "f32_sine_row": (torch.float32, 3, 2 * n * n * 4),
        "f64_fft_col_conv": (torch.float64, 1, 2 * n * (n + 1) * 16 + (n + 1) * (n + 1) * 8),
        "f64_sine_col_scale": (torch.float64, 4, 2 * n * n * 8),
    }
    prof = {}
    for name, (dt, pid, nbytes) in passes.items():
        ms = op.profile_pass(dt, pid, reps=args.pass_reps)
        gbs = nbytes / (ms * 1e-3) / 1e9
        prof[name] = {"ms": ms, "bytes": nbytes, "GBps": gbs}
        log(f"[bench] pass {name}: {ms * 1e3:.1f} us  {gbs:.0f} GB/s (algorithmic)")
    passes3d = passes_3d(fl, torch, args.passes_3d, args.pass_reps) if args.passes_3d > 0 else None
    # Kernels that the timed solver (learned + FP32 refinement) launches once
    # per inner iteration: the FP32 application (row forward, symbol column
    # pass, row inverse), the FP32 sine passes (first / last row pass are two
    # kernels of equal shape; the scaled column pass) and, with a network, its
    # layers.  The FP64 passes run once per refinement step only.  The
    # roofline object reports the kernel with the largest time per solve.
    per_iter = {"f32_sine_col_scale": 1, "f32_fft_col_conv": 1, "f32_fft_row_fwd": 1, "f32_fft_row_inv": 1,
                "f32_sine_row": 1}
    if net is not None:
        # network layers at the solver grid (BF16 NHWC activations, 32 channels):
        # level-0 conv reads a0 (64 B/px) and the coarse c1 (16 B/px), writes c0 (64 B/px)
        for name, which, nbytes in (("net_conv_l0", 1, 144 * n * n), ("net_in_layer", 2, 68 * n * n),
                                    ("net_out_layer", 3, 68 * n * n), ("net_forward", 0, None)):
            ms = net.profile(which, n, n, reps=20)
            prof[name] = {"ms": ms, "bytes": nbytes, "GBps": (nbytes / (ms * 1e-3) / 1e9) if nbytes else None}
            gb = f"{prof[name]['GBps']:.0f} GB/s (algorithmic)" if nbytes else ""
            log(f"[bench] pass {name}: {ms * 1e3:.1f} us  {gb}")
        per_iter.update({"net_conv_l0": 1, "net_in_layer": 1, "net_out_layer": 1})
    iters_best = results.get(best, {}).get("iters") or 1
    per_solve = {k: prof[k]["ms"] * c * iters_best for k, c in per_iter.items()}
    ranked = sorted(per_solve, key=lambda k: -per_solve[k])
    dom = ranked[0]

    def hbm_roof(k):
        r = {"bound": "hbm", "achieved": round(prof[k]["GBps"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(prof[k]["GBps"] / HBM_PEAK_GBS, 4), "traffic": measured_traffic(f"{k}_{n}_hbm_counters.md"),
             "kernel": k, "avg_us": round(prof[k]["ms"] * 1e3, 2), "bytes_per_launch": prof[k]["bytes"],
             "ms_per_solve": round(per_solve[k], 4)}
        if k == "net_conv_l0":
            tf = 2 * 9 * 32 * 32 * n * n / (prof[k]["ms"] * 1e-3) / 1e12
            r["mfma_bf16_tflops"] = round(tf, 1)
            r["mfma_frac"] = round(tf / 2500.0, 4)
        return r
    roof = hbm_roof(dom)
    roof_next = hbm_roof(ranked[1]) if len(ranked) > 1 else None

    batched = None
    if not args.no_batched:
        batched = batched_workloads(fl, torch, args)
    learned3d = None
    if not args.no_learned_3d:
        learned3d = learned_3d_workload(fl, torch, args)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(n, alpha, h, f_np, results.get("fp64_pcg", {}).get("iters"))

    line = {
        "metric": "time to 1e-8 rel residual, 1024^2 alpha=1: learned+FP32 vs plain FP64 PCG",
        "value": round(good[best]["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(good[best]["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"learned_f32": "bf16+f32+f64", "learned_fp64": "bf16+f64"}.get(
            best, "f32+f64" if best.startswith("f32") else "f64"),
        "data": "synthetic (seeded Gaussian-bump right-hand side)",
        "config": {"workload": f"elliptic 2D n={n}x{n} alpha={alpha} (-1,1)^2 32 bumps seed 2000 tol {tol}",
                   "solver": best, "make_weights_ms": round(t_make, 1), "sine_plans": op.plan()},
        "learned_training": train_info,
        "baseline_fp64_ms": None if base_ms is None else round(base_ms, 3),
        "speedup_vs_fp64": None if base_ms is None else round(base_ms / good[best]["ms"], 3),
        # the network's own contribution: learned + FP32 against the same
        # refinement loop with the sine-basis diagonal alone (N = 0)
        "learned_vs_spectral": (round(good["learned_f32"]["ms"] / good["f32_spectral"]["ms"], 3)
                                if "learned_f32" in good and "f32_spectral" in good else None),
        "solvers": {k: {kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in results.items()},
        "passes_us": {k: round(v["ms"] * 1e3, 2) for k, v in prof.items()},
        "passes_GBps": {k: round(v["GBps"], 1) for k, v in prof.items() if v["GBps"]},
        "roofline": roof,
        "roofline_next": roof_next,
        "passes_3d": passes3d,
        "batched": batched,
        "learned_3d": learned3d,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def passes_3d(fl, torch, n, reps):
    """Time the passes of the FP32 and FP64 application and preconditioner on
    an n^3 grid (alpha = 1.2), HIP events on the op's stream.  Algorithmic
    bytes per launch (P = padded length, H = P/2 + 1, b = bytes per real):
      rows forward  n^3 b + n^2 H 2b          (real in, half spectrum out)
      axis-1 pair   2 (n^2 H + n P H) 2b      (forward and inverse, W1 <-> W2)
      axis-0 conv   2 n P H 2b + H^3 b        (W2 in place, folded symbol)
      rows inverse  n^2 H 2b + n^3 b
      sine passes   2 n^3 b each (first, middle pair, scaled column, last)."""
    op = fl.Op(3, 1.2, 2.0 / (n + 1), (n,) * 3)
    P = op.padded()[0]
    H = P // 2 + 1
    out = {}
    for dt, tag, b in ((torch.float32, "f32", 4), (torch.float64, "f64", 8)):
        rows = n ** 3 * b + n * n * H * 2 * b
        conv = 2 * n * P * H * 2 * b + H ** 3 * b
        pair = 2 * (n * n * H + n * P * H) * 2 * b
        sine = 2 * n ** 3 * b
        for name, pid, nbytes in ((f"{tag}_rows_fwd", 0, rows), (f"{tag}_col0_conv", 1, conv),
                                  (f"{tag}_rows_inv", 2, rows), (f"{tag}_apply", 6, 2 * rows + conv + pair),
                                  (f"{tag}_sine_first", 3, sine), (f"{tag}_sine_col0_scale", 4, sine),
                                  (f"{tag}_sine_last", 5, sine), (f"{tag}_precond", 7, 5 * sine)):
            ms = op.profile_pass(dt, pid, reps=max(3, reps // 5))
            out[name] = {"us": round(ms * 1e3, 2), "bytes": nbytes,
                         "GBps": round(nbytes / (ms * 1e-3) / 1e9, 1),
                         "frac": round(nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"[bench] 3d {n}^3 pass {name}: {ms * 1e3:.1f} us  {out[name]['GBps']:.0f} GB/s (algorithmic)")
    op.close()
    return {"n": n, "passes": out}


def measured_traffic(name):
    """HBM bytes per launch from a committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, copy-kernel calibrated), or None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.strip().startswith("- traffic_bytes_per_launch:"):
            return int(float(line.split(":")[1]))
    return None


def batched_workloads(fl, torch, args):
    """The batched row of the hot path on its two workloads (one launch per
    pass over all problems, captured iteration graphs):
      rhs16_256cubed: d=3, 256^3, alpha=1.2, 16 right-hand sides of one operator, FP32
          inner PCG + FP64 refinement to 1e-8 (FD preconditioner, and the
          sine-basis diagonal with its one-off table build timed apart);
      uneven_2d_steps: 32 uneven 2D backward-Euler problems (n in {128,256,384,512},
          alpha ~ U[0.3,1.8]), dt = 1e-3, `uneven_steps` steps, tol 1e-10."""
    from workloads import workload_rhs_256cubed, workload_uneven_steps
    out = {}
    s = torch.cuda.Stream()
    # uneven 2D steps
    probs = workload_uneven_steps(32)
    t0 = time.perf_counter()
    ops = [fl.Op(2, p["alpha"], p["h"], (p["n"], p["n"]), stream=s) for p in probs]
    torch.cuda.synchronize()
    t_make = time.perf_counter() - t0
    unk = sum(p["n"] ** 2 for p in probs)
    res = {}
    for name, pc in (("spectral", fl.FL_PC_SPECTRAL), ("fd", fl.FL_PC_FD)):
        opts = fl.solve_opts(pc=pc)
        us = [torch.from_numpy(p["u0"]).cuda() for p in probs]
        # the first call builds the batch (and the diagonal tables); the timed
        # call with the same problems and dt reuses it
        fl.step_batched(ops, [u.clone() for u in us], [1e-3] * 32, theta=1.0, nsteps=2, tol=1e-10, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = fl.step_batched(ops, us, [1e-3] * 32, theta=1.0, nsteps=args.uneven_steps, tol=1e-10,
                                   opts=opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        res[name] = {"ms_total": round(ms, 1), "ms_per_step": round(ms / args.uneven_steps, 3),
                     "unknown_steps_per_s": round(unk * args.uneven_steps / (ms * 1e-3), 1),
                     "iters_per_step_mean": round(sum(i["iters"] for i in infos) / (32 * args.uneven_steps), 2),
                     "max_rel_res_true": max(i["rel_res_true"] for i in infos)}
        log(f"[bench] uneven 2D {name}: {args.uneven_steps} steps of 32 uneven problems in {ms:.1f} ms "
            f"({ms / args.uneven_steps:.2f} ms/step), mean iters/step {res[name]['iters_per_step_mean']}, "
            f"max true res {res[name]['max_rel_res_true']:.1e}")
    out["uneven_2d_steps"] = {"workload": "32 uneven 2D backward-Euler problems, n in {128,256,384,512}, dt=1e-3",
                              "steps": args.uneven_steps, "make_weights_s": round(t_make, 2), **res}
    for o in ops:
        o.close()
    del ops, us
    # 16 right-hand sides at 256^3
    w0 = workload_rhs_256cubed(0)
    t0 = time.perf_counter()
    op = fl.Op(3, w0["alpha"], w0["h"], (w0["n"],) * 3, stream=s)
    torch.cuda.synchronize()
    t_make = time.perf_counter() - t0
    fs = [torch.from_numpy(workload_rhs_256cubed(k)["f"]).cuda() for k in range(16)]
    b3d = {"workload": "3D 256^3 alpha=1.2, 16 right-hand sides, FP32 inner + FP64 refinement, tol 1e-8",
          "make_weights_ms": round(t_make * 1e3, 1)}
    for name, pc in (("fd", fl.FL_PC_FD), ("spectral", fl.FL_PC_SPECTRAL)):
        opts = fl.solve_opts(pc=pc, mixed=1)
        if pc == fl.FL_PC_SPECTRAL:
            t0 = time.perf_counter()
            op.tau()
            b3d["tau_build_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, infos = fl.solve_batched([op] * 16, fs, tol=1e-8, opts=opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        b3d[name] = {"ms": round(ms, 1), "ms_per_rhs": round(ms / 16, 2),
                    "iters_mean": round(sum(i["iters"] for i in infos) / 16, 1),
                    "max_rel_res_true": max(i["rel_res_true"] for i in infos)}
        log(f"[bench] 256^3 x16 {name}: 16 x 256^3 in {ms:.1f} ms, mean iters {b3d[name]['iters_mean']}, "
            f"max true res {b3d[name]['max_rel_res_true']:.1e}")
    out["rhs16_256cubed"] = b3d
    op.close()
    return out


def learned_3d_workload(fl, torch, args):
    """The learned preconditioner in 3D (3 x 3 x 3 kernels): trained on
    solver-generated pairs at `train3d_n`^3 (alpha ~ U[0.2, 1.9]; 5 iterate
    errors + 5 random-field errors per problem), evaluated in flexible CG at
    128^3, alpha = 1.5, 16-bump right-hand side, tol 1e-8, against FD PCG and
    the spectral preconditioner alone (FP64 and FP32 + FP64 refinement).
    Each solve is timed over 2 runs after 1 warm-up."""
    import numpy as np

    from paper_1802_03770_amd import learned as L
    from workloads import bump_field, learned_training_plan
    s = torch.cuda.Stream()
    t0 = time.perf_counter()
    plan = learned_training_plan(nalpha=args.train3d_problems, n=args.train3d_n, seed=5600, d=3)
    R, T, A = L.make_pairs(plan, iters=5, fields=5, stream=s)
    t_pairs = time.perf_counter() - t0
    t0 = time.perf_counter()
    net, losses = L.train(R, T, A, steps=args.train3d_steps, batch=4, lr=2e-3, seed=2, stream=s)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    l0, l1 = float(np.mean(losses[:20])), float(np.mean(losses[-20:]))
    log(f"[bench] learned 3d: {R.shape[0]} pairs at {args.train3d_n}^3 in {t_pairs:.1f} s, {len(losses)} Adam steps "
        f"(batch 4) in {t_train:.1f} s ({t_train * 1e3 / max(1, len(losses)):.2f} ms/step), "
        f"loss {l0:.3e} -> {l1:.3e}")
    out = {"workload": "evaluated at 128^3 alpha=1.5 (16 bumps seed 5500) and 256^3 alpha=1.2 (the first of "
                       "the 16 right-hand sides at 256^3)",
           "training": {"pairs": int(R.shape[0]), "grid": args.train3d_n, "pairs_s": round(t_pairs, 2),
                        "steps": len(losses), "batch": 4, "train_s": round(t_train, 2),
                        "ms_per_adam_step": round(t_train * 1e3 / max(1, len(losses)), 3), "loss_first": l0,
                        "loss_last": l1}}
    del R, T, A
    from workloads import workload_rhs_256cubed
    w256 = workload_rhs_256cubed(0)
    evals = [("128cubed", 128, 1.5, bump_field(128, 3, 16, 5500, width=(0.05, 0.2)), 2),
             ("256cubed", 256, w256["alpha"], (w256["f"], w256["h"]), 1)]
    for key, n, alpha, (f_np, h), reps in evals:
        f = torch.from_numpy(f_np).cuda()
        op = fl.Op(3, alpha, h, (n,) * 3, stream=s)
        configs = {
            "fp64_pcg": fl.solve_opts(pc=fl.FL_PC_FD, mixed=0),
            "f32_pcg": fl.solve_opts(pc=fl.FL_PC_FD, mixed=1),
            "fp64_spectral": fl.solve_opts(pc=fl.FL_PC_SPECTRAL, mixed=0),
            "f32_spectral": fl.solve_opts(pc=fl.FL_PC_SPECTRAL, mixed=1),
            "learned_f32": fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=1, net=net),
            "learned_fp64": fl.solve_opts(pc=fl.FL_PC_LEARNED, mixed=0, net=net),
        }
        res = {}
        for name, opts in configs.items():
            op.solve(f, tol=1e-8, opts=opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = [op.solve(f, tol=1e-8, opts=opts)[1] for _ in range(reps)]
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            worst = max(i["rel_res_true"] for i in infos)
            res[name] = {"ms": round(ms, 3), "iters": infos[-1]["iters"], "outer": infos[-1]["outer_iters"],
                         "rel_res_true": float(f"{worst:.3g}"), "ok": bool(worst <= 1e-8),
                         "fell_back": infos[-1]["fell_back"]}
            log(f"[bench] learned 3d {key} {name}: {ms:.2f} ms/solve iters={infos[-1]['iters']} "
                f"outer={infos[-1]['outer_iters']} true_res={worst:.2e}")
        ev = {"workload": f"3D {n}^3 alpha={alpha} (-1,1)^3, tol 1e-8", "solvers": res,
              "net_forward_ms": round(net.profile(0, n, n, reps=3, D=n), 3)}
        if res["learned_f32"]["ok"] and res["fp64_pcg"]["ok"]:
            ev["learned_f32_vs_fp64_pcg_speedup"] = round(res["fp64_pcg"]["ms"] / res["learned_f32"]["ms"], 3)
        out[key] = ev
        op.close()
        del f
    return out


def cpu_baseline(n, alpha, h, f, iters):
    """The oracle's FP64 PCG (explicit-DFT application, dense sine-matrix
    preconditioner) timed on the host for a bounded number of its own
    iterations and scaled to the iteration count of the solve; and, beside it,
    the paper's method with a library FFT (scipy.fft) solved in full."""
    from oracle import cpu_fft as CF
    from oracle import krylov as KR
    from oracle import operator as O
    from oracle import precond as PC
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"[bench] cpu baseline: oracle at {n}^2 ({threads} threads)")
    t0 = time.perf_counter()
    ref = O.Operator(2, alpha, h, (n, n))
    lam = ref.lam_full
    t_sym = time.perf_counter() - t0
    sc = PC.pc_scale(2, alpha, h)
    k = 16
    t0 = time.perf_counter()
    KR.pcg(lambda v: O.apply_dft(lam, v), f, lambda r: PC.apply_inverse(r, sc), tol=1e-30, maxit=k)
    t_it = (time.perf_counter() - t0) / k
    it = iters or 100
    est_ms = (t_sym + it * t_it) * 1e3
    log(f"[bench] oracle: symbol {t_sym:.1f} s, {t_it:.2f} s per PCG iteration ({k} timed) -> {est_ms / 1e3:.0f} s "
        f"for {it} iterations")
    t0 = time.perf_counter()
    cs = CF.FFTSolver(2, alpha, h, (n, n), workers=threads)
    _, it_fft, res_fft, _ = cs.solve(f, tol=1e-8)
    t_fft = (time.perf_counter() - t0) * 1e3
    log(f"[bench] scipy.fft FP64 PCG: {t_fft / 1e3:.2f} s, {it_fft} iterations, recurrence residual {res_fft:.1e}")
    return {"value": round(est_ms, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"{k} iterations of the oracle's FP64 PCG (explicit-DFT apply, dense sine-matrix "
                      f"preconditioner) at {n}^2 timed, plus its symbol, scaled to {it} iterations (the FP64 "
                      f"PCG count on the GPU, equal to the oracle's within one)",
            "paper_method_scipy_fft": {"ms": round(t_fft, 1), "iters": it_fft, "workers": threads,
                                       "what": "FP64 PCG, FD preconditioner, scipy.fft transforms, full solve "
                                               "to 1e-8"}}


if __name__ == "__main__":
    main()
