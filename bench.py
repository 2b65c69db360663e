#!/usr/bin/env python3
"""MAID hot-path benchmark on one MI355X.

A step is one outer iteration of Algorithm 2 (MAID) on a synthetic
semi-blind deblurring instance: the InexactGradient of Algorithm 1 (lower-
level FISTA solve, upper-level gradient, CG adjoint solve, FP64-MFMA
hypergradient) and the psi trials of Eq. (3.4), each trial a further lower-
level solve.  The metric is pixel-iterations per second: (lower-level
iterations + CG iterations) x pixels (C*H*W) per second of wall time, inputs
resident in HBM.  The default workload is the 256x256 grayscale FP32 case
(9x9 kernel).

Prints ONE JSON line.  Extra objects: `roofline` for the kernel with the
largest total GPU time in the timed region (durations from HIP events on
the library's stream, algorithmic bytes or flops per launch from the kernel
model below), and `cpu_baseline`, the FP64 oracle timed on the host cores on
a bounded sample of the same workload (fixed lower-level and CG iterations).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM = 8.0e12          # B/s, MI355X HBM3E
PEAK_FP32 = 157.3e12       # flop/s, FP32 vector (published; packed FP32 instructions)
PEAK_FP64 = 78.6e12        # flop/s, FP64 vector and FP64 matrix

# MAID settings per workload (initial accuracy eps0 = delta0, initial step s0);
# the factors are the paper's (Section 4.1).
MAID_SETTINGS = {
    "cfg1": dict(eps0=1e-5, step0=1e-4),
    "cfg2": dict(eps0=1e-4, step0=1e-4),
    "cfg3": dict(eps0=1e-3, step0=1e-5),
    "cfg5": dict(eps0=1e-3, step0=1e-6),
    "paper": dict(eps0=1e-2, step0=1e-2),
}


def kernel_model(kind: str, K: int, esz: int, C: int):
    """Algorithmic (bytes, flops) per image element for one launch of a
    kernel kind: each input read once and each output written once (halo
    re-reads excluded), flops of the convolutions (2K^2 per tap pass) and
    the stencils / vector updates."""
    k2 = 2 * K * K
    if kind == "apg_grad":      # x, x_prev, Kx, Kx_prev, y -> G
        return 6 * esz, k2 + 45
    if kind == "apg_trial":     # x, x_prev, G, Kx, Kx_prev, y -> x+, Kx+
        return 8 * esz, k2 + 50
    if kind == "cg_dir":        # r, p_old -> p, Kp
        return 4 * esz, k2 + 2
    if kind == "cg_hvp":        # Kp, p, x -> Hp
        return 4 * esz, k2 + 60
    if kind == "cg_update":     # q, p, r, Hp -> q, r
        return 6 * esz, 6
    if kind == "conv":          # in (+ sub) -> out
        return 3 * esz, k2 + 1
    if kind == "hg_corr":       # rho, q, theta*q, x -> KxK partial sums (two 16/32-padded contractions)
        kt = 16 if K <= 16 else 32
        return 4 * esz, 2 * 2 * kt * kt
    return 0, 0


def roofline_for(prof: dict, N: int, K: int, esz: int, C: int):
    """Roofline of the kernel kind with the largest total GPU time.  Solver
    passes launched in chunks exit early once a solve has finished; only the
    launches that did a pass of work carry algorithmic bytes, so the bytes per
    launch are the work launches' bytes averaged over all launches, divided
    by the average duration of all launches (= work bytes / total time)."""
    name, (launches, work, ms) = max(prof.items(), key=lambda kv: kv[1][2])
    if launches == 0:
        return None, name
    avg_s = ms / launches / 1e3
    b, f = kernel_model(name, K, esz, C)
    bytes_launch, flops_launch = b * N * work / launches, f * N * work / launches
    peak_alu = PEAK_FP64 if (esz == 8 or name == "hg_corr") else PEAK_FP32
    t_hbm, t_alu = bytes_launch / PEAK_HBM, flops_launch / peak_alu
    if t_hbm >= t_alu:
        ach = bytes_launch / avg_s / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 2), peak=PEAK_HBM / 1e9, unit="GB/s",
                    frac=round(ach / (PEAK_HBM / 1e9), 4), traffic=None)
    else:
        ach = flops_launch / avg_s / 1e12
        roof = dict(bound="mfma" if name == "hg_corr" else "alu", achieved=round(ach, 3),
                    peak=peak_alu / 1e12, unit="TFLOP/s", frac=round(ach / (peak_alu / 1e12), 4), traffic=None)
    roof.update(kernel=name, launches=launches, work_launches=work, avg_us=round(avg_s * 1e6, 3),
                algorithmic_bytes_per_work_launch=b * N, algorithmic_flops_per_work_launch=f * N)
    return roof, name


def cpu_baseline(inst, budget_s: float = 15.0):
    """The FP64 oracle on the host cores: fixed lower-level (FISTA) and CG
    iterations on the same instance, scaled to pixel-iterations/s."""
    import numpy as np
    import oracle as O

    p = O.Problem.of(inst)
    y = inst.y.astype(np.float32).astype(np.float64)
    N = p.N

    def run(n):
        t0 = time.perf_counter()
        x, _, _ = O.lower_solve(p, inst.a, y, y, tol=0.0, max_iter=n, L=0.0, replay_bt=[0] * n)
        g, _, _ = O.upper_value_grad(p, inst.a, y, x)
        O.adjoint_solve(p, inst.a, x, g, tol=0.0, max_iter=n)
        return time.perf_counter() - t0

    t1 = run(1)
    n = max(2, min(400, int(budget_s / max(t1, 1e-4) / 2)))
    t = run(n)
    return dict(value=2 * n * N / t, unit="pixel-iterations/s", cores=O.num_threads(), kind="oracle",
                sample=f"{n} FISTA + {n} CG iterations (fixed, no backtracking) on the full {inst.C}x{inst.H}x{inst.W} "
                       f"instance, FP64, {t:.1f} s")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build runs on a single MI355X (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2502_09758_amd import synth
    from paper_2502_09758_amd import _lib as L
    from paper_2502_09758_amd.maid import Maid, MaidState

    torch.cuda.set_device(0)
    inst = synth.make(args.workload)
    dt = torch.float64 if inst.meta["dtype"] == "f64" else torch.float32
    esz = 8 if dt == torch.float64 else 4
    C, H, W, K = inst.C, inst.H, inst.W, inst.K
    N = C * H * W
    ms = MAID_SETTINGS[args.workload]
    m = Maid(C, H, W, K, dt, alpha=inst.alpha, eps_tv=inst.eps_tv, beta=inst.beta)
    a = torch.tensor(inst.a, dtype=torch.float64, device="cuda")
    y = torch.tensor(inst.y, dtype=dt, device="cuda")

    def fresh():
        return MaidState(a.clone(), y.clone(), torch.zeros_like(y), eps=ms["eps0"], delta=ms["eps0"],
                         step=ms["step0"])

    hp = dict(eps_min=1e-6)
    state = fresh()
    restarts = 0

    def step():
        nonlocal state, restarts
        rc, info = m.maid_step(a, y, state, **hp)
        if rc == L.ACCURACY_FLOOR:      # MAID's stop (accuracy below 1e-6): start a new run from theta_0
            state = fresh()
            restarts += 1
        return rc, info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if not args.no_profile:
        m.profile(True)
    lower = cg = accepted = trials = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, info = step()
        lower += info["lower_iters"]
        cg += info["cg_iters"]
        accepted += info["accepted"]
        trials += info["trials"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = m.profile_read() if not args.no_profile else {}
    m.profile(False)
    elapsed = t1 - t0
    value = (lower + cg) * N / elapsed

    roof, dom = roofline_for(prof, N, K, esz, C) if prof else (None, None)

    # time to hypergradient: one cold InexactGradient at eps = delta = tol
    tth = {}
    for tol in (1e-2, 1e-4):
        x = y.clone()
        q = torch.zeros_like(y)
        grad = torch.empty_like(y)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        li = m.lower_solve(a, y, x, tol, max_iter=300)
        m.upper_value_grad(a, y, x, grad)
        ci = m.adjoint_solve(a, x, grad, q, tol, max_iter=1000)
        m.hypergrad(a, a, y, x, q)
        torch.cuda.synchronize()
        tth[str(tol)] = dict(ms=round((time.perf_counter() - s0) * 1e3, 3), lower_iters=li.iters, cg_iters=ci.iters,
                             lower_status=L.CODE_NAMES[li.status], cg_status=L.CODE_NAMES[ci.status])

    out = {
        "metric": "pixel-iterations/s (lower+CG)",
        "value": round(value, 1),
        "unit": "pixel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if esz == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {H}x{W}x{C} piecewise-constant image, {K}x{K} kernel, "
                               f"alpha={inst.alpha:g}, smoothed TV eps={inst.eps_tv:g}, "
                               f"{'FP64' if esz == 8 else 'FP32 storage / FP64 reductions'}, plain MAID",
                   "eps0": ms["eps0"], "step0": ms["step0"], "tiles": m.config()},
        "roofline": roof,
        "lower_iters": lower, "cg_iters": cg, "accepted_steps": accepted, "psi_trials": trials,
        "maid_restarts": restarts,
        "time_to_hypergrad": tth,
        "kernel_ms": {k: dict(launches=v[0], work=v[1], ms=round(v[2], 3)) for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
