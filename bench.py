"""Benchmark: interior-point solve of the 256 x 256 right-triangle grid with
K = 64 on one MI355X (5-Gaussian-mixture marginals plus a 1e-3 background,
synthetic), mixed precision (FP32 BB preconditioner, FP64 Newton / FGMRES)
against the FP64 path.  One step = one continuation run, mu = 0.2^l from 1
down to mu_stop (8e-3 by default on this grid: below it the interior-point
iteration itself slows to step lengths of 1e-3..1e-1 on this workload),
every mu solved to |F| <= 1e-6 with BB-preconditioned FGMRES Newton steps.

Prints one JSON line: value = Krylov (FGMRES) iterations per second of the
mixed path over the timed steps, the time-to-tolerance of both paths, the
roofline of one hot-path kernel timed with HIP events on its own stream
during the timed steps, and the oracle's time-to-tolerance on a bounded
sample of the same workload on the host cores.
"""

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# the CPU sample: the metric workload's marginal recipe on a reduced grid
SAMPLE_N, SAMPLE_K = 24, 12
COPY_BYTES = 1 << 30          # reference copy of the counter loop: 1 GiB read, 1 GiB written
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# `bench.py --counter-loop 20` (KiB per dispatch), scaled by what the same
# counters read for the 1 GiB reference copy (fetch x2.0000, write x1.0000);
# profiles/k_schur_out_256x256_K64_traffic.md.  Valid only for the kernel
# version those runs measured, on the 256 x 256, K = 64 workload.
TRAFFIC_BYTES = {("schur_out", 3): 73838.51 * 1024 * 1.99995 + 8192.0 * 1024 * 1.00000}
KERNEL_NAMES = {"schur_out": "k_schur_out", "schur_btilde": "k_schur_btilde_tb", "cheb_fine": "k_cheb_step<., 1>",
                "tri_fine": "k_tri_scan<., 1>", "multidot": "k_multidot", "saddle_phi": "k_saddle_phi"}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=0,
                   help="untimed full solves before the timed ones (a small solve always runs first)")
    p.add_argument("--config", type=int, default=3, help="workload: 1, 2 or 3 (256^2, K=64)")
    p.add_argument("--kernel", default="schur_out", help="kernel whose roofline is reported")
    p.add_argument("--mu-stop", type=float, default=None,
                   help="end the continuation after this mu (default: 8e-3 for config 3, full run otherwise)")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solve")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--gpu-sample", action="store_true",
                   help="also solve the CPU sample on the GPU (adds small launches to a profile)")
    p.add_argument("--verbose", type=int, default=0)
    p.add_argument("--cpu-sample-only", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--counter-loop", type=int, default=0,
                   help="only run N pseudo-Schur applications of the workload's mixed state and N plain "
                        "copies of a known size (for hardware-counter runs), then exit")
    return p.parse_args()


def cpu_sample():
    """The oracle's full solve of the reduced sample (run in a child process
    pinned to one BLAS thread); prints its JSON and exits."""
    import numpy as np  # noqa: F401

    import otinputs
    from oracle.ipm import Problem, solve_ipm
    from oracle.mesh import structured_mesh

    ri, rf = otinputs.mixture_pair(SAMPLE_N, 5, 3, background=1e-3)
    prob = Problem(structured_mesh(SAMPLE_N), SAMPLE_K, ri, rf)
    t0 = time.perf_counter()
    r = solve_ipm(prob, tol=1e-6)
    dt = time.perf_counter() - t0
    print(json.dumps({"seconds": dt, "cost": r.cost, "newton": int(sum(r.newton_per_mu)),
                      "converged": bool(r.converged)}))


def run_cpu_baseline():
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample-only"], env=env,
                         capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        raise RuntimeError("oracle sample failed: " + out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def counter_loop(a, ot, otinputs, torch, dev):
    """Hardware-counter workload: the mixed state of the benchmark problem after
    one Newton step, N applications of its pseudo-Schur operator (one launch of
    each pass per application), then N device copies of COPY_BYTES."""
    import ctypes as C

    import numpy as np

    n, K, ri, rf = otinputs.config_marginals(a.config)
    mesh = ot.Mesh.structured(n)
    st = ot.State(mesh, ri, rf, K, precision="mixed")
    st.newton_step(raise_on_error=False)
    z = np.random.default_rng(0).standard_normal(st.m_rho)
    out = np.zeros(st.m_rho)
    dp = C.POINTER(C.c_double)
    for _ in range(a.counter_loop):
        ot.check(ot.lib().otbb_debug_schur_apply(st._h, z.ctypes.data_as(dp), out.ctypes.data_as(dp)))
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(a.counter_loop):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"counter_loop": a.counter_loop, "copy_bytes": COPY_BYTES, "m_rho": st.m_rho}), flush=True)


def main():
    a = parse()
    if a.cpu_sample_only:
        cpu_sample()
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import otinputs
    import paper_2209_00315_amd as ot

    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    if a.counter_loop > 0:
        counter_loop(a, ot, otinputs, torch, dev)
        return

    mu_stop = a.mu_stop if a.mu_stop is not None else (8e-3 if a.config == 3 else 0.0)

    def solve(n, K, ri, rf, precision, mu_stop=0.0):
        mesh = ot.Mesh.structured(n)
        ri_d = torch.as_tensor(ri, dtype=torch.float64, device=dev)
        rf_d = torch.as_tensor(rf, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ot.solve(mesh, ri_d, rf_d, K, tol=1e-6, device=True, precision=precision, verbose=a.verbose,
                       mu_stop=mu_stop, raise_on_error=False)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    def log(msg):
        print("# " + msg, file=sys.stderr, flush=True)

    n, K, ri, rf = otinputs.config_marginals(a.config)
    # code-object load and first allocations outside the timed region: one
    # Newton step of the same problem in each precision, so that every launch
    # in this process has the workload's shape
    mesh_w = ot.Mesh.structured(n)
    for prec in ("mixed", "fp64"):
        stw = ot.State(mesh_w, torch.as_tensor(ri, device=dev), torch.as_tensor(rf, device=dev), K, device=True,
                       precision=prec)
        stw.newton_step(raise_on_error=False)
        del stw
    torch.cuda.synchronize()

    for w in range(a.warmup):
        out, dt = solve(n, K, ri, rf, "mixed", mu_stop)
        log(f"warmup {w}: {dt:.2f}s outer {out['stats'].outer_iters}")

    ot.kprof_select(a.kernel, 4)          # the FP32 instantiation of the mixed path
    its = systems = 0
    T = 0.0
    results = []
    for s in range(a.steps):
        out, dt = solve(n, K, ri, rf, "mixed", mu_stop)
        T += dt
        results.append(out)
        its += out["stats"].outer_iters
        systems += out["stats"].linear_systems
        log(f"step {s}: {dt:.2f}s outer {out['stats'].outer_iters} newton {out['stats'].newton_steps} "
            f"cost {out['cost']:.12g}")
    launches, kms, kbytes = ot.kprof_read()
    ot.kprof_select("none")
    st = results[-1]["stats"]
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
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
        "dtype": "f64 (Newton, FGMRES, Laplacian PCG vectors) + f32 (BB preconditioner kernels)",
        "data": "synthetic",
        "config": {"workload": f"BB-preconditioned interior-point solve, {n}x{n} right-triangle grid "
                               f"({2 * n * n} fine triangles), K={K}, 5-Gaussian mixtures + 1e-3 background"
                               if a.config == 3 else f"config {a.config}: {n}x{n} grid, K={K}",
                   "n": n, "K": K, "unknowns_per_newton_system": int((K + 1) * n * n + K * (n * n // 2)),
                   "continuation": (f"mu = 0.2^l from 1 down to {mu_stop:g}, each mu solved to |F| <= 1e-6"
                                    if mu_stop > 0 else "mu = 0.2^l from 1 down to the first mu below 1e-6")},
        "time_to_tol_s": T / a.steps,
        "rc": [r["rc"] for r in results],          # library status of each timed solve (0 = converged)
        "mu_final": st.mu,
        "linear_systems": systems // a.steps,
        "outer_per_linear_system": its / max(systems, 1),
        "newton_steps": st.newton_steps,
        "ip_steps": st.ip_steps,
        "inner_S_per_outer": st.inner_S_iters / max(st.prec_applies, 1),
        "inner_A_per_outer": st.inner_A_iters / max(st.prec_applies, 1),
        "failures": st.failures,
        "cost": results[-1]["cost"],
        "gap": st.gap,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": TRAFFIC_BYTES.get((a.kernel, a.config)), "traffic_unit": "bytes per launch",
                     "kernel": f"{KERNEL_NAMES.get(a.kernel, a.kernel)} (FP32)", "launches": launches,
                     "avg_us": 1000.0 * kms / launches if launches else None,
                     "bytes_per_launch": kbytes / launches if launches else None},
    }
    if not a.no_fp64:
        o64, t64 = solve(n, K, ri, rf, "fp64", mu_stop)
        log(f"fp64: {t64:.2f}s outer {o64['stats'].outer_iters} cost {o64['cost']:.12g}")
        line["fp64"] = {"time_to_tol_s": t64, "krylov_its_per_s": o64["stats"].outer_iters / t64,
                        "outer_iters": o64["stats"].outer_iters, "newton_steps": o64["stats"].newton_steps,
                        "rc": o64["rc"], "cost": o64["cost"]}
        line["cost_rel_diff_mixed_vs_fp64"] = abs(o64["cost"] - results[-1]["cost"]) / abs(o64["cost"])
        line["speedup_mixed_vs_fp64"] = t64 / (T / a.steps)
    if not a.no_cpu:
        cb = run_cpu_baseline()
        line["cpu_baseline"] = {
            "value": cb["seconds"], "unit": "s time-to-tol", "cores": 1, "kind": "oracle",
            "sample": f"full interior-point solve of the same marginal recipe on a {SAMPLE_N}x{SAMPLE_N} "
                      f"grid, K={SAMPLE_K}, tol 1e-6 (sparse direct Newton solves, 1 BLAS thread)",
            "oracle_cost": cb["cost"], "host_cpus": os.cpu_count()}
        if a.gpu_sample:
            ris, rfs = otinputs.mixture_pair(SAMPLE_N, 5, 3, background=1e-3)
            og, tg = solve(SAMPLE_N, SAMPLE_K, ris, rfs, "mixed")
            line["cpu_baseline"]["gpu_same_sample_s"] = tg
            line["cpu_baseline"]["cost_rel_diff_gpu_vs_oracle"] = abs(og["cost"] - cb["cost"]) / cb["cost"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
