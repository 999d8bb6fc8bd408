"""Benchmark: interior-point solve of the 256 x 256 right-triangle grid with
K = 64 on one MI355X (5-Gaussian-mixture marginals plus a 1e-3 background,
synthetic), mixed precision (FP32 BB preconditioner, FP64 Newton residual /
FGMRES / update) against the FP64 path; default preconditioner (BB, handing
over to SIMPLE for the late mu).

What is timed
  * time to tolerance, once per precision: the interior-point continuation
    mu = 0.2^l from 1 until the first mu below 1e-6 is solved to
    |F_mu| <= 1e-6 (ot_state_solve), with the inputs already in HBM.  Each
    run has a wall-time limit (ot_options.max_seconds); a run that hits it,
    or ends with a solver error, is reported as not reached, with the last
    mu it solved.
  * steps: one step is one inexact Newton step (residual, linearisation,
    BB-preconditioned FGMRES, recovery, line search, update) of the mixed
    path from a fixed iterate.  The iterates are snapshots taken by the
    mixed continuation at the start of every mu it reached while still on
    BB (the converged iterate of the previous mu with mu reduced, i.e. the
    first Newton system of each interior-point step), used in turn, so the
    timed steps cover the early and the late BB systems.  W untimed steps,
    then exactly K timed ones
    bracketed by device synchronisations; value = FGMRES (Krylov)
    iterations per second over them.  A deadline stops the loop early (the
    line then says how many steps ran) so that the line is always printed.
The JSON line also carries the roofline of one hot-path kernel, timed with
HIP events on the stream it runs on during the timed steps, and the
oracle's time to tolerance on a bounded sample of the same workload on the
host cores.
"""

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

T_START = time.monotonic()
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
# the CPU sample: the metric workload's marginal recipe on a reduced grid
SAMPLE_N, SAMPLE_K = 24, 12
COPY_BYTES = 1 << 30          # reference copy of the counter loop: 1 GiB read, 1 GiB written
# HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# `bench.py --counter-loop 20` (KiB per dispatch), scaled by what the same
# counters read for the 1 GiB reference copy (fetch x2.0000, write x1.0000);
# profiles/k_schur_out_256x256_K64_traffic.md.  Valid only for the kernel
# version those runs measured (XCD-banded blocks), on the 256 x 256, K = 64
# workload.
TRAFFIC_BYTES = {("schur_out", 3): 47914.7 * 1024 * 2.0 + 8192.0 * 1024 * 1.0}
KERNEL_NAMES = {"schur_out": "k_schur_out", "schur_btilde": "k_schur_btilde_tb", "cheb_fine": "k_cheb_step<., 1>",
                "tri_fine": "k_tri_scan<., 1>", "multidot": "k_multidot", "saddle_phi": "k_saddle_phi"}
METRIC = "time-to-tol (s) & Krylov iters/s, 256^2 mesh K=64: mixed vs FP64, 1 GPU"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10, help="timed Newton steps")
    p.add_argument("--warmup", type=int, default=2, help="untimed Newton steps before the timed ones")
    p.add_argument("--config", type=int, default=3, help="workload: 1, 2, 3 (256^2, K=64) or 5")
    p.add_argument("--kernel", default="schur_out", help="kernel whose roofline is reported")
    p.add_argument("--budget", type=float, default=540.0,
                   help="wall seconds (from process start) by which the line must be printed")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 time to tolerance")
    p.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    p.add_argument("--tol-only", choices=("mixed", "fp64"), default=None,
                   help="only the time to tolerance of one precision, with the whole budget (no timed steps, "
                        "no CPU sample); prints its own JSON line")
    p.add_argument("--batch", action="store_true",
                   help="instead: the 32-problem batch (grid sides 32..128, K 8..32, 1-4 Gaussians) solved by one "
                        "ot_solve_batched call, mixed precision, default preconditioner; prints its own JSON line")
    p.add_argument("--batch-streams", type=int, default=8, help="members in flight at once in --batch")
    p.add_argument("--verbose", type=int, default=0)
    p.add_argument("--cpu-sample-only", action="store_true", help=argparse.SUPPRESS)
    p.add_argument("--counter-loop", type=int, default=0,
                   help="only run N pseudo-Schur applications of the workload's mixed state and N plain "
                        "copies of a known size (for hardware-counter runs), then exit")
    return p.parse_args()


def elapsed():
    return time.monotonic() - T_START


def log(msg):
    print(f"# [{elapsed():6.1f}s] {msg}", file=sys.stderr, flush=True)


def cpu_sample():
    """The oracle's full solve of the reduced sample (run in a child process
    pinned to one BLAS thread); prints its JSON and exits."""
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


def run_cpu_baseline(timeout):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-sample-only"], env=env,
                         capture_output=True, text=True, timeout=timeout)
    if out.returncode != 0:
        raise RuntimeError("oracle sample failed: " + out.stderr[-2000:])
    return json.loads(out.stdout.strip().splitlines()[-1])


def counter_loop(a, ot, otinputs, torch):
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
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.counter_loop):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"counter_loop": a.counter_loop, "copy_bytes": COPY_BYTES, "m_rho": st.m_rho}), flush=True)


def run_batch(a, ot, otinputs, torch):
    """The 32-problem batch through one ot_solve_batched call (mixed, default
    preconditioner), after an untimed call on its two smallest members."""
    specs = [otinputs.config_marginals(4, p) for p in range(32)]
    meshes = {}
    for n, *_ in specs:
        if n not in meshes:
            meshes[n] = ot.Mesh.structured(n)
    small = sorted(range(32), key=lambda p: specs[p][0] ** 2 * specs[p][1])[:2]
    ot.solve_batched([meshes[specs[p][0]] for p in small], [specs[p][2] for p in small],
                     [specs[p][3] for p in small], [specs[p][1] for p in small], tol=1e-6,
                     batch_streams=a.batch_streams, raise_on_error=False)
    torch.cuda.synchronize()
    log("batch warm-up done")
    t0 = time.perf_counter()
    # verbose: every member's Newton steps go to stderr (progress of a long call)
    out = ot.solve_batched([meshes[n] for n, *_ in specs], [x[2] for x in specs], [x[3] for x in specs],
                           [x[1] for x in specs], tol=1e-6, batch_streams=a.batch_streams, verbose=a.verbose,
                           raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = out["stats"]
    its = sum(x.outer_iters for x in st)
    serial = sum(x.seconds_total for x in st)
    print(json.dumps({
        "metric": "32-problem batch time-to-tol (s)", "value": dt, "unit": "s", "higher_is_better": False,
        "n_gpus": 1, "rc": out["rc"], "batch_streams": a.batch_streams,
        "members_ok": int(sum(1 for x in st if x.mu < 1e-6)), "members": 32,
        "krylov_its": its, "krylov_its_per_s": its / dt, "sum_member_seconds": serial,
        "members_spec": [[n, K] for n, K, *_ in specs],
        "member_seconds": [round(x.seconds_total, 3) for x in st],
        "member_newton": [int(x.newton_steps) for x in st],
        "member_simple_systems": [int(x.simple_systems) for x in st],
        "dtype": "f64 + f32 (BB preconditioner kernels)", "data": "synthetic", "wall_s": elapsed()}), flush=True)


def main():
    a = parse()
    if a.cpu_sample_only:
        cpu_sample()
        return
    if a.gpus != 1:
        print("bench.py measures one GPU: the solver runs one problem per GPU and this build has no "
              "multi-GPU path; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch

    import otinputs
    import paper_2209_00315_amd as ot

    torch.cuda.set_device(0)
    dev = torch.device("cuda")
    if a.counter_loop > 0:
        counter_loop(a, ot, otinputs, torch)
        return

    if a.batch:
        run_batch(a, ot, otinputs, torch)
        return

    n, K, ri, rf = otinputs.config_marginals(a.config)
    mesh = ot.Mesh.structured(n)
    ri_d = torch.as_tensor(ri, dtype=torch.float64, device=dev)
    rf_d = torch.as_tensor(rf, dtype=torch.float64, device=dev)
    log(f"workload n={n} K={K}; budget {a.budget:.0f}s")

    def state(prec, **kw):
        return ot.State(mesh, ri_d, rf_d, K, device=True, precision=prec, verbose=a.verbose, **kw)

    # code-object load and first allocations outside every timed region: one
    # Newton step of the same problem in each precision
    for prec in ("mixed", "fp64"):
        stw = state(prec)
        stw.newton_step(raise_on_error=False)
        del stw
    torch.cuda.synchronize()
    log("warm-up Newton steps done")

    def remaining():
        return a.budget - elapsed()

    def time_to_tol(prec, limit, snapshots=None):
        """Continuation from the start point in one state; mu by mu through
        ot_state_solve with mu_stop, so that the iterate at the start of each
        mu can be kept.  Returns a summary dict."""
        st = state(prec, max_seconds=max(limit, 1.0))
        mu, mus = 1.0, []
        while True:
            mus.append(mu)
            if mu < 1e-6:
                break
            mu *= 0.2
        its = systems = newton = fails = simple = 0
        rc, mu_done = ot.OT_OK, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for mu_l in mus:
            # snapshots only while every system so far was solved with BB:
            # the timed steps measure the BB-preconditioned path
            if snapshots is not None and mu_l < 1.0 and simple == 0:
                # the converged iterate of the previous mu, with mu reduced
                phi, rho, s, _ = st.export()
                snapshots.append((phi, rho, s, mu_l))
            left = limit - (time.perf_counter() - t0)
            if left <= 0:
                rc = ot.OT_ETIME
                break
            st.set_options(mu_stop=mu_l * (1 + 1e-9), max_seconds=left)
            rc, stt = st.solve(1e-6, raise_on_error=False)
            its += stt.outer_iters
            systems += stt.linear_systems
            newton += stt.newton_steps
            fails += stt.failures
            simple += stt.simple_systems
            if rc != ot.OT_OK:
                break
            mu_done = stt.mu
            log(f"{prec}: mu {mu_l:.3e} solved: Newton {stt.newton_steps} FGMRES {stt.outer_iters} "
                f"SIMPLE systems {stt.simple_systems} t {time.perf_counter() - t0:.1f}s")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        cost, dual, _ = st.outputs()
        reached = rc == ot.OT_OK and mu_done is not None and mu_done < 1e-6
        return {"reached": reached, "time_to_tol_s": dt if reached else None, "seconds_run": dt, "rc": rc,
                "mu_last_solved": mu_done, "newton_steps": newton, "linear_systems": systems,
                "outer_iters": its, "krylov_its_per_s": its / dt if dt > 0 else None, "failures": fails,
                "simple_systems": simple,
                "cost": cost, "gap": cost - dual, "limit_s": limit}

    if a.tol_only:
        r = time_to_tol(a.tol_only, max(30.0, remaining() - 15.0))
        print(json.dumps({"metric": "time-to-tol (s), " + METRIC.split(", ", 1)[1], "precision": a.tol_only,
                          "value": r["time_to_tol_s"], "unit": "s", "higher_is_better": False,
                          "config": {"n": n, "K": K, "config": a.config}, **r, "wall_s": elapsed()}), flush=True)
        return

    # order: mixed continuation (it records the snapshots), the timed steps,
    # the FP64 continuation, the CPU sample; each stage leaves the later
    # ones a reserve so that the line is printed within the budget
    cpu_reserve = 0.0 if a.no_cpu else 25.0
    step_reserve = 12.0 + 2.5 * (a.steps + a.warmup)
    snaps = []
    mixed = time_to_tol("mixed", max(30.0, remaining() - step_reserve - cpu_reserve - 15.0), snaps)
    log(f"mixed continuation: {mixed}")

    # timed Newton steps of the mixed path from the snapshots, in turn
    st = state("mixed")
    deadline = a.budget - cpu_reserve - 15.0
    order = list(range(len(snaps))) if snaps else []

    def one_step(i):
        phi, rho, s, mu = snaps[order[i % len(order)]]
        st.import_(phi, rho, s, mu)
        rc, stt, _ = st.newton_step(raise_on_error=False)
        return stt.outer_iters

    for w in range(a.warmup):
        if not order or elapsed() > deadline:
            break
        one_step(w)
    ot.kprof_select(a.kernel, 4)          # the FP32 instantiation of the mixed path
    its = done = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        if not order or elapsed() > deadline:
            break
        its += one_step(k)
        done += 1
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    launches, kms, kbytes = ot.kprof_read()
    ot.kprof_select("none")
    log(f"timed steps: {done} of {a.steps}, {its} FGMRES its in {T:.2f}s")
    del st

    fp64 = None
    if not a.no_fp64:
        fp64 = time_to_tol("fp64", max(30.0, remaining() - cpu_reserve - 10.0))
        log(f"fp64 continuation: {fp64}")
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else None
    line = {
        "metric": METRIC,
        "value": its / T if T > 0 and done else None,
        "unit": "Krylov it/s",
        "n_gpus": 1,
        "steps": done,
        "steps_requested": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1000.0 * T / done if done else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (residual, FGMRES, update, Laplacian PCG vectors, SIMPLE) + f32 (BB preconditioner kernels)",
        "data": "synthetic",
        "config": {"workload": f"interior-point solve (BB preconditioner, SIMPLE for late mu), "
                               f"{n}x{n} right-triangle grid "
                               f"({2 * n * n} fine triangles), K={K}, "
                               + ("5-Gaussian mixtures + 1e-3 background" if a.config == 3 else
                                  f"benchmark configuration {a.config}"),
                   "n": n, "K": K, "unknowns_per_newton_system": int((K + 1) * n * n + K * (n * n // 2)),
                   "step": "one inexact Newton step of the mixed path from a snapshot iterate (the first "
                           "Newton system of each interior-point step reached while the continuation "
                           "still ran on the BB preconditioner), snapshots in turn",
                   "snapshots_mu": [x[3] for x in snaps]},
        "time_to_tol_s": mixed["time_to_tol_s"],
        "mixed": mixed,
        "fp64": fp64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": TRAFFIC_BYTES.get((a.kernel, a.config)),
                     "kernel": f"{KERNEL_NAMES.get(a.kernel, a.kernel)} (FP32)", "launches": launches,
                     "avg_us": 1000.0 * kms / launches if launches else None,
                     "bytes_per_launch": kbytes / launches if launches else None},
    }
    if fp64 is not None:
        if mixed["reached"] and fp64["reached"]:
            line["speedup_mixed_vs_fp64"] = fp64["time_to_tol_s"] / mixed["time_to_tol_s"]
            line["cost_rel_diff_mixed_vs_fp64"] = abs(fp64["cost"] - mixed["cost"]) / abs(fp64["cost"])
    if not a.no_cpu:
        try:
            cb = run_cpu_baseline(timeout=max(10.0, a.budget - 10.0 - elapsed()))
            line["cpu_baseline"] = {
                "value": cb["seconds"], "unit": "s time-to-tol", "cores": 1, "kind": "oracle",
                "sample": f"full interior-point solve of the same marginal recipe on a {SAMPLE_N}x{SAMPLE_N} "
                          f"grid, K={SAMPLE_K}, tol 1e-6 (sparse direct Newton solves, 1 BLAS thread)",
                "oracle_cost": cb["cost"], "host_cpus": os.cpu_count()}
            ris, rfs = otinputs.mixture_pair(SAMPLE_N, 5, 3, background=1e-3)
            ms = ot.Mesh.structured(SAMPLE_N)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            og = ot.solve(ms, ris, rfs, SAMPLE_K, tol=1e-6, precision="mixed", raise_on_error=False)
            tg = time.perf_counter() - t0
            line["cpu_baseline"]["gpu_same_sample_s"] = tg
            line["cpu_baseline"]["cost_rel_diff_gpu_vs_oracle"] = abs(og["cost"] - cb["cost"]) / cb["cost"]
        except Exception as e:  # the line is printed in any case
            line["cpu_baseline"] = {"value": None, "error": str(e)[:300]}
    line["wall_s"] = elapsed()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
