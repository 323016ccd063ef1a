#!/usr/bin/env python3
"""EGFEM Newton hot-path benchmark on one MI355X.

A step is one complete EGFEM Newton solve (pointwise coefficient update fused
into the tensor actions, residual action, Jacobian emission, Jacobi-BiCGStab,
damped update) of the 2D nonlinear-diffusion workload
-div((1+u^2) grad u) = f on the 256x256 right-triangle P1 mesh (66,049 nodes),
from u = 0 to ||F|| <= 1e-10 ||F(0)||, inputs resident in HBM.  The offline
tensor build is not timed (the paper's online-time convention).

Prints ONE JSON line (rank 0).  Extra keys report the tensor-action kernels
alone (warm and cache-flushed), the per-kernel split of the solve and the CPU
oracle timed on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "tensor-action GB/s + Newton solves/s (FP64, rel. 1e-10) vs per-instance"


# ----------------------------------------------------------------------------
# algorithmic bytes of one launch of each kernel (every stored tensor value and
# index, every pattern array and every vector touched once)
# ----------------------------------------------------------------------------
def bytes_action_raw(info):
    N, S, Z = info.n_nodes, info.slots, info.nnz
    return 12 * Z + 8 * S + 4 * (N + 1) + 24 * N           # vA,kA | kptr,col | rowptr | u,a,r


def bytes_action_problem(info, trial: bool):
    N, S, Z = info.n_nodes, info.slots, info.nnz
    vec = 8 * N * (3 + (2 if trial else 0)) + N             # u,d,F [+delta,u_try] + mask
    return 12 * Z + 8 * S + 4 * (N + 1) + vec


def bytes_jacobian(info):
    N, S, Z = info.n_nodes, info.slots, info.nnz
    streams = 12 * Z + (0 if info.symmetric else 12 * Z)    # A (+ B) streams
    ptrs = 4 * (S + 1) * (1 if info.symmetric else 2) + 4 * S + 4 * (N + 1)
    return streams + ptrs + 8 * N + N + 8 * S + 8 * N         # u, mask, J values, 1/diag


def bytes_krylov(info, iters: int):
    """Per BiCGStab iteration: two passes over J (values + columns + row
    pointers; the first gathers two vectors), and the row-local vector phases:
    A 56N (gather phat, rh; write v, z, vhat; read 1/diag, rhat), B 56N (gather
    vhat; read v, r, z, rhat; write s, t), C 96N (read 1/diag, s, phat, x, t, v, p;
    write x, r, p, phat, rh)."""
    N, S = info.n_nodes, info.slots
    per_iter = 24 * S + 8 * (N + 1) + 208 * N
    setup = 16 * N + 48 * N                                  # rhs, 1/diag | x, r, rhat, p, phat, rh
    return iters * per_iter + setup


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_06193_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str):
    """HBM traffic per launch measured with rocprofv3 --pmc (FETCH_SIZE,
    WRITE_SIZE), scaled by a copy kernel; None when absent or stale."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    ent = d.get(kernel)
    if not ent or ent.get("source_sha") != kernel_source_sha():
        return None
    return ent.get("bytes_per_launch")


# ----------------------------------------------------------------------------
def gpu_setup(n: int):
    import numpy as np
    import torch
    import paper_2005_06193_amd as eg
    import workloads as W

    wl = W.nonlinear_diffusion_2d(n)
    T = eg.Tensor.from_mesh(wl.mesh, wl.form)
    dev = torch.device("cuda:0")
    f = torch.tensor(wl.f, dtype=torch.float64, device=dev)
    load = T.matvec(f, "M")
    dirm = torch.tensor(wl.mesh.dirichlet, dtype=torch.uint8, device=dev)
    p = eg.Problem(T.n, load, dirm, None, 1.0, False)
    torch.cuda.synchronize()
    return wl, T, p


def time_solves(T, p, steps: int, warmup: int, opts):
    import torch
    u = torch.zeros(T.n, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        u.zero_()
        T.newton(p, u, opts)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        u.zero_()
        stats.append(T.newton(p, u, opts))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, stats, u


def time_action(T, reps: int, cold: bool):
    """Raw tensor action r = T:(u (x) a) launched back to back (warm), or with
    a 1 GiB overwrite between launches so the stream comes from HBM (cold).
    Times with torch events on the stream the library launches on."""
    import torch
    n = T.n
    g = torch.Generator(device="cuda").manual_seed(5)
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    a = torch.rand(n, dtype=torch.float64, device="cuda", generator=g) + 1.0
    r = torch.empty_like(u)
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda") if cold else None
    for _ in range(5):
        T.residual(u, a, r)
    torch.cuda.synchronize()
    if not cold:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            T.residual(u, a, r)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    tot = 0.0
    for i in range(reps):
        flush.fill_(float(i))
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        T.residual(u, a, r)
        e1.record()
        torch.cuda.synchronize()
        tot += e0.elapsed_time(e1)
    return tot / reps


def time_jacobian(T, p, reps: int):
    import torch
    u = torch.rand(T.n, dtype=torch.float64, device="cuda")
    jv = torch.empty(T.info.slots, dtype=torch.float64, device="cuda")
    dinv = torch.empty(T.n, dtype=torch.float64, device="cuda")
    for _ in range(5):
        T.problem_jacobian(p, u, jv, dinv)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        T.problem_jacobian(p, u, jv, dinv)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(n: int, budget_s: float = 20.0):
    """The CPU oracle (numpy/scipy, SuperLU direct solves) on the same workload:
    EGFEM Newton solves, plus one SGA (re-assembly) solve for context."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as W
    from oracle import egfem_oracle as O

    with threadpool_limits(limits=1):
        wl = W.nonlinear_diffusion_2d(n)
        prob = O.build_problem(wl)
        times = []
        t_start = time.perf_counter()
        while True:
            t0 = time.perf_counter()
            O.newton(prob, tol=wl.tol)
            times.append(time.perf_counter() - t0)
            if time.perf_counter() - t_start > budget_s * 0.6 or len(times) >= 5:
                break
        t0 = time.perf_counter()
        _, sst = O.sga_newton(prob, tol=wl.tol)
        t_sga = time.perf_counter() - t0
    egfem_s = sum(times) / len(times)
    return {
        "value": 1.0 / egfem_s,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{len(times)} full EGFEM Newton solve(s) of the same 66,049-node workload "
                  f"(numpy/scipy, SuperLU direct solves, tol 1e-10), mean {egfem_s:.3f} s; "
                  f"one SGA re-assembly Newton solve took {t_sga:.3f} s",
        "sga_solves_per_s": 1.0 / t_sga,
        "cpu": _cpu_model(),
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-micro", action="store_true", help="skip the tensor-action microbenchmarks")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the build targets a single MI355X); "
              f"--gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_06193_amd as eg

    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        sys.exit(1)
    wl, T, p = gpu_setup(args.n)
    info = T.info
    opts = eg.NewtonOptions(tol=wl.tol, forcing=1, timing=1)
    elapsed, stats, u = time_solves(T, p, args.steps, args.warmup, opts)
    ok = all(s.status == 0 and s.res <= wl.tol * s.res0 for s in stats)
    ms_per_step = 1000.0 * elapsed / args.steps
    solves_per_s = args.steps / elapsed

    # per-kernel split over the timed region (events inside the driver)
    t_act = sum(s.t_action_ms for s in stats)
    n_act = sum(s.n_action for s in stats)
    t_jac = sum(s.t_jacobian_ms for s in stats)
    n_jac = sum(s.n_jacobian for s in stats)
    t_kry = sum(s.t_krylov_ms for s in stats)
    n_kry = sum(s.n_krylov for s in stats)
    k_it = sum(s.krylov_iters for s in stats)
    n_trial = n_act - len(stats)
    b_act = len(stats) * bytes_action_problem(info, False) + n_trial * bytes_action_problem(info, True)
    b_jac = n_jac * bytes_jacobian(info)
    b_kry = sum(bytes_krylov(info, it) for s in stats for it in s.krylov_hist)
    kernels = {
        "krylov_bicgstab": {"ms": t_kry, "launches": n_kry, "bytes": b_kry,
                            "GBps": b_kry / (t_kry * 1e6) if t_kry else None,
                            "iters_per_solve": k_it / len(stats)},
        "tensor_action": {"ms": t_act, "launches": n_act, "bytes": b_act,
                          "GBps": b_act / (t_act * 1e6) if t_act else None},
        "jacobian_emission": {"ms": t_jac, "launches": n_jac, "bytes": b_jac,
                              "GBps": b_jac / (t_jac * 1e6) if t_jac else None},
    }
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    dk = kernels[dom]
    avg_ms = dk["ms"] / dk["launches"]
    bytes_per_launch = dk["bytes"] / dk["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e6)
    traffic = load_traffic(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch}

    micro = None
    if not args.no_micro:
        warm = time_action(T, 200, cold=False)
        cold = time_action(T, 30, cold=True)
        jac = time_jacobian(T, p, 200)
        ba = bytes_action_raw(info)
        bj = bytes_jacobian(info)
        micro = {
            "residual_action": {"bytes": ba, "warm_us": warm * 1e3, "warm_GBps": ba / (warm * 1e6),
                                "cold_us": cold * 1e3, "cold_GBps": ba / (cold * 1e6),
                                "cold_frac": ba / (cold * 1e6) / HBM_PEAK_GBS,
                                "nnz_per_s_warm": info.nnz / (warm * 1e-3)},
            "jacobian_emission": {"bytes": bj, "warm_us": jac * 1e3, "warm_GBps": bj / (jac * 1e6)},
        }

    cpu = None if args.no_cpu else cpu_baseline(args.n)
    out = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"nonlinear_diffusion_2d_{args.n}x{args.n}_p1",
                   "nodes": info.n_nodes, "tensor_nnz": info.nnz, "slots": info.slots,
                   "newton_tol": wl.tol, "forcing": "eisenstat-walker-2",
                   "krylov": "bicgstab-jacobi"},
        "converged": ok,
        "newton_iters_per_solve": sum(s.newton_iters for s in stats) / len(stats),
        "roofline": roofline,
        "kernels": kernels,
        "tensor_action": micro,
        "cpu_baseline": cpu,
    }
    if cpu:
        out["speedup_vs_cpu_oracle"] = solves_per_s / cpu["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
