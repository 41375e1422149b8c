#!/usr/bin/env python
"""Benchmark of the SG-DD-PCG hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 256x256 P1
mesh (66,049 nodes), 8x8 subdomains, KLE 4 terms, sigma 0.3, correlation
length 0.3, PCE order 3 (P = 35, 2.28 M unknowns), dt = 1e-3, PCG rtol 1e-8,
pulse centre drawn from seed 2.  A step is one Newmark time step of the whole
hot path (effective force, condensation, interface PCG with the two-level
NN preconditioner and its subdomain solves, recovery, update) with the state
resident in HBM.  Set-up (mesh, KLE/PCE, factors, coarse grid) is excluded
and reported separately.

Prints one JSON line.  Extra legs:
* accuracy: the first two steps are compared with the oracle's (relative L2
  of the mean and standard-deviation fields);
* roofline: per-launch HIP event timing of the SG apply and the subdomain
  triangular solves inside the timed region; the dominant one is reported
  against the 8 TB/s HBM peak;
* cpu_baseline: the oracle (numpy/scipy, mean-preconditioned CG) timed on
  the host for the same two steps.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SG-DD-PCG time-steps/s at ≤1e-6 rel err vs FP64 oracle; PCG iters/step; GB/s"
HBM_PEAK_GBS = 8000.0
KERNEL_NAMES = {0: "k_sg_apply (SG operator apply, K1)",
                1: "k_tri_solve (batched supernodal triangular solves, K3)"}


def traffic_from_profiles(kernel_kind):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for
    the current kernel source (profiles/traffic_*.txt), else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_k%d_cfg2.txt" % kernel_kind)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = open(os.path.join(ROOT, "paper_2512_23027_amd", "csrc", "kernels.hip"), "rb").read()
    if vals.get("kernels_hip_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(prm, nsteps):
    """The oracle timed on the host for the first nsteps steps."""
    import numpy as np
    from oracle.sg import SGProblem
    threads = 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        pass
    pr = SGProblem(prm, solver="cg")
    U, V, A = pr.initial_state()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        U, V, A = pr.step(U, V, A)
    dt = time.perf_counter() - t0
    mean, std = pr.moments(U)
    return {"value": nsteps / dt, "unit": "time-steps/s", "cores": threads, "kind": "oracle",
            "sample": "first %d time steps of the same workload (numpy/scipy FP64, CG with "
                      "the mean-matrix preconditioner to 1e-14, no domain decomposition)"
                      % nsteps}, mean, std


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the domain decomposition would shard by subdomain blocks; see DESIGN.md)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2512_23027_amd as sgw
    import workloads
    from oracle.sg import rel_l2

    torch.cuda.set_device(0)
    prm = workloads.config("cfg2")
    warm = max(args.warmup, 2)
    t0 = time.perf_counter()
    # rtol 1e-9: the workload's nominal 1e-8 leaves the standard-deviation
    # field of the first steps at ~2e-6 relative error, above the metric's
    # 1e-6 bound; Neumann solves inside the preconditioner to 1e-4 (flexible
    # interface PCG)
    rtol = 1e-9
    s = sgw.Solver(prm, rtol=rtol, inner_rtol=1e-3 * rtol, precond_rtol=1e-4)
    s.factor()
    tune = s.autotune()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    s.set_state()
    s.step(2)
    mean2, var2 = s.moments()
    mean2, std2 = mean2.cpu().numpy(), np.sqrt(var2.cpu().numpy())
    if warm > 2:
        s.step(warm - 2)
    torch.cuda.synchronize()
    s.profile(True)
    t1 = time.perf_counter()
    st = s.step(args.steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    prof = {k: s.profile_read(k) for k in (0, 1)}
    s.profile(False)
    s.close()

    kdom = max(prof, key=lambda k: prof[k][1])
    n_l, ms, nbytes = prof[kdom]
    achieved = (nbytes / (ms * 1e-3)) / 1e9 if ms > 0 else 0.0
    traffic = traffic_from_profiles(kdom)
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": warm,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "cfg2: 256x256 P1 mesh (66,049 nodes), 8x8 subdomains, KLE 4 "
                               "terms, sigma 0.3, corr. length 0.3, PCE order 3 (P=35, 2.28M "
                               "unknowns), dt 1e-3, interface rtol 1e-9 (preconditioner solves 1e-4), plain FP64 DD-PCG",
                   "global_batch": 1, "precision": "fp64"},
        "pcg_iters_per_step": st["outer_iters"] / st["steps"],
        "inner_iters_per_step": st["inner_iters"] / st["steps"],
        "setup_s": setup_s,
        "autotune_us": tune,
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[kdom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "launches": n_l, "avg_launch_us": 1e3 * ms / max(n_l, 1),
                     "algorithmic_bytes_per_launch": nbytes / max(n_l, 1)},
        "kernels": {KERNEL_NAMES[k]: {"launches": v[0], "ms": v[1],
                                      "GB/s": (v[2] / (v[1] * 1e-3)) / 1e9 if v[1] > 0 else 0}
                    for k, v in prof.items()},
    }
    if not args.no_cpu_baseline:
        cb, m_or, s_or = cpu_baseline(prm, 2)
        out["cpu_baseline"] = cb
        out["rel_err_vs_oracle"] = {"steps": 2, "mean": rel_l2(mean2, m_or),
                                    "std": rel_l2(std2, s_or)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
