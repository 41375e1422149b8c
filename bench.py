#!/usr/bin/env python
"""Benchmark of the SG-DD-PCG hot path on one MI355X.

Workload (default, the largest configuration; one GPU holds it): 512x512 P1
mesh (263,169 nodes), 16x16 subdomains, KLE 8 terms, sigma 0.3, correlation
length 0.25, PCE order 3 (P = 165, 43.1 M SG unknowns), dt = 1e-3, rtol
1e-8, pulse centre drawn from seed 5.  A step is one Newmark time step of
the whole hot path (effective force, condensation, interface PCG with the
two-level NN preconditioner and its batched subdomain solves, recovery,
update) with the state resident in HBM.  Set-up (mesh, KLE/PCE, factors,
coarse grid, autotuning) is excluded and reported separately.

Two solver stacks run on the same GPU, one after the other:
* full stack (the headline value): FP32 DD-PCG inside FP64 iterative
  refinement of the whole SG system (relative SG residual <= 1e-8 per
  step; FP32 interface PCG and Dirichlet solves to 3e-5, Neumann solves to
  1e-2), batched subdomain solves with the degree-8 Chebyshev mean-matrix
  preconditioner and autotuned tiles, Newmark-extrapolated initial guess;
* plain FP64 DD-PCG (the paper's method: previous-solution guess, FP64
  throughout, interface rtol 1e-9).
--workload cfg2 runs the 256x256, P = 35 configuration instead.

Prints one JSON line.  Extra legs:
* accuracy: after the timed steps each stack runs on to the stored oracle
  steps beyond them, then restarts from the initial state for the stored
  steps it passed; the mean and standard-deviation fields over all mesh
  nodes are compared with the stored oracle values
  (tests/golden/<workload>_oracle.npz, written from the oracle alone) at
  every stored step (relative L2); accuracy_ok needs a comparison after the
  timed steps;
* roofline: per-launch HIP event timing of the kernel kinds inside the timed
  region; the dominant one is reported against its roofline (HBM bytes or
  FP32 vector arithmetic, whichever bounds it), with the HBM traffic per
  launch that rocprofv3 counters measured for the same kernel in this
  command (profiles/<kernel>_traffic.json, used only while the kernel's
  generated source is unchanged);
* cpu_baseline: the oracle (numpy/scipy FP64, mean-preconditioned CG, no
  domain decomposition) on the host: a bounded sample of its first time step
  (see cpu_baseline()).

--copy-calibration runs only a plain device copy of known size (the
reference kernel for scaling HBM traffic counters).
"""

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("SGW_PROGRESS", "1")  # set-up stages on stderr

METRIC = "SG-DD-PCG time-steps/s at ≤1e-6 rel err vs FP64 oracle; PCG iters/step; GB/s"
HBM_PEAK_GBS = 8000.0
# MI355X vector peaks (256 CUs, 2.4 GHz): FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s
# with packed (two-per-lane) FMAs, which this build does not emit, so its
# FP32 code can reach at most the 78.6 of one FMA per lane per clock
FP32_VECTOR_PEAK_TFS = 157.3
FP64_VECTOR_PEAK_TFS = 78.6
KERNEL_NAMES = {0: "k1 SG operator apply, FP64 (K1)",
                1: "k_tri_solve batched supernodal triangular solves, FP64 (K3)",
                2: "k_cheb Chebyshev subdomain preconditioner, FP64 (K3c)",
                3: "k1 SG operator apply, FP32 (K1)",
                4: "k_tri_solve batched supernodal triangular solves, FP32 (K3)",
                5: "k_cheb Chebyshev subdomain preconditioner, FP32 (K3c)"}
PROFILE_EVERY = 7    # time every 7th launch of each kind: a prime, so that the sample rotates
                     # over the positions of a step (50 SG applies per step at 512x512; every
                     # 5th launch saw the same 10 positions in every step)

WORKLOADS = {
    "cfg5": "cfg5: 512x512 P1 mesh (263,169 nodes), 16x16 subdomains, KLE 8 terms, sigma 0.3, "
            "corr. length 0.25, PCE order 3 (P=165, 43.1M SG unknowns), dt 1e-3, pulse seed 5",
    "cfg2": "cfg2: 256x256 P1 mesh (66,049 nodes), 8x8 subdomains, KLE 4 terms, sigma 0.3, "
            "corr. length 0.3, PCE order 3 (P=35, 2.28M SG unknowns), dt 1e-3, pulse seed 2",
    "cfg3": "cfg3: 8 independent 384x384 problems (148,225 nodes each), seeded uneven "
            "rectilinear splits (8-10 strips per side), sigma ~ U[0.1, 0.4], corr. length ~ "
            "U[0.2, 0.6], KLE 6 terms, PCE order 3 (P=84, 12.3M SG unknowns each), dt 1e-3, "
            "seeds 300-307, advanced together by sgw_step_batch",
}


def sg_apply_counts(prm):
    """(algorithmic bytes per row of one FP32 SG apply, flops per row, bytes
    per row of the fused PCG update): 7 (M+1) matrix values + 7 column
    indices + one vector in and one out (P modes each), 4-byte values; the
    fused p update reads z and writes p as well (two more vectors); flops =
    2 (7 |KJ| + nnz(c)) with |KJ| the distinct (k, j) pairs of the Galerkin
    tensor (each W_kj = K_k x_j costs 7 FMAs, each tensor entry one FMA)."""
    from paper_2512_23027_amd import gen_k1
    nk, P, ent = gen_k1.entries(prm["L"], prm["p_in"], prm["p_out"])
    kj = {(e[0], e[2]) for e in ent}
    bpr = 7 * nk * 4 + 7 * 4 + 2 * P * 4
    fpr = 2 * (7 * len(kj) + len(ent))
    return bpr, fpr, 2 * P * 4


def measured_traffic(prm, kind):
    """HBM bytes per dispatch of the dominant kernel from rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads for a
    plain copy of known size), stored under profiles/ by the run that took
    them together with a hash of the kernel's generated source; None when
    there is no such record or the source has changed since."""
    import hashlib
    if kind != 3:
        return None
    from paper_2512_23027_amd import gen_k1
    tag = gen_k1.tag(prm["L"], prm["p_in"], prm["p_out"])
    path = os.path.join(ROOT, "profiles", "%s_pcg_f_traffic.json" % tag)
    src = os.path.join(ROOT, "paper_2512_23027_amd", "csrc", "k1_gen_L%d_%d_%d.hip"
                       % (prm["L"], prm["p_in"], prm["p_out"]))
    if not (os.path.exists(path) and os.path.exists(src)):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return {"bytes_per_dispatch": rec["fetch_bytes"] + rec["write_bytes"],
            "source": "profiles/%s_pcg_f_traffic.json" % tag}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(prm, golden_steps):
    """The oracle on the host, on a bounded sample of the same workload.

    Full oracle steps take minutes at the largest size, so the sample is its
    first time step's conjugate-gradient work, timed for as many CG
    iterations as fit in about 20 s: each CG iteration is one SG operator
    apply plus one mean-matrix preconditioner solve (the oracle's own
    apply_Kt and factor), and a step costs the per-step iteration count the
    oracle reports for this workload (its golden run).  Returns the rate in
    time-steps/s."""
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
    import scipy.sparse.linalg as spla
    lu = spla.splu(pr.Kt[0].tocsc())
    its, t0, c0 = 0, time.perf_counter(), time.process_time()
    while True:  # the two operations of a CG iteration on the step's vectors
        Q = pr.apply_Kt(U)
        lu.solve(Q)
        its += 1
        if time.perf_counter() - t0 > 20.0:
            break
    wall = time.perf_counter() - t0
    per_it = wall / its
    busy = (time.process_time() - c0) / wall  # cores kept busy on average
    cg_per_step = golden_steps.get("cg_iterations_per_step")
    if not cg_per_step:
        return None
    return {"value": 1.0 / (per_it * cg_per_step), "unit": "time-steps/s",
            "cores": max(1, int(round(busy))), "kind": "oracle", "cpu_model": cpu_model(),
            "host_cpus": os.cpu_count(),
            "threads_note": "cores = process CPU time / wall time over the sample (%.2f): %d BLAS "
                            "threads in the dense Galerkin contractions, scipy's sparse products "
                            "and triangular solves on one thread" % (busy, threads),
            "sample": "%d CG iterations (SG operator apply + mean-matrix preconditioner solve, "
                      "%.2f s each) of the oracle's first time step, scaled by the %.1f CG "
                      "iterations per step the oracle takes on this workload"
                      % (its, per_it, cg_per_step)}


def solver_settings(precision="mixed"):
    """Solver options of the two timed stacks."""
    import paper_2512_23027_amd as sgw
    if precision == "fp64":
        # the nominal 1e-8 leaves the standard deviation of the first steps
        # at ~2e-6 relative error on this path; 1e-9 keeps it below 1e-6
        return dict(precision=sgw.SGW_FP64, guess=sgw.SGW_GUESS_PREV, rtol=1e-9,
                    inner_rtol=1e-12, precond_rtol=1e-4, inner_prec=sgw.SGW_INNER_CHEBYSHEV,
                    cheb_degree=8)
    # refinement sweeps: FP32 interface PCG and Dirichlet solves to 3e-5,
    # Neumann solves to 1e-2 (500 steps of the 256x256 workload stay within
    # 3.3e-7 of the oracle)
    return dict(precision=sgw.SGW_FP32_IR64, guess=sgw.SGW_GUESS_NEWMARK, rtol=1e-8,
                inner_rtol=1e-11, precond_rtol=1e-4, inner_prec=sgw.SGW_INNER_CHEBYSHEV,
                cheb_degree=8, ir_rtols=(3e-5, 3e-5, 1e-2))


def copy_calibration(nbytes=1 << 30, reps=10):
    """A plain elementwise copy kernel (y = 1.0 * x) over nbytes, reps times."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}))


def write_traffic(kernel_re, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv,
                  workload="cfg5", nbytes=1 << 30, reps=10):
    """profiles/<basis>_pcg_f_traffic.json from rocprofv3 counter CSVs: the
    dominant kernel's FETCH_SIZE and WRITE_SIZE (KiB per dispatch, averaged
    over its dispatches), each scaled by the ratio of the bytes a plain copy
    moved (--copy-calibration: one fill of nbytes, then reps copies
    reading and writing nbytes) to what the same counter read for it."""
    import csv
    import hashlib
    import re

    import workloads
    from paper_2512_23027_amd import gen_k1

    def per_kernel(path, counter, pat):
        tot, n = 0.0, 0
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] == counter and re.search(pat, r["Kernel_Name"]):
                tot += float(r["Counter_Value"])
                n += 1
        return tot, n

    cf, _ = per_kernel(copy_fetch_csv, "FETCH_SIZE", "elementwise")
    cw, _ = per_kernel(copy_write_csv, "WRITE_SIZE", "elementwise")
    f_scale = reps * nbytes / (cf * 1024.0)
    w_scale = (reps + 1) * nbytes / (cw * 1024.0)
    kf, nf = per_kernel(fetch_csv, "FETCH_SIZE", kernel_re)
    kw, nw = per_kernel(write_csv, "WRITE_SIZE", kernel_re)
    prm = workloads.config(workload)
    tag = gen_k1.tag(prm["L"], prm["p_in"], prm["p_out"])
    src = os.path.join(ROOT, "paper_2512_23027_amd", "csrc", "k1_gen_L%d_%d_%d.hip"
                       % (prm["L"], prm["p_in"], prm["p_out"]))
    rec = {"kernel": kernel_re, "workload": workload, "dispatches": [nf, nw],
           "fetch_bytes": kf * 1024.0 * f_scale / max(nf, 1),
           "write_bytes": kw * 1024.0 * w_scale / max(nw, 1),
           "fetch_scale": f_scale, "write_scale": w_scale,
           "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest()}
    out = os.path.join(ROOT, "profiles", "%s_pcg_f_traffic.json" % tag)
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def trace_window(trace_csv, steps):
    """Per-kernel time inside the first timed region of a rocprofv3 kernel
    trace of this command (between the first two marker kernels), per step."""
    import collections
    import csv
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Start_Timestamp"]))
    marks = [i for i, r in enumerate(rows) if "spin" in r["Kernel_Name"]
             or "sleep" in r["Kernel_Name"].lower()]
    a, b = marks[0], marks[1]
    t0, t1 = int(rows[a]["End_Timestamp"]), int(rows[b]["Start_Timestamp"])
    busy, cnt = collections.defaultdict(int), collections.Counter()
    for r in rows[a + 1:b]:
        k = r["Kernel_Name"].split("(")[0].replace("void ", "")
        busy[k] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        cnt[k] += 1
    kt = sum(busy.values())
    print("timed region: %.3f ms per step, kernels %.3f ms per step, %d launches per step, "
          "idle %.1f%%" % ((t1 - t0) / 1e6 / steps, kt / 1e6 / steps, sum(cnt.values()) // steps,
                           100.0 * (t1 - t0 - kt) / (t1 - t0)))
    print("| kernel | launches/step | ms/step | share | avg us |")
    print("|---|---|---|---|---|")
    for k, v in sorted(busy.items(), key=lambda x: -x[1])[:20]:
        print("| %s | %.1f | %.3f | %.1f%% | %.1f |" % (k, cnt[k] / steps, v / 1e6 / steps,
                                                      100.0 * v / (t1 - t0), v / 1e3 / cnt[k]))


def load_golden(name):
    """{step: (mean, std)} of the stored oracle run, and its metadata."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "%s_oracle.npz" % name)
    if not os.path.exists(path):
        return {}, {}
    z = np.load(path, allow_pickle=False)
    out = {int(s): (z["mean_%d" % s], z["std_%d" % s]) for s in z["steps"]}
    meta = {}
    if "cg_iterations" in z.files:
        meta["cg_iterations_per_step"] = float(np.mean(z["cg_iterations"]))
    return out, meta


def pulse_modes(prm, P, seed):
    """Initial displacement chaos coefficients [P][(n+1)^2] of the workload's
    problem with its pulse centred where `seed` draws it (mode 0 only): the
    input of a training trajectory of the learned guess."""
    import numpy as np
    import workloads
    n = prm["n"]
    x0, y0 = workloads.pulse_centre(seed)
    x = np.tile(np.arange(n + 1) / n, n + 1)
    y = np.repeat(np.arange(n + 1) / n, n + 1)
    u = np.zeros((P, (n + 1) ** 2))
    u[0] = prm["amp"] * np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / prm["width"] ** 2)
    return u


# learned guess of the full stack: trained, after the set-up, on trajectories
# of the same problem with the pulse elsewhere (seeds other than the timed one)
LEARN = dict(seeds=(51, 52), nsteps=10, epochs=1, batch=16384, lr=1e-3)


def run_stack(sgw, prm, opts, warm, steps, golden, log, learn=None):
    """Set up one solver stack, time `steps` steps after `warm` warm-up steps,
    then rerun from the initial state to the stored oracle steps.  learn: train
    the learned guess first (LEARN) and time the stack with it."""
    import numpy as np
    import torch
    from oracle.sg import rel_l2
    t0 = time.perf_counter()
    s = sgw.Solver(prm, **opts)
    log("context created (%.1f s)" % (time.perf_counter() - t0))
    s.factor()
    log("coarse grid factored (%.1f s)" % (time.perf_counter() - t0))
    tune = s.autotune()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log("autotuned; set-up %.1f s" % setup_s)
    train = None
    if learn:
        t2 = time.perf_counter()
        model = sgw.GuessModel(4, 1, 256, seed=7)
        s.set_guess_model(model)
        s.set_guess(sgw.SGW_GUESS_NEWMARK)
        loss = 0.0
        for q, sd in enumerate(learn["seeds"]):
            s.set_state(U=torch.from_numpy(pulse_modes(prm, s.P, sd)))
            last = q + 1 == len(learn["seeds"])
            loss = s.guess_train(learn["nsteps"], epochs=learn["epochs"] if last else 0,
                                 batch=learn["batch"], lr=learn["lr"], seed=2, clear=q == 0)
            log("learned guess: trajectory %d recorded%s (%.1f s)"
                % (q + 1, ", network trained" if last else "", time.perf_counter() - t2))
        s.set_guess(sgw.SGW_GUESS_LEARNED)
        torch.cuda.synchronize()
        train = {"trajectories": len(learn["seeds"]), "steps_each": learn["nsteps"],
                 "samples": s.stored_samples(), "epochs": learn["epochs"],
                 "final_loss": loss, "seconds": time.perf_counter() - t2}
        log("learned guess trained: %s" % train)
    s.set_state()
    if warm:
        s.step(warm)
    # marker kernels just outside the timed region (a kernel trace of this
    # command splits at them: --trace-window)
    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    s.profile(True, every=PROFILE_EVERY)
    t1 = time.perf_counter()
    st = s.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    torch.cuda._sleep(1000)
    prof = {k: s.profile_read(k) for k in range(6)}
    s.profile(False)
    log("timed %d steps: %.3f s" % (steps, elapsed))
    errors = []

    def compare(step, after):
        m, v = s.moments()
        gm, gs = golden[step]
        errors.append({"step": step, "after_timing": after,
                       "mean": rel_l2(m.cpu().numpy(), gm),
                       "std": rel_l2(np.sqrt(v.cpu().numpy()), gs)})

    if golden:
        # the timed trajectory itself continues to the stored steps after it
        done = warm + steps
        for step in [g for g in sorted(golden) if g >= done]:
            s.step(step - done)
            done = step
            compare(step, True)
        # the stored steps it passed: the same trajectory again from the start
        earlier = [g for g in sorted(golden) if g < warm + steps]
        if earlier:
            s.set_state()
            done = 0
            for step in earlier:
                s.step(step - done)
                done = step
                compare(step, False)
        log("accuracy: %s" % errors)
    fallbacks = s.guess_fallbacks() if learn else None
    s.close()
    return {"steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "learned_guess": train, "guess_fallbacks": fallbacks,
            "pcg_iters_per_step": st["outer_iters"] / st["steps"],
            "inner_iters_per_step": st["inner_iters"] / st["steps"],
            "ir_sweeps_per_step": st["ir_sweeps"] / st["steps"], "setup_s": setup_s,
            "autotune_us": tune, "prof": prof, "errors": errors}


def run_batch(sgw, names, opts, warm, steps, log):
    """The batched workload: every problem set up, then advanced together
    (sgw_step_batch: one stream and host thread per problem); the timed
    region covers `steps` batched steps.  Problems with stored oracle values
    are compared after the timed steps (the trajectory run on to the stored
    steps beyond them) and, for stored steps it passed, after a rerun of the
    batch from the initial states."""
    import numpy as np
    import torch
    from oracle.sg import rel_l2
    import workloads
    t0 = time.perf_counter()
    ss = []
    for nm in names:
        s = sgw.Solver(workloads.config(nm), **opts)
        s.factor()
        s.autotune()
        s.set_state()
        ss.append(s)
        log("%s set up (%.1f s)" % (nm, time.perf_counter() - t0))
    setup_s = time.perf_counter() - t0
    if warm:
        sgw.step_batch(ss, warm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = sgw.step_batch(ss, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    log("timed %d batched steps: %.3f s" % (steps, elapsed))
    goldens = {i: load_golden(nm)[0] for i, nm in enumerate(names)}
    errors = []

    def compare(i, step, after):
        m, v = ss[i].moments()
        gm, gs = goldens[i][step]
        errors.append({"problem": names[i], "step": step, "after_timing": after,
                       "mean": rel_l2(m.cpu().numpy(), gm),
                       "std": rel_l2(np.sqrt(v.cpu().numpy()), gs)})

    done = warm + steps
    for i in goldens:
        d = done
        for step in [g for g in sorted(goldens[i]) if g >= done]:
            ss[i].step(step - d)
            d = step
            compare(i, step, True)
        earlier = [g for g in sorted(goldens[i]) if g < done]
        if earlier:
            ss[i].set_state()
            d = 0
            for step in earlier:
                ss[i].step(step - d)
                d = step
                compare(i, step, False)
    log("accuracy: %s" % errors)
    for s in ss:
        s.close()
    return {"problem_steps_per_s": len(names) * steps / elapsed,
            "ms_per_batched_step": 1e3 * elapsed / steps,
            "pcg_iters_per_step": [x["outer_iters"] / steps for x in st],
            "inner_iters_per_step": [x["inner_iters"] / steps for x in st],
            "setup_s": setup_s, "errors": errors}


SWEEPS = {
    # the paper's studies with its mesh sizes (13,472 / 37,267 vertices) on
    # structured meshes of about the same node counts, the Courant number 0.65
    # it uses, sigma 0.3, correlation length 0.25, input order 2
    "subdomains": [dict(n=120, L=7, p_out=3, ns=ns) for ns in (2, 3, 4, 5, 6, 8, 10, 12)],
    "rvs": [dict(n=192, L=L, p_out=3, ns=8) for L in range(3, 10)],
    "order": [dict(n=128, L=3, p_out=p, ns=8) for p in range(2, 10)],
}


def sweep(name, steps, warm, log):
    """One-GPU replica of one of the paper's scaling studies (Sec. 6.3, 6.4):
    outer (interface) and subdomain PCG iterations per step and time-steps/s
    of the plain FP64 method against the number of subdomains, the number of
    random variables or the chaos order."""
    import torch
    import paper_2512_23027_amd as sgw
    import workloads
    rows = []
    for c in SWEEPS[name]:
        n, ns = c["n"], c["ns"]
        prm = workloads.config("cfg5", n=n, L=c["L"], p_out=c["p_out"], sigma=0.3, bx=0.25,
                               by=0.25, dt=0.65 / n, xsplits=workloads.uniform_splits(n, ns),
                               ysplits=workloads.uniform_splits(n, ns), x0=0.5, y0=0.5,
                               width=0.1)
        t0 = time.perf_counter()
        s = sgw.Solver(prm, **solver_settings("fp64"))
        s.factor()
        s.autotune()
        setup = time.perf_counter() - t0
        s.set_state()
        s.step(warm)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st = s.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        row = {"mesh_nodes": (n + 1) ** 2, "subdomains": ns * ns, "L": c["L"],
               "order": c["p_out"], "P": s.P, "sg_unknowns": s.P * s.nfree,
               "coarse_unknowns": s.P * s.ncorner,
               "outer_iters_per_step": st["outer_iters"] / steps,
               "outer_iters_max": st["outer_iters_max"],
               "inner_iters_per_step": st["inner_iters"] / steps,
               "steps_per_s": steps / el, "setup_s": setup}
        s.close()
        log("sweep %s: %s" % (name, row))
        rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="cfg5")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 stack")
    ap.add_argument("--guess", choices=("newmark", "learned"), default="newmark",
                    help="initial guess of the full stack (learned: trained after the set-up "
                         "on trajectories of other pulse positions)")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--trace-window", metavar="KERNEL_TRACE_CSV", default=None,
                    help="per-step kernel times of the first timed region of a kernel trace")
    ap.add_argument("--write-traffic", nargs=5, metavar=("KERNEL_RE", "FETCH_CSV", "WRITE_CSV",
                                                         "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/<basis>_pcg_f_traffic.json from rocprofv3 counters")
    ap.add_argument("--sweep", choices=sorted(SWEEPS), default=None,
                    help="run one of the scaling studies instead (JSON rows)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.trace_window:
        trace_window(args.trace_window, args.steps)
        return
    if args.write_traffic:
        write_traffic(*args.write_traffic, workload=args.workload)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the domain decomposition would shard by blocks of subdomains)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2512_23027_amd as sgw
    import workloads

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.sweep:
        rows = sweep(args.sweep, args.steps, args.warmup, log)
        print(json.dumps({"sweep": args.sweep, "solver": "plain FP64 DD-PCG (two-level NN)",
                          "steps": args.steps, "warmup": args.warmup, "rows": rows}),
              flush=True)
        return
    if args.workload == "cfg3":
        names = ["cfg3-%d" % p for p in range(8)]
        res = run_batch(sgw, names, solver_settings("mixed"), args.warmup, args.steps, log)
        errs = res["errors"]
        ok = any(e["after_timing"] for e in errs) and all(max(e["mean"], e["std"]) <= 1e-6
                                                          for e in errs)
        print(json.dumps({
            "metric": METRIC, "value": res["problem_steps_per_s"],
            "unit": "problem time-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms_per_batched_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64-refinement", "data": "synthetic",
            "config": {"workload": WORKLOADS["cfg3"] + "; full stack as for cfg5",
                       "global_batch": len(names)},
            "pcg_iters_per_step": res["pcg_iters_per_step"],
            "inner_iters_per_step": res["inner_iters_per_step"], "setup_s": res["setup_s"],
            "rel_err_vs_oracle": errs, "accuracy_ok": ok}), flush=True)
        return
    prm = workloads.config(args.workload)
    golden, gmeta = load_golden(args.workload)
    log("workload %s, stored oracle steps %s" % (args.workload, sorted(golden)))
    full = run_stack(sgw, prm, solver_settings("mixed"), args.warmup, args.steps, golden, log,
                     learn=LEARN if args.guess == "learned" else None)
    plain = None
    if not args.no_fp64:
        plain = run_stack(sgw, prm, solver_settings("fp64"), args.warmup, args.steps, golden,
                          log)

    prof = full["prof"]
    kdom = max(prof, key=lambda k: prof[k][1])
    n_l, ms, nbytes = prof[kdom]
    avg_s = ms * 1e-3 / max(n_l, 1)
    bytes_per_launch = nbytes / max(n_l, 1)
    gbs = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
    roof = {"bound": "hbm", "kernel": KERNEL_NAMES[kdom], "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": None,
            "timed_launches": n_l, "avg_launch_us": 1e6 * avg_s,
            "algorithmic_bytes_per_launch": bytes_per_launch}
    if kdom in (0, 3):
        # the SG apply: bytes and flops per row; ALU-bound when the flops
        # take longer at the vector peak than the bytes at the HBM peak
        bpr, fpr, fused = sg_apply_counts(prm)
        w = 4 if kdom == 3 else 8
        bpr = bpr if w == 4 else bpr * 2 - 7 * 4
        rows = bytes_per_launch / bpr
        flops = rows * fpr
        roof["rows_per_launch"] = rows
        roof["fused_update_bytes_per_launch"] = rows * fused * (w // 4)
        tfs = flops / avg_s / 1e12 if avg_s > 0 else 0.0
        peak = FP32_VECTOR_PEAK_TFS if w == 4 else FP64_VECTOR_PEAK_TFS
        roof["flops_per_launch"] = flops
        roof["hbm_frac"] = roof["frac"]
        roof["alu_tflops"] = tfs
        if flops / (peak * 1e12) > bytes_per_launch / (HBM_PEAK_GBS * 1e9):
            roof.update({"bound": "alu", "achieved": tfs, "peak": peak, "unit": "TFLOP/s",
                         "frac": tfs / peak,
                         "note": "FP32 peak counts packed (two per lane) FMAs, which this "
                                 "build does not emit (one FMA per lane per clock: 78.6)"
                         if w == 4 else "FP64 vector peak"})
    tr = measured_traffic(prm, kdom)
    if tr:
        roof["traffic"] = tr["bytes_per_dispatch"]
        roof["traffic_source"] = tr["source"]
    # step-level effective GB/s: the device-counted bytes of the sampled
    # SG-apply and Chebyshev launches, scaled to all launches of the timed
    # steps (a lower bound of the step's traffic: vectors, dots and the
    # coarse grid are not counted)
    step_bytes = sum(v[2] for v in prof.values()) * PROFILE_EVERY / max(args.steps, 1)
    roof["step_counted_bytes"] = step_bytes
    roof["step_effective_GBs"] = step_bytes * full["steps_per_s"] / 1e9
    errs = full["errors"]
    out = {
        "metric": METRIC,
        "value": full["steps_per_s"],
        "unit": "time-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": full["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64-refinement",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + "; full stack: FP32 DD-PCG in FP64 "
                   "iterative refinement to SG residual 1e-8, batched Chebyshev-preconditioned "
                   "subdomain solves, autotuned tiles, " + (
                       "learned guess (trained after the set-up on %d trajectories of %d steps "
                       "with the pulse elsewhere)" % (len(LEARN["seeds"]), LEARN["nsteps"])
                       if args.guess == "learned" else "Newmark-extrapolated guess"),
                   "global_batch": 1},
        "learned_guess_training": full["learned_guess"],
        "guess_fallbacks": full["guess_fallbacks"],
        "pcg_iters_per_step": full["pcg_iters_per_step"],
        "inner_iters_per_step": full["inner_iters_per_step"],
        "ir_sweeps_per_step": full["ir_sweeps_per_step"],
        "setup_s": full["setup_s"],
        "roofline": roof,
        "kernels": {KERNEL_NAMES[k]: {"timed_launches": v[0], "ms": v[1],
                                      "avg_launch_us": 1e3 * v[1] / v[0],
                                      "GB/s": (v[2] / (v[1] * 1e-3)) / 1e9}
                    for k, v in prof.items() if v[0] > 0},
        "kernel_timing": "HIP events around every %dth launch of each kind in the timed steps "
                         "(the Chebyshev launches have theirs recorded with their dispatch); "
                         "bytes of the fused SG-apply and Chebyshev launches counted on the "
                         "device over the rows they process" % PROFILE_EVERY,
        "rel_err_vs_oracle": errs,
    }
    if plain is not None:
        out["plain_fp64_same_gpu"] = {
            "value": plain["steps_per_s"], "ms_per_step": plain["ms_per_step"],
            "pcg_iters_per_step": plain["pcg_iters_per_step"],
            "inner_iters_per_step": plain["inner_iters_per_step"], "setup_s": plain["setup_s"],
            "config": "FP64 DD-PCG (interface rtol 1e-9, Neumann solves 1e-4), previous-solution "
                      "guess, batched Chebyshev-preconditioned subdomain solves",
            "rel_err_vs_oracle": plain["errors"]}
        out["speedup_vs_plain_fp64"] = full["steps_per_s"] / plain["steps_per_s"]
    if not args.no_cpu_baseline:
        cb = cpu_baseline(prm, gmeta)
        if cb:
            out["cpu_baseline"] = cb
    ok = any(e["after_timing"] for e in errs) and all(max(e["mean"], e["std"]) <= 1e-6
                                                      for e in errs)
    if plain is not None and plain["errors"]:
        ok = ok and all(max(e["mean"], e["std"]) <= 1e-6 for e in plain["errors"])
    out["accuracy_ok"] = ok
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
