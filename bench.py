#!/usr/bin/env python3
"""Benchmark of the orthogonality-preserving eigensolver step on one MI355X.

Workload: 3D 7-point Dirichlet Laplacian on the 64^3 interior grid of the unit
cube plus 8 seeded Gaussian wells (seed 0), N = 128 lowest pairs, plain FP64,
fixed tau = 45 (0.9 of the stability limit 2 / (1/lambda_1 - 1/lambda_max)),
start block a seeded Gaussian orthonormalised by QR.  One benchmark step is one
full step of scheme (4.1) (Section 4.1, Steps 1-4) with every row of the hot
path: stencil, Grams, energy/residual reductions, warm-started CG for Step 1
(in the headline preconditioned by one multigrid V-cycle per iteration; the
plain CG step is measured beside it), the FP64 small solve and the in-place
update.  Inputs are resident in HBM before the timed region starts.

Prints one JSON line: outer steps per second (whole job, one GPU), the live
roofline of the dominant kernel (CG sweep B in both the preconditioned and the
plain CG step, timed with HIP events on the library's stream), per-kernel
timings (the V-cycle's fused post-smoothing with its counter traffic among
them), the mixed-precision and learned forms'
steps per second on the same workload, measured time-to-residual-1e-8 (plain
FP64; mixed precision to 1e-4 then FP64; learned steps judged by the plain
step) on problems that converge within the run (64^3 and 96^3 grids, N = 17,
which closes a level shell) with every form's Ritz values against the
committed reference eigenvalues, an extrapolated (labelled) time to residual
1e-8 at 64^3, N = 128 from measured step costs and the linearised rate,
Algorithm 1's energy stops with the fixed and the adaptive step, Table 1's
step counts on the finite-difference oscillator, the batched and the large
(96^3, N = 512) workloads, and the CPU oracle timed on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-residual-1e-8 and iter/s at 64³,N=128: plain FP64 vs mixed vs learned"
HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


GOLDEN_EIGS = os.path.join(ROOT, "tests", "golden", "reference_eigs.json")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def reference_eigenvalues(name, k):
    """The k lowest eigenvalues of a benchmark operator from the committed
    reference file (written by the oracle's library eigensolver)."""
    import numpy as np
    d = json.load(open(GOLDEN_EIGS))
    for c in d["cases"]:
        if c["name"] == name and c["k"] >= k:
            return np.array(c["eigenvalues"][:k])
    raise KeyError(name)


def ritz_error(ritz, ref):
    import numpy as np
    return float(np.max(np.abs(np.asarray(ritz) - ref) / np.abs(ref)))


def sweep_b_bytes(n, N):
    """Algorithmic HBM bytes of one CG sweep B, averaged over its two forms
    (one launch per CG iteration, alternating): even iterations read p, r and
    write r' (three n x N FP64 blocks); odd ones also read y and p_prev and
    write y (six blocks).  4.5 blocks plus the n-entry diagonal."""
    return 4.5 * n * N * 8 + 8 * n


def kernel_bytes(kind, n, N):
    blk = n * N * 8
    return {
        "stencil": 2 * blk + 8 * n,          # read X, write HX, diagonal
        "cg_sweep_a": 3 * blk + 8 * n,       # read r, p_old, write p, diagonal
        "cg_sweep_b": sweep_b_bytes(n, N),
        "cg_sweep_b_odd": 6 * blk + 8 * n,   # read p, r, y, p_prev, write r', y, diagonal
    }.get(kind)


PMC_SOURCES = {"cg_sweep_b": "k_stencil.hip", "mg_post": "k_mg.hip"}


def full_sweep_b(tags, ms, its, launches, n, N):
    """The CG sweep-B launches of a timed run that swept, from the per-launch
    CG iteration tags and times (ope_profile_end_launches) and every step's
    inner_iterations: a step's CG starts at tag 0, and its launches with a tag
    below the step's count ran a full sweep (even tag: 3 FP64 blocks + the
    diagonal, odd: 6 + the diagonal); the others, enqueued past the
    convergence of every column, returned at once or added only the pending y
    term.  Returns (full launches, their total ms, their algorithmic bytes,
    [even, odd] counts); zero launches when the tags do not cover the run."""
    steps = []
    for tg, t_ms in zip(tags, ms):
        if tg == 0 or not steps:
            steps.append([])
        steps[-1].append((tg, t_ms))
    full, full_ms, full_bytes, parity = 0, 0.0, 0.0, [0, 0]
    if len(steps) != len(its) or len(tags) != launches:
        return 0, 0.0, 0.0, [0, 0]
    blk = n * N * 8
    for st, k in zip(steps, its):
        for tg, t_ms in st:
            if 0 <= tg < k:
                full += 1
                full_ms += t_ms
                full_bytes += (6 if tg % 2 else 3) * blk + 8 * n
                parity[tg % 2] += 1
    return full, full_ms, full_bytes, parity


def traffic_from_pmc(n, N, kernel="cg_sweep_b", mix=None):
    """HBM bytes per working launch of a kernel from the committed rocprofv3
    counter summary (profiles/pmc_traffic_<kernel>.json; for CG sweep B also
    profiles/pmc_traffic.json), or None when its source changed since the
    counters were taken, or none were taken for this workload.  `mix` gives
    per-kernel launch counts for a record of several kernels (CG sweep B: even
    and odd form) to weight their per-dispatch bytes with; else their mean."""
    path = os.path.join(ROOT, "profiles", f"pmc_traffic_{kernel}.json")
    if not os.path.exists(path):
        path = PMC_FILE if kernel == "cg_sweep_b" else None
    if path is None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2511_06788_amd", "csrc", PMC_SOURCES[kernel])
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha or rec.get("n") != n or rec.get("N") != N:
        return None
    pk = rec.get("per_kernel", [])
    if mix is not None and len(pk) == len(mix) and sum(mix) > 0:
        kib = sum(w * (k["fetch_kib"] + k["write_kib"]) for w, k in zip(mix, pk)) / sum(mix)
        return kib * 1024.0 * rec["copy_scale"]
    return (rec["fetch_kib_per_dispatch"] + rec["write_kib_per_dispatch"]) * 1024.0 * rec["copy_scale"]


def cpu_baseline(problem, tau, steps):
    """The oracle, as it stands, on the same workload: `steps` outer steps with
    the same warm start and inner tolerance rule, composed from oracle functions."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        blas_threads = 1
    op = O.Operator(problem.grid.m, problem.grid.h, problem.V)
    U = problem.U0.copy()
    its = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        HU = O.apply_H(op, U)
        Lam = U.T @ HU
        res = np.linalg.norm(HU - U @ Lam) / np.linalg.norm(Lam)
        eta = max(1e-12, 0.1 * res)
        st = {}
        Y = O.cg_source(op, U, Y0=U @ np.linalg.inv(Lam), tol=eta, stats=st)
        its += st["iterations"]
        U = O.step_general(U, Y, tau)["U"]
    dt = time.perf_counter() - t0
    logical, physical = host_cores()
    return {
        "value": steps / dt, "unit": "iter/s", "cores": int(blas_threads), "kind": "oracle",
        "host_logical_cpus": logical, "host_physical_cores": physical,
        "sample": (f"{steps} outer step(s) of the same 64^3 N=128 workload from the same start block "
                   f"({its} inner CG iterations, {dt:.1f} s); numpy/scipy FP64: the BLAS products "
                   f"(Grams, row products) ran on {blas_threads} threads, the stencil and the CG vector "
                   f"updates are single-threaded numpy; the host has {logical} logical CPUs"
                   + (f" ({physical} physical cores)" if physical else "")),
    }


def host_cores():
    """Logical CPUs and, when lscpu reports them, physical cores of the host."""
    import subprocess
    logical = os.cpu_count()
    physical = None
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, timeout=10).stdout
        pairs = {tuple(l.split(",")) for l in out.splitlines() if l and not l.startswith("#")}
        physical = len(pairs) or None
    except Exception:  # pragma: no cover
        pass
    return logical, physical


def time_to_residual(ope, torch, m=64, tol=1e-8, switch=1e-4, switch_mg=1e-4):
    """Wall time of Algorithm 1 from the start block to residual `tol` on an m^3
    wells problem whose block width N = 17 closes a level shell (it converges
    in a few hundred steps): plain FP64; the mixed form until `switch`, then
    FP64 steps (both with the default sweep shapes, and again autotuned); and
    the learned form (shipped weights, plain-step judge and fallback)."""
    import numpy as np
    import workloads as W
    p = W.wells_3d(m=m, N=17, seed=0)
    tau = 45.0
    out = {"workload": f"wells3d_{m}^3_N17_seed0", "tau": tau, "res_tol": tol}
    with ope.Context(p.grid, p.V, p.N) as cd, ope.Context(p.grid, p.V, p.N, precision=ope.OPE_MIXED) as cm:
        # warm the code paths
        ope.ope_solve(cd.handle, torch.from_numpy(p.U0).to("cuda"), tau, tol, 3)
        ope.ope_solve(cm.handle, torch.from_numpy(p.U0.astype(np.float32)).to("cuda"), tau, tol, 3)
        U = torch.from_numpy(p.U0).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        si = ope.ope_solve(cd.handle, U, tau, tol, 20000)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        ritz_plain = ope.ope_residual(cd.handle, U, p.N)[1]
        U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
        U64 = torch.empty_like(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sm = ope.ope_solve(cm.handle, U32, tau, switch, 20000)
        ope.ope_convert(cm.handle, U32, U64, p.grid.n * p.N, True)
        sf = ope.ope_solve(cd.handle, U64, tau, tol, 20000)
        torch.cuda.synchronize()
        t_mixed = time.perf_counter() - t0
        ritz_mixed = ope.ope_residual(cd.handle, U64, p.N)[1]
        # the mixed phase on its own: to its FP32 floor, eigenvalues and drift
        # of the FP32 iterate against the FP64 reference
        U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
        sm_floor = ope.ope_solve(cm.handle, U32, tau, 1e-8, 20000)
        res_floor, ritz_floor, drift_floor = ope.ope_residual(cm.handle, U32, p.N)
    ref = reference_eigenvalues(f"wells3d_{m}^3_seed0", p.N)
    out["reference_eigenvalues"] = "tests/golden/reference_eigs.json (oracle LOBPCG)"
    out["plain_fp64"] = {"converged": bool(si.converged), "steps": int(si.steps), "seconds": t_plain,
                         "final_residual": si.residual, "final_drift": si.drift,
                         "ritz_max_rel_error_vs_reference": ritz_error(ritz_plain, ref)}
    out["mixed_then_fp64"] = {"converged": bool(sf.converged), "mixed_steps": int(sm.steps),
                              "fp64_steps": int(sf.steps), "switch_residual": switch, "seconds": t_mixed,
                              "final_residual": sf.residual, "final_drift": sf.drift,
                              "ritz_max_rel_error_vs_reference": ritz_error(ritz_mixed, ref)}
    out["mixed_alone_to_fp32_floor"] = {"steps": int(sm_floor.steps), "stalled": bool(sm_floor.stalled),
                                        "residual": res_floor, "drift": drift_floor,
                                        "ritz_max_rel_error_vs_reference": ritz_error(ritz_floor, ref)}
    out["speedup_mixed"] = t_plain / t_mixed
    # plain and mixed-then-FP64 again with the sweep shapes autotuned for this
    # problem (the tuning itself is outside the timed regions, reported beside)
    with ope.Context(p.grid, p.V, p.N) as ct, ope.Context(p.grid, p.V, p.N, precision=ope.OPE_MIXED) as cmt:
        t0 = time.perf_counter()
        ope.ope_autotune(ct.handle)
        t_tune = time.perf_counter() - t0
        t0 = time.perf_counter()
        ope.ope_autotune(cmt.handle)
        t_tune_m = time.perf_counter() - t0
        ope.ope_solve(ct.handle, torch.from_numpy(p.U0).to("cuda"), tau, tol, 3)
        ope.ope_solve(cmt.handle, torch.from_numpy(p.U0.astype(np.float32)).to("cuda"), tau, tol, 3)
        U = torch.from_numpy(p.U0).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ope.ope_solve(ct.handle, U, tau, tol, 20000)
        torch.cuda.synchronize()
        t_tuned = time.perf_counter() - t0
        shape = list(ope.ope_get_sweep_shape(ct.handle))
        U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
        U64 = torch.empty_like(U)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        smt = ope.ope_solve(cmt.handle, U32, tau, switch, 20000)
        ope.ope_convert(cmt.handle, U32, U64, p.grid.n * p.N, True)
        sft = ope.ope_solve(ct.handle, U64, tau, tol, 20000)
        torch.cuda.synchronize()
        t_mixed_tuned = time.perf_counter() - t0
        shape_m = list(ope.ope_get_sweep_shape(cmt.handle))
    out["plain_fp64_autotuned"] = {"converged": bool(st.converged), "steps": int(st.steps), "seconds": t_tuned,
                                   "autotune_seconds": t_tune, "sweep_shape": shape,
                                   "final_residual": st.residual, "final_drift": st.drift}
    out["mixed_then_fp64_autotuned"] = {"converged": bool(sft.converged), "mixed_steps": int(smt.steps),
                                        "fp64_steps": int(sft.steps), "seconds": t_mixed_tuned,
                                        "autotune_seconds": t_tune_m, "sweep_shape": shape_m,
                                        "final_residual": sft.residual, "final_drift": sft.drift}
    with ope.Context(p.grid, p.V, p.N) as cl:
        net = ope.Net(cl, p.N, ope.load_net_weights())
        ope.ope_set_preconditioner(cl.handle, net.handle, judge=True)
        ope.ope_solve(cl.handle, torch.from_numpy(p.U0).to("cuda"), tau, tol, 3)
        U = torch.from_numpy(p.U0).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sl = ope.ope_solve(cl.handle, U, tau, tol, 20000)
        torch.cuda.synchronize()
        t_learned = time.perf_counter() - t0
        ope.ope_set_preconditioner(cl.handle, None)
        ritz_learned = ope.ope_residual(cl.handle, U, p.N)[1]
        net.close()
    out["learned_judged"] = {"converged": bool(sl.converged), "steps": int(sl.steps),
                             "learned_steps_kept": int(sl.learned_steps), "seconds": t_learned,
                             "final_residual": sl.residual, "final_drift": sl.drift,
                             "ritz_max_rel_error_vs_reference": ritz_error(ritz_learned, ref)}
    out["speedup_learned"] = t_plain / t_learned
    # the plain FP64 form with the multigrid-preconditioned Step 1
    with ope.Context(p.grid, p.V, p.N) as cg:
        ope.ope_set_multigrid(cg.handle, True)
        ope.ope_solve(cg.handle, torch.from_numpy(p.U0).to("cuda"), tau, tol, 3)
        U = torch.from_numpy(p.U0).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sg = ope.ope_solve(cg.handle, U, tau, tol, 20000)
        torch.cuda.synchronize()
        t_mg = time.perf_counter() - t0
        ritz_mg = ope.ope_residual(cg.handle, U, p.N)[1]
        # the mixed form with its own preconditioned Step 1, then FP64 (also preconditioned)
        with ope.Context(p.grid, p.V, p.N, precision=ope.OPE_MIXED) as cmg:
            ope.ope_set_multigrid(cmg.handle, True)
            ope.ope_solve(cmg.handle, torch.from_numpy(p.U0.astype(np.float32)).to("cuda"), tau, tol, 3)
            U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
            U64 = torch.empty_like(U)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            smg = ope.ope_solve(cmg.handle, U32, tau, switch_mg, 20000)
            ope.ope_convert(cmg.handle, U32, U64, p.grid.n * p.N, True)
            sfg = ope.ope_solve(cg.handle, U64, tau, tol, 20000)
            torch.cuda.synchronize()
            t_mixed_mg = time.perf_counter() - t0
            ritz_mixed_mg = ope.ope_residual(cg.handle, U64, p.N)[1]
    out["mixed_then_fp64_multigrid"] = {"converged": bool(sfg.converged), "mixed_steps": int(smg.steps),
                                        "fp64_steps": int(sfg.steps), "switch_residual": switch_mg,
                                        "seconds": t_mixed_mg, "final_residual": sfg.residual,
                                        "final_drift": sfg.drift,
                                        "ritz_max_rel_error_vs_reference": ritz_error(ritz_mixed_mg, ref)}
    out["speedup_mixed_multigrid"] = t_plain / t_mixed_mg
    out["speedup_mixed_multigrid_vs_plain_multigrid"] = t_mg / t_mixed_mg
    out["plain_fp64_multigrid"] = {"converged": bool(sg.converged), "steps": int(sg.steps), "seconds": t_mg,
                                   "inner_iterations": int(sg.inner_iterations),
                                   "final_residual": sg.residual, "final_drift": sg.drift,
                                   "ritz_max_rel_error_vs_reference": ritz_error(ritz_mg, ref)}
    out["speedup_multigrid"] = t_plain / t_mg
    return out


def mixed_floor_reached(hist, chunk, gain=0.99):
    """True when the last `chunk` steps lowered the residual by less than the
    factor `gain` (1% by default): `hist` holds (steps so far, residual) after
    each solve call, the starting block's first."""
    steps, res = hist[-1]
    back = [r for s, r in hist if s <= steps - chunk]
    return bool(back) and res > gain * back[-1]


def long_run_time_to_residual(ope, torch, minutes=16.0, tol=1e-8, chunk=1500, multigrid=True, mixed=False,
                              switch=1e-4, recycle=False, mixed_steps=0):
    """Algorithm 1 at 64^3, N = 128, tau = 45 (plain FP64, multigrid-
    preconditioned Step 1) MEASURED from the start block for up to `minutes`
    of wall time, in chunks of `chunk` steps (a progress line per chunk on
    stderr).  If the residual has not reached `tol` by then, the remainder is
    EXTRAPOLATED from the measured rate: the slope of ln(residual) over the
    last quarter of the measured steps (at least the last two chunks) and
    their measured cost per step.  With `mixed`, the mixed-precision form
    (FP32 V-cycle) runs first, to residual `switch` (or its FP32 floor), and
    the FP64 step takes over from the converted block; with `mixed_steps` > 0
    the mixed form runs exactly that many steps instead.  With `recycle`, the
    FP64 step's inner CG starts from the previous step's correction
    (ope_set_recycle)."""
    import numpy as np
    import workloads as W
    p = W.wells_3d(m=64, N=128, seed=0)
    tau = 45.0
    traj = []
    mixed_done = 0
    with ope.Context(p.grid, p.V, p.N) as ctx:
        ope.ope_set_multigrid(ctx.handle, multigrid)
        ope.ope_set_recycle(ctx.handle, recycle)
        U = torch.from_numpy(p.U0).to("cuda")
        steps = 0
        converged = False
        if mixed:
            with ope.Context(p.grid, p.V, p.N, precision=ope.OPE_MIXED) as cm:
                ope.ope_set_multigrid(cm.handle, multigrid)
                U32 = torch.from_numpy(p.U0.astype(np.float32)).to("cuda")
                hist = [(0, float(ope.ope_residual(cm.handle, U32, p.N, want_ritz=False)[0]))]
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                # The library's stall rule (no 10% gain within 60 steps) fires in the slow
                # phase long before the FP32 floor, where a 10% gain takes hundreds of
                # steps; here the mixed phase goes on while `chunk` steps still lower the
                # residual by 1%.
                while time.perf_counter() - t0 < 60.0 * minutes:
                    n = min(chunk, mixed_steps - steps) if mixed_steps > 0 else chunk
                    sm = ope.ope_solve(cm.handle, U32, tau, switch, n)
                    torch.cuda.synchronize()
                    steps += int(sm.steps)
                    hist.append((steps, float(sm.residual)))
                    if not traj or steps >= traj[-1][1] + chunk or sm.converged:
                        traj.append((time.perf_counter() - t0, steps, float(sm.residual)))
                        print(f"long run (mixed): {traj[-1][0]:.1f} s, {steps} steps, residual {sm.residual:.3e}",
                              file=sys.stderr, flush=True)
                    if sm.converged or int(sm.steps) == 0:
                        break
                    if mixed_steps > 0:
                        if steps >= mixed_steps:
                            break
                    elif mixed_floor_reached(hist, chunk):
                        break
                torch.cuda.synchronize()
                traj.append((time.perf_counter() - t0, steps, float(hist[-1][1])))
                mixed_done = steps
                ope.ope_convert(cm.handle, U32, U, p.grid.n * p.N, True)
        else:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        while time.perf_counter() - t0 < 60.0 * minutes:
            si = ope.ope_solve(ctx.handle, U, tau, tol, chunk)
            torch.cuda.synchronize()
            steps += int(si.steps)
            traj.append((time.perf_counter() - t0, steps, float(si.residual)))
            print(f"long run: {traj[-1][0]:.1f} s, {steps} steps, residual {si.residual:.3e}", file=sys.stderr,
                  flush=True)
            if si.converged:
                converged = True
                break
        res, ritz, drift = ope.ope_residual(ctx.handle, U, p.N)
    out = {"workload": "wells3d_64^3_N128_seed0", "tau": tau, "res_tol": tol,
           "form": ("mixed for %d steps, then plain FP64" % mixed_steps if mixed_steps > 0 else
                    "mixed to %g or its floor, then plain FP64" % switch) if mixed else "plain FP64",
           "mixed_steps": mixed_done,
           "inner": ("multigrid-preconditioned CG" if multigrid else "CG") +
                    (", recycled warm start" if recycle else ""), "measured_seconds": traj[-1][0],
           "measured_steps": steps, "residual_reached": res, "drift": drift, "converged": converged,
           "trajectory": [{"seconds": a, "steps": b, "residual": c} for a, b, c in traj]}
    if converged:
        out["seconds"] = traj[-1][0]
        out["label"] = "MEASURED"
        lam = reference_eigenvalues("wells3d_64^3_seed0", p.N)
        out["ritz_max_rel_error_vs_reference"] = ritz_error(ritz, lam)
        return out
    q = [t for t in traj if t[1] >= 0.75 * steps]
    if len(q) < 2:
        q = traj[-2:]
    if len(q) >= 2 and q[-1][2] < q[0][2]:
        slope = (np.log(q[-1][2]) - np.log(q[0][2])) / (q[-1][1] - q[0][1])
        sec_per_step = (q[-1][0] - q[0][0]) / (q[-1][1] - q[0][1])
        more = float(np.log(tol / res) / slope)
        out.update({"label": "MEASURED for the first part, the remainder EXTRAPOLATED from the measured rate",
                    "measured_residual_factor_per_step": float(np.exp(slope)), "ms_per_step_late": 1e3 * sec_per_step,
                    "remaining_steps": more, "seconds": traj[-1][0] + more * sec_per_step})
        out["hours"] = out["seconds"] / 3600.0
    return out


def extrapolated_time_to_residual(ope, torch, p, tau, tol=1e-8, run=200, late=20, multigrid=True):
    """EXTRAPOLATION (not a measurement) of Algorithm 1's time to residual `tol`
    at 64^3, N = 128: `run` steps from the start block are timed, then `late`
    more give the per-step cost of the slow phase; the remaining steps follow
    from the slow factor of the fixed-point linearisation,
    rho = 1 - tau (1/lambda_N - 1/lambda_{N+1}), with lambda_N, lambda_{N+1} from
    the committed reference eigenvalues: steps = ln(res / tol) / (-ln rho)."""
    import numpy as np
    lam = reference_eigenvalues(f"wells3d_{p.grid.m[0]}^3_seed0", p.N + 1)
    rho = 1.0 - tau * (1.0 / lam[p.N - 1] - 1.0 / lam[p.N])
    with ope.Context(p.grid, p.V, p.N) as ctx:
        if multigrid:
            ope.ope_set_multigrid(ctx.handle, True)
        U = torch.from_numpy(p.U0).to("cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(run):
            ope.ope_step(ctx.handle, U, tau)
        torch.cuda.synchronize()
        t_run = time.perf_counter() - t0
        res_a = ope.ope_residual(ctx.handle, U, p.N, want_ritz=False)[0]
        its = 0
        t0 = time.perf_counter()
        for _ in range(late):
            its += ope.ope_step(ctx.handle, U, tau).inner_iterations
        torch.cuda.synchronize()
        t_late = time.perf_counter() - t0
        res_b = ope.ope_residual(ctx.handle, U, p.N, want_ritz=False)[0]
    ms_late = 1e3 * t_late / late
    more = float(np.log(res_b / tol) / -np.log(rho)) if res_b > tol else 0.0
    seconds = t_run + t_late + more * ms_late * 1e-3
    return {"label": "EXTRAPOLATED from measured step costs and the linearised rate, not measured",
            "workload": f"wells3d_{p.grid.m[0]}^3_N{p.N}_seed0", "tau": tau, "res_tol": tol,
            "inner": "multigrid-preconditioned CG" if multigrid else "CG",
            "lambda_N": float(lam[p.N - 1]), "lambda_N_plus_1": float(lam[p.N]), "rho": rho,
            "measured_steps": run + late, "measured_seconds": t_run + t_late,
            "residual_after_measured_steps": res_b,
            "measured_residual_factor_per_step_late": float((res_b / res_a) ** (1.0 / late)),
            "ms_per_step_late": ms_late, "cg_iterations_per_step_late": its / late,
            "remaining_steps_model": more, "seconds": seconds, "hours": seconds / 3600.0}


def algorithm1_energy_stops(ope, torch, m=64, N=17, tol=1e-10):
    """Algorithm 1's energy stops on the m^3, N = 17 wells problem: the
    relative energy error against the reference ground-state energy
    (Section 5's stop) at the fixed tau = 45 and with the adaptive step
    (start at the stability limit estimated from ope_spectrum_bounds, tau in
    [1, 2 x limit]); and Algorithm 1's own err_E stop at tau = 45."""
    import numpy as np
    import workloads as W
    p = W.wells_3d(m=m, N=N, seed=0)
    lam = reference_eigenvalues(f"wells3d_{m}^3_seed0", N)
    Egs = 0.5 * float(np.sum(lam))
    out = {"workload": f"wells3d_{m}^3_N{N}_seed0", "energy_ref": Egs, "energy_tol": tol}
    with ope.Context(p.grid, p.V, p.N) as c:
        lmin, lmax = ope.ope_spectrum_bounds(c.handle)
        tlim = 2.0 / (1.0 / lmin - 1.0 / lmax)
        out["lanczos_lambda_min"], out["lanczos_lambda_max"], out["tau_limit_estimate"] = lmin, lmax, tlim
        ope.ope_solve(c.handle, torch.from_numpy(p.U0).to("cuda"), 45.0, 1e-8, 3)
        for name, kw in (("fixed_tau45", dict(tau=45.0)),
                         ("adaptive", dict(tau=tlim, tau_min=1.0, tau_max=2.0 * tlim, grow=1.25)),
                         ("algorithm1_errE_1e-12_tau45", dict(tau=45.0))):
            U = torch.from_numpy(p.U0).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name.startswith("algorithm1"):
                si = ope.ope_solve_ex(c.handle, U, energy_tol=1e-12, max_steps=20000, **kw)
            else:
                si = ope.ope_solve_ex(c.handle, U, energy_tol=tol, energy_ref=Egs, max_steps=20000, **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ritz = ope.ope_residual(c.handle, U, N)[1]
            out[name] = {"seconds": dt, "steps": int(si.steps), "rejected": int(si.rejected),
                         "converged": bool(si.converged), "final_tau": si.tau,
                         "rel_energy_error": (si.energy - Egs) / abs(Egs), "residual": si.residual,
                         "ritz_max_rel_error_vs_reference": ritz_error(ritz, lam)}
    return out


def paper_hydrogen(ope, torch):
    """Section 5.2's hydrogen atom in its finite-difference form (48^3 on
    (-10, 10)^3, -1/2 Lap - 1/sqrt(|x|^2 + 0.1^2), shifted by 1, N = 5):
    Algorithm 1 at 0.9 of the step limit from the Lanczos estimates to
    residual 1e-8, plain and multigrid-preconditioned Step 1; Ritz values
    against the oracle eigensolver's, and (context) the unshifted energies
    against the exact hydrogen ones, -1/2 and -1/8 (the grid's error)."""
    import numpy as np
    import workloads as W
    ref_case = [c for c in json.load(open(GOLDEN_EIGS))["cases"] if c["name"] == "hydrogen_soft_48"][0]
    ref = np.array(ref_case["eigenvalues"][:5])
    p = W.hydrogen_softened(m=48, N=5, half=10.0, shift=1.0)
    exact = np.array([-0.5, -0.125, -0.125, -0.125, -0.125])
    out = {"workload": "hydrogen_soft_48^3_N5 (finite-difference stand-in for the P2-FEM hydrogen of Section 5.2)",
           "shift": 1.0, "res_tol": 1e-8}
    for mg in (False, True):
        with ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic, shift=p.shift) as c:
            ope.ope_set_multigrid(c.handle, mg)
            lo, hi = ope.ope_spectrum_bounds(c.handle)
            tau = 0.9 * 2.0 / (1.0 / lo - 1.0 / hi)
            ope.ope_solve(c.handle, torch.from_numpy(p.U0).to("cuda"), tau, 1e-8, 3)
            U = torch.from_numpy(p.U0).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            si = ope.ope_solve(c.handle, U, tau, 1e-8, 4000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res, ritz, drift = ope.ope_residual(c.handle, U, p.N)
        ritz = np.sort(ritz)
        out["multigrid" if mg else "plain"] = {
            "tau": tau, "converged": bool(si.converged), "steps": int(si.steps), "seconds": dt,
            "inner_iterations": int(si.inner_iterations), "final_residual": res, "drift": drift,
            "ritz_max_rel_error_vs_reference": float(np.max(np.abs(ritz - ref) / ref)),
            "energies": (ritz - 1.0).tolist(),
            "grid_error_vs_exact_hydrogen": (ritz - 1.0 - exact).tolist()}
    return out


def paper_table1(ope, torch, taus=(0.5, 1.0, 1.5)):
    """Section 5.1's Table 1 on the finite-difference oscillator (99 x 99,
    N = 15): steps and wall time to relative energy error 1e-10, Step 1
    solved to 1e-13 (the paper's Step 1 is exact)."""
    import numpy as np
    import workloads as W
    p = W.oscillator_2d_paper(m=99)
    lam = reference_eigenvalues("oscillator2d_99", 15)
    Egs = 0.5 * float(np.sum(lam))
    printed = {0.5: 681, 1.0: 301, 1.5: 209}
    out = {"workload": "oscillator2d_99x99_N15 (finite-difference stand-in for the P2-FEM mesh)", "energy_ref": Egs}
    with ope.Context(p.grid, p.V, p.N, kinetic=p.kinetic) as c:
        # the paper solves Step 1 exactly; here CG to 1e-13
        ope.ope_set_inner(c.handle, 0.0, 1e-13, 20000)
        for tau in taus:
            U = torch.from_numpy(p.U0).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            si = ope.ope_solve_ex(c.handle, U, tau, energy_tol=1e-10, energy_ref=Egs, max_steps=5000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            ritz = ope.ope_residual(c.handle, U, 15)[1]
            err = np.abs(ritz - lam) / lam
            out[f"tau_{tau}"] = {"steps": int(si.steps), "printed_steps": printed.get(tau), "seconds": dt,
                                 "err_first_ten_max": float(err[:10].max()), "err_last_five_max": float(err[10:].max())}
    return out


def mg_steps_per_second(ope, torch, p, tau, steps, warmup):
    """Steps per second with the multigrid-preconditioned Step 1
    (ope_set_multigrid) from the seeded start over the given window, with the
    V-cycle's share (HIP events around its launches) and the inner iterations."""
    U = torch.from_numpy(p.U0).to("cuda")
    with ope.Context(p.grid, p.V, p.N) as c:
        ope.ope_set_multigrid(c.handle, True)
        levels, coarsest = ope.ope_mg_info(c.handle)
        for _ in range(warmup):
            ope.ope_step(c.handle, U, tau)
        torch.cuda.synchronize()
        inner = 0
        last = None
        t0 = time.perf_counter()
        for _ in range(steps):
            last = ope.ope_step(c.handle, U, tau)
            inner += last.inner_iterations
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        parts = {}
        for name, kid in (("vcycle", ope.OPE_KERNEL_MG), ("cg_sweep_a", ope.OPE_KERNEL_CG_SWEEP_A),
                          ("cg_sweep_b", ope.OPE_KERNEL_CG_SWEEP_B), ("cg_sweep_b_odd", ope.OPE_KERNEL_CG_SWEEP_B_Y),
                          ("cg_reduce", ope.OPE_KERNEL_CG_REDUCE)):
            ope.ope_profile_begin(c.handle, kid)
            its = 0
            for _ in range(3):
                its += ope.ope_step(c.handle, U, tau).inner_iterations
            nl, tms = ope.ope_profile_end(c.handle)
            parts[name] = {"ms_per_step": tms / 3.0, "launches_per_step": nl / 3.0}
    return {"iter_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps, "inner_iterations_per_step": inner / steps,
            "levels": levels, "coarsest_nodes": coarsest, "residual_at_end": last.residual,
            "drift_at_end": last.drift, "parts": parts}


def learned_steps_per_second(ope, torch, p, tau, steps, warmup):
    """The learned form on the benchmark workload: Algorithm 1 with the shipped
    network, each learned step judged by the plain step (replaced when
    rejected, with back-off after rejections), for a fixed number of steps."""
    U = torch.from_numpy(p.U0).to("cuda")
    with ope.Context(p.grid, p.V, p.N) as ctx:
        net = ope.Net(ctx, p.N, ope.load_net_weights())
        ope.ope_set_preconditioner(ctx.handle, net.handle, judge=True)
        ope.ope_solve(ctx.handle, U, tau, 0.0, warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        si = ope.ope_solve(ctx.handle, U, tau, 0.0, steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        net.close()
    return {"iter_per_s": si.steps / dt, "ms_per_step": 1e3 * dt / max(si.steps, 1),
            "learned_steps_kept": int(si.learned_steps), "steps": int(si.steps), "warmup": warmup,
            "residual_at_end": si.residual}


def sweep_b_rate(ope, torch, ctx, U, tau, n, N, esz, steps=10):
    """Sweep B's rate over `steps` further steps, timed per counted CG
    iteration with the library's HIP events (as for the headline line), for
    blocks of `esz`-byte elements."""
    ope.ope_profile_begin(ctx.handle, ope.OPE_KERNEL_CG_SWEEP_B)
    inner = 0
    for _ in range(steps):
        inner += ope.ope_step(ctx.handle, U, tau).inner_iterations
    torch.cuda.synchronize()
    launches, total_ms = ope.ope_profile_end(ctx.handle)
    avg_ms = total_ms / max(inner, 1)
    algo = 4.5 * n * N * esz + esz * n
    achieved = algo / (avg_ms * 1e-3) / 1e9
    return {"algorithmic_bytes": algo, "avg_ms_per_iteration": avg_ms, "achieved_GB_per_s": achieved,
            "frac": achieved / HBM_PEAK_GBS, "counted_iterations": inner, "launches": launches, "steps": steps}


def steps_per_second(ope, torch, p, tau, precision, steps, warmup, multigrid=False):
    import numpy as np
    mixed = precision == ope.OPE_MIXED
    U = torch.from_numpy(p.U0.astype(np.float32 if mixed else np.float64)).to("cuda")
    with ope.Context(p.grid, p.V, p.N, precision=precision) as ctx:
        if multigrid:
            ope.ope_set_multigrid(ctx.handle, True)
        for _ in range(warmup):
            ope.ope_step(ctx.handle, U, tau)
        torch.cuda.synchronize()
        inner = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            inner += ope.ope_step(ctx.handle, U, tau).inner_iterations
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # after the timed steps, so that their events do not touch the rate above
        sweep = sweep_b_rate(ope, torch, ctx, U, tau, p.grid.n, p.N, 4 if mixed else 8)
    return {"iter_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps, "inner_iterations_per_step": inner / steps,
            "steps": steps, "warmup": warmup, "cg_sweep_b": sweep}


def batched_throughput(ope, torch, steps=5, tau=30.0, count=64):
    """The batched workload (64 well problems, grid edges 24..48, N 16..128):
    problem-steps per second of ope_batch_step (per-problem CG launches on the
    problems' streams, the default; shared CG launches; each before and after
    the autotuner), of replays of the captured step (ope_batch_capture, both
    launch modes, checked bit for bit against the eager steps), and of the same
    problems stepped one after the other with ope_step."""
    import numpy as np
    import workloads as W
    probs = W.batched_problems(count)
    out = {"workload": f"{count} wells3d problems, m 24..48, N 16..128, seed 0", "tau": tau, "steps": steps,
           "grid_points_x_columns": int(sum(p.grid.n * p.N for p in probs))}
    with ope.Batch(probs) as b:
        U0 = [torch.from_numpy(p.U0).to("cuda") for p in probs]
        U = [u.clone() for u in U0]

        def reset():
            for u, u0 in zip(U, U0):
                u.copy_(u0)
            torch.cuda.synchronize()

        def timed(fn):
            reset()
            fn()
            reset()
            t0 = time.perf_counter()
            inner = fn()
            torch.cuda.synchronize()
            return time.perf_counter() - t0, inner

        # algorithmic bytes of the CG sweeps: 7.5 n x N block passes per iteration
        blk = [7.5 * p.grid.n * p.N * 8 for p in probs]

        most = [0]

        def batch_steps():
            inner, nbytes = 0, 0
            for _ in range(steps):
                for k, i in enumerate(b.step(U, tau)):
                    inner += i.inner_iterations
                    nbytes += i.inner_iterations * blk[k]
                    most[0] = max(most[0], i.inner_iterations)
            return inner, nbytes

        def graph_steps():
            inner, nbytes = 0, 0
            for _ in range(steps):
                for k, i in enumerate(b.replay()):
                    inner += i.inner_iterations
                    nbytes += i.inner_iterations * blk[k]
            return inner, nbytes

        def sequential_steps():
            inner, nbytes = 0, 0
            for _ in range(steps):
                for k in range(count):
                    it = ope.ope_step(b.context(k), U[k], tau).inner_iterations
                    inner += it
                    nbytes += it * blk[k]
            return inner, nbytes

        t_seq, in_seq = timed(sequential_steps)
        b.set_shared(False)
        t_b0, in_b0 = timed(batch_steps)
        b.set_shared(True)
        t_s0, in_s0 = timed(batch_steps)
        t_tune0 = time.perf_counter()
        buckets = b.autotune()
        t_tune = time.perf_counter() - t_tune0
        t_s1, in_s1 = timed(batch_steps)
        b.set_shared(False)
        t_b1, in_b1 = timed(batch_steps)
        ref = [u.clone() for u in U]
        # whole steps as graph replays, with the CG iteration count the
        # largest any problem needed in the eager steps (multiple of 4)
        K = max(4, -(-most[0] // 4) * 4)
        b.capture(U, tau, K)
        t_g0, in_g0 = timed(graph_steps)
        same0 = all(torch.equal(a, r) for a, r in zip(U, ref))
        b.set_shared(True)
        b.capture(U, tau, K)
        t_g1, in_g1 = timed(graph_steps)
        same1 = all(torch.equal(a, r) for a, r in zip(U, ref))
        # every problem with the multigrid-preconditioned Step 1 (own launches)
        b.set_shared(False)
        for i in range(count):
            ope.ope_set_multigrid(b.context(i), True)
        most[0] = 0
        t_m, in_m = timed(batch_steps)
        Km = max(4, -(-most[0] // 4) * 4)
        ref_m = [u.clone() for u in U]
        b.capture(U, tau, Km)
        t_gm, in_gm = timed(graph_steps)
        same_m = all(torch.equal(a, r) for a, r in zip(U, ref_m))
    ps = count * steps

    def rec(t, r):
        return {"problem_steps_per_s": ps / t, "seconds": t, "inner_iterations": r[0],
                "cg_sweep_GB_per_s": r[1] / t / 1e9}
    out["sequential"] = rec(t_seq, in_seq)
    out["batched"] = rec(t_b0, in_b0)
    out["batched_shared_launches"] = rec(t_s0, in_s0)
    out["batched_shared_launches_autotuned"] = dict(rec(t_s1, in_s1), buckets=buckets, autotune_seconds=t_tune)
    out["batched_autotuned"] = rec(t_b1, in_b1)
    out["graph_replay_autotuned"] = dict(rec(t_g0, in_g0), cg_iterations=K, equal_to_eager=same0)
    out["graph_replay_shared_launches_autotuned"] = dict(rec(t_g1, in_g1), cg_iterations=K, equal_to_eager=same1)
    out["batched_multigrid_autotuned"] = rec(t_m, in_m)
    out["graph_replay_multigrid_autotuned"] = dict(rec(t_gm, in_gm), cg_iterations=Km, equal_to_eager=same_m)
    out["speedup_multigrid_vs_batched"] = min(t_b0, t_b1) / min(t_m, t_gm)
    out["speedup_vs_sequential"] = t_seq / min(t_b0, t_b1)
    return out


def small_batch_graph(ope, torch, count=16, m=24, N=16, tau=30.0, steps=20):
    """A batch of small problems (sixteen 24^3 wells, N = 16), where launch
    latency and host checks dominate: problem-steps per second of eager
    batched steps with per-problem and with shared CG launches, and of replays
    of the captured step (ope_batch_capture) whose fixed CG iteration count is
    the largest count the eager shared steps needed, rounded up to a multiple
    of 4; the replayed blocks are checked against the eager ones bit for bit."""
    import workloads as W
    probs = [W.wells_3d(m=m, N=N, seed=100 + k) for k in range(count)]
    out = {"workload": f"{count} wells3d problems, {m}^3, N = {N}, seeds 100..{99 + count}", "tau": tau,
           "steps": steps}
    with ope.Batch(probs) as b:
        U0 = [torch.from_numpy(p.U0).to("cuda") for p in probs]
        U = [u.clone() for u in U0]

        def reset():
            for u, u0 in zip(U, U0):
                u.copy_(u0)
            torch.cuda.synchronize()

        def eager(shared):
            b.set_shared(shared)
            reset()
            b.step(U, tau)
            reset()
            t0 = time.perf_counter()
            most = 0
            for _ in range(steps):
                most = max(most, max(i.inner_iterations for i in b.step(U, tau)))
            torch.cuda.synchronize()
            return time.perf_counter() - t0, most

        t_own, _ = eager(False)
        t_sh, most = eager(True)
        ref = [u.clone() for u in U]
        K = max(4, -(-most // 4) * 4)
        reset()
        b.capture(U, tau, K)
        b.replay()
        reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.replay(wait=False)
        torch.cuda.synchronize()
        t_g = time.perf_counter() - t0
        same = all(torch.equal(a, r) for a, r in zip(U, ref))
    ps = count * steps
    out["batched"] = {"problem_steps_per_s": ps / t_own, "seconds": t_own}
    out["batched_shared_launches"] = {"problem_steps_per_s": ps / t_sh, "seconds": t_sh}
    out["graph_replay"] = {"problem_steps_per_s": ps / t_g, "seconds": t_g, "cg_iterations": K,
                           "equal_to_shared_steps": same}
    out["graph_speedup_vs_shared"] = t_sh / t_g
    return out


def large_mixed(ope, torch, steps=5, warmup=2, tau=45.0):
    """The large mixed-precision workload: 96^3 grid, N = 512, 8 wells (seed 0):
    steps per second of the mixed form and of plain FP64 from the same start
    block, with the orthogonality drift each leaves."""
    import numpy as np
    import workloads as W
    p = W.wells_3d(m=96, N=512, seed=0)
    out = {"workload": "wells3d_96^3_N512_seed0", "tau": tau, "steps": steps, "warmup": warmup}
    ritzs = {}
    for name, prec, dt_ in (("mixed", ope.OPE_MIXED, np.float32), ("plain_fp64", ope.OPE_FP64, np.float64)):
        with ope.Context(p.grid, p.V, p.N, precision=prec) as ctx:
            U = torch.from_numpy(p.U0.astype(dt_)).to("cuda")
            for _ in range(warmup):
                ope.ope_step(ctx.handle, U, tau)
            torch.cuda.synchronize()
            inner = 0
            t0 = time.perf_counter()
            for _ in range(steps):
                inner += ope.ope_step(ctx.handle, U, tau).inner_iterations
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            res, ritz, drift = ope.ope_residual(ctx.handle, U, p.N)
        out[name] = {"iter_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps, "inner_iterations_per_step": inner / steps,
                     "residual_at_end": res, "drift_at_end": drift}
        ritzs[name] = np.asarray(ritz)
    out["speedup_mixed"] = out["mixed"]["iter_per_s"] / out["plain_fp64"]["iter_per_s"]
    out["ritz_max_rel_diff_mixed_vs_fp64_same_steps"] = float(
        np.max(np.abs(ritzs["mixed"] - ritzs["plain_fp64"]) / np.abs(ritzs["plain_fp64"])))
    return out


def net_forward_rate(ope, torch, reps=10):
    """The network alone on 128 residual columns of the 64^3 workload (the
    learned step's dominant kernels): algorithmic TFLOP/s of the forward pass."""
    import numpy as np
    import workloads as W
    p = W.wells_3d(m=64, N=128, seed=0, with_u0=False)
    n = p.grid.n
    with ope.Context(p.grid, p.V, 128) as ctx, ope.Net(ctx, 128, ope.load_net_weights()) as net:
        X = torch.randn(128, n, device="cuda", dtype=torch.float32)
        F = torch.empty_like(X)
        ope.ope_net_forward(net.handle, X, None, 128, F)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ope.ope_net_forward(net.handle, X, None, 128, F)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
    flop = 2.0 * (27 * 2 * 16 + 2 * 27 * 16 * 16 + 27 * 16) * n * 128
    return {"ms_per_application": 1e3 * dt, "algorithmic_TFLOP_per_s": flop / dt / 1e12, "columns": 128,
            "flop_per_application": flop}


def copy_calibration(torch, gib=1.0, reps=5):
    """A plain device copy of known size, for scaling rocprofv3 byte counters."""
    n = int(gib * (1 << 30) // 8)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "reps": reps}))


def mg_post_bytes(n, N):
    """Algorithmic HBM bytes of the finest prolongation + post-smoothing launch
    of a V-cycle: read r and write z (two n x N FP64 blocks), read the coarse
    correction (an eighth of a block), the diagonal and the Jacobi factors
    (two n-entry arrays)."""
    return 2.125 * n * N * 8 + 16 * n


def step_rate(ope, torch, p, args, multigrid):
    """Outer steps per second of the plain FP64 step on workload p over the
    window (warm-up, then timed steps from the seeded start), with or without
    the multigrid-preconditioned Step 1, with the live roofline of the dominant
    kernel, CG sweep B (HIP events the library records on its own stream, over
    the timed steps)."""
    n, N = p.grid.n, p.N
    U = torch.from_numpy(p.U0).to("cuda")
    ctx = ope.Context(p.grid, p.V, N)
    h = ctx.handle
    levels = coarsest = 0
    if multigrid:
        ope.ope_set_multigrid(h, True)
        levels, coarsest = ope.ope_mg_info(h)
    for _ in range(args.warmup):
        ope.ope_step(h, U, args.tau)
    torch.cuda.synchronize()
    # the dominant kernel of both steps is CG sweep B (at 64^3, N = 128 with the
    # V-cycle: its two forms 1.5 ms of a 6.9 ms step, then the four row
    # products 1.1 ms and the fused post-smoothing 0.7 ms; without the V-cycle
    # 8.2 ms of 28.6)
    ope.ope_profile_begin(h, ope.OPE_KERNEL_CG_SWEEP_B)
    inner = 0
    its = []
    last = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = ope.ope_step(h, U, args.tau)
        inner += last.inner_iterations
        its.append(last.inner_iterations)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, total_ms, tags, lms = ope.ope_profile_end_launches(h, 1 << 20)
    dt = t1 - t0
    ms_per_step = 1e3 * dt / max(args.steps, 1)
    name = "cg_sweep_b"
    # Every step's CG starts at iteration tag 0; the iterations with a tag
    # below the step's inner_iterations ran a full sweep B (even: 3 blocks,
    # odd: 6 blocks, plus the diagonal), the ones enqueued past the
    # convergence of every column return at once or, in an odd iteration, add
    # only the pending y term.  The roofline is taken over the full sweeps.
    full, full_ms, full_bytes, parity = full_sweep_b(tags, lms, its, launches, n, N)
    # the counter record lists the even form first, then the odd one
    traffic = traffic_from_pmc(n, N, "cg_sweep_b", mix=parity if full else None)
    if full:
        nbytes = full_bytes / full
        avg_ms = full_ms / full
    else:
        # no per-launch tags: every counted CG iteration taken as one full sweep
        full, nbytes, avg_ms, full_ms = inner, sweep_b_bytes(n, N), total_ms / max(inner, 1), total_ms
    achieved = nbytes / (avg_ms * 1e-3) / 1e9
    res = {
        "iter_per_s": args.steps / dt, "ms_per_step": ms_per_step,
        "inner_iterations_per_step": inner / max(args.steps, 1),
        "residual_at_end": last.residual if last else None, "drift_at_end": last.drift if last else None,
        "levels": levels, "coarsest_nodes": coarsest,
        "roofline": {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "algorithmic_bytes": nbytes,
                     "avg_launch_ms": avg_ms, "working_launches": full, "launches": launches,
                     "working_ms": full_ms, "total_ms": total_ms,
                     "avg_ms_all_launches": total_ms / max(launches, 1)},
    }
    if not args.no_extras:
        kernels = {}
        ids = [("stencil", ope.OPE_KERNEL_STENCIL), ("cg_sweep_a", ope.OPE_KERNEL_CG_SWEEP_A),
               ("cg_sweep_b", ope.OPE_KERNEL_CG_SWEEP_B), ("cg_sweep_b_odd", ope.OPE_KERNEL_CG_SWEEP_B_Y),
               ("cg_reduce", ope.OPE_KERNEL_CG_REDUCE), ("gram", ope.OPE_KERNEL_GRAM),
               ("rowmm", ope.OPE_KERNEL_ROWMM), ("small", ope.OPE_KERNEL_SMALL)]
        if multigrid:
            ids += [("vcycle", ope.OPE_KERNEL_MG), ("mg_post", ope.OPE_KERNEL_MG_POST)]
        for kname, k in ids:
            ope.ope_profile_begin(h, k)
            its = 0
            for _ in range(5):
                its += ope.ope_step(h, U, args.tau).inner_iterations
            nl, tms = ope.ope_profile_end(h)
            # a CG sweep's (or V-cycle's) time per working launch, as above
            if kname in ("cg_sweep_a", "cg_sweep_b", "cg_reduce"):
                per = its
            elif kname == "cg_sweep_b_odd":
                per = its / 2.0
            elif kname in ("vcycle", "mg_post"):
                per = its + 5
            else:
                per = nl
            rec = {"avg_ms": tms / max(per, 1), "launches_per_step": nl / 5.0, "ms_per_step": tms / 5.0}
            b = mg_post_bytes(n, N) if kname == "mg_post" else kernel_bytes(kname, n, N)
            if b:
                rec["GB/s"] = b / (rec["avg_ms"] * 1e-3) / 1e9
                rec["frac"] = rec["GB/s"] / HBM_PEAK_GBS
            if kname == "mg_post":
                rec["algorithmic_bytes"] = b
                rec["traffic"] = traffic_from_pmc(n, N, "mg_post")
            if kname == "gram":
                rec["TFLOP/s_fp64"] = 2.0 * n * N * N / (rec["avg_ms"] * 1e-3) / 1e12
            if kname == "rowmm":
                rec["TFLOP/s_fp64_N_by_N"] = 2.0 * n * N * N / (rec["avg_ms"] * 1e-3) / 1e12
            kernels[kname] = rec
        res["kernels"] = kernels
        # window-independent cost: an inner iteration (both sweeps, the column
        # reductions and, preconditioned, the V-cycle) and what a step spends
        # outside Step 1
        per_it = kernels["cg_sweep_a"]["avg_ms"] + kernels["cg_sweep_b"]["avg_ms"] + kernels["cg_reduce"]["avg_ms"]
        if multigrid:
            per_it += kernels["vcycle"]["avg_ms"]
        its_step = inner / max(args.steps, 1)
        res["cost_model"] = {"ms_per_inner_iteration": per_it, "inner_iterations_per_step": its_step,
                             "ms_per_step_outside_inner": ms_per_step - its_step * per_it,
                             "note": "ms_per_step = inner_iterations_per_step x ms_per_inner_iteration + outside; "
                                     "the iteration count depends on the window (early steps need more)"}
    ctx.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--m", type=int, default=64)
    ap.add_argument("--minutes", type=float, default=16.0, help="wall-time budget of --form longrun")
    ap.add_argument("--mixed", action="store_true", help="--form longrun: the mixed form first, then FP64")
    ap.add_argument("--switch", type=float, default=1e-4, help="--form longrun --mixed: residual at which FP64 takes over")
    ap.add_argument("--mixed-steps", type=int, default=0,
                    help="--form longrun --mixed: a fixed number of mixed steps before FP64")
    ap.add_argument("--recycle", action="store_true",
                    help="--form longrun: the inner CG starts from the previous step's correction")
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tau", type=float, default=45.0)
    ap.add_argument("--cpu-steps", type=int, default=2, help="outer steps of the CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip per-kernel timings and time-to-residual")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a 1 GiB device copy")
    ap.add_argument("--form", choices=["mixed", "learned", "net", "batched", "large", "extrapolate", "energy",
                                       "table1", "hydrogen", "ttr", "graph", "mg", "mgmixed", "longrun"],
                    default=None,
                    help="only run the measurement of one form (short; for profiling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        if int(os.environ.get("RANK", "0")) == 0:
            print("bench.py measures one GPU: the library runs the step on a single MI355X and has no "
                  "multi-GPU path (the grid would shard by z-slabs with halo exchange; not built).", flush=True)
        sys.exit(2)

    import torch
    from paper_2511_06788_amd import ope
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a visible MI355X")
    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.form:
        if args.form == "large":
            r = large_mixed(ope, torch, steps=args.steps, warmup=args.warmup)
        elif args.form == "batched":
            r = batched_throughput(ope, torch, steps=args.steps)
        elif args.form == "graph":
            r = small_batch_graph(ope, torch)
        elif args.form == "net":
            r = net_forward_rate(ope, torch, reps=args.steps)
        elif args.form == "energy":
            r = algorithm1_energy_stops(ope, torch)
        elif args.form == "longrun":
            r = long_run_time_to_residual(ope, torch, minutes=args.minutes, mixed=args.mixed, recycle=args.recycle,
                                          switch=args.switch, mixed_steps=args.mixed_steps)
        elif args.form == "hydrogen":
            r = paper_hydrogen(ope, torch)
        elif args.form == "table1":
            r = paper_table1(ope, torch)
        elif args.form == "ttr":
            r = time_to_residual(ope, torch, m=args.m)
        else:
            p = W.wells_3d(m=args.m, N=args.N, seed=args.seed, tau=args.tau)
            if args.form == "mixed":
                r = steps_per_second(ope, torch, p, args.tau, ope.OPE_MIXED, args.steps, args.warmup)
            elif args.form == "mg":
                r = mg_steps_per_second(ope, torch, p, args.tau, args.steps, args.warmup)
            elif args.form == "mgmixed":
                r = steps_per_second(ope, torch, p, args.tau, ope.OPE_MIXED, args.steps, args.warmup, multigrid=True)
            elif args.form == "extrapolate":
                r = extrapolated_time_to_residual(ope, torch, p, args.tau)
            else:
                r = learned_steps_per_second(ope, torch, p, args.tau, args.steps, args.warmup)
        print(json.dumps({"form": args.form, **r}), flush=True)
        return

    log(f"building workload {args.m}^3 N={args.N} seed={args.seed}")
    p = W.wells_3d(m=args.m, N=args.N, seed=args.seed, tau=args.tau)
    n, N = p.grid.n, p.N

    log("multigrid-preconditioned step (the headline)")
    mg = step_rate(ope, torch, p, args, multigrid=True)
    log("plain CG step")
    plain = step_rate(ope, torch, p, args, multigrid=False)
    out = {
        "metric": METRIC,
        "value": mg["iter_per_s"],
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mg["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"wells3d_{args.m}^3_N{N}_seed{args.seed}", "n": n, "N": N, "tau": args.tau,
                   "form": "plain FP64",
                   "inner": "preconditioned CG, one symmetric multigrid V-cycle per iteration, "
                            "eta = max(1e-12, 0.25 res), warm start U Lam^-1",
                   "window": {"warmup_steps": args.warmup, "timed_steps": args.steps,
                              "start": "seeded orthonormal start block"}},
        "roofline": mg["roofline"],
        "inner_iterations_per_step": mg["inner_iterations_per_step"],
        "residual_at_end": mg["residual_at_end"],
        "drift_at_end": mg["drift_at_end"],
        "multigrid": {"levels": mg["levels"], "coarsest_nodes": mg["coarsest_nodes"]},
    }
    if "kernels" in mg:
        out["kernels"] = mg["kernels"]
        out["cost_model"] = mg["cost_model"]
    out["plain_cg"] = {k: plain[k] for k in ("iter_per_s", "ms_per_step", "inner_iterations_per_step", "roofline",
                                             "residual_at_end", "drift_at_end")}
    if "kernels" in plain:
        out["plain_cg"]["kernels"] = plain["kernels"]
        out["plain_cg"]["cost_model"] = plain["cost_model"]
    out["speedup_multigrid_vs_plain_cg"] = mg["iter_per_s"] / plain["iter_per_s"]
    ms_per_step = plain["ms_per_step"]
    dt = plain["ms_per_step"] * args.steps / 1e3
    inner = plain["inner_iterations_per_step"] * args.steps
    if not args.no_extras:
        log("mixed-precision form at the same workload")
        ks = min(args.steps, 100)
        out["forms"] = {
            "plain_fp64_multigrid": {"iter_per_s": mg["iter_per_s"], "ms_per_step": mg["ms_per_step"],
                                     "inner_iterations_per_step": mg["inner_iterations_per_step"]},
            "plain_fp64": {"iter_per_s": args.steps / dt, "ms_per_step": ms_per_step,
                           "inner_iterations_per_step": inner / max(args.steps, 1)},
            "mixed": steps_per_second(ope, torch, p, args.tau, ope.OPE_MIXED, ks, args.warmup),
            "mixed_multigrid": steps_per_second(ope, torch, p, args.tau, ope.OPE_MIXED, ks, args.warmup,
                                                multigrid=True),
        }
        log("learned form at the same workload")
        out["forms"]["learned"] = learned_steps_per_second(ope, torch, p, args.tau, min(ks, 40), 5)
        log("time to residual on the 64^3 N=17 problem")
        out["time_to_residual"] = time_to_residual(ope, torch)
        log("time to residual on the 96^3 N=17 problem")
        out["time_to_residual_96"] = time_to_residual(ope, torch, m=96)
        log("extrapolated time to residual 1e-8 at 64^3, N=128")
        out["time_to_residual_64_N128_extrapolated"] = extrapolated_time_to_residual(ope, torch, p, args.tau)
        out["time_to_residual_64_N128_extrapolated_plain_cg"] = extrapolated_time_to_residual(
            ope, torch, p, args.tau, run=60, multigrid=False)
        log("Algorithm 1 energy stops and the adaptive step (64^3, N=17)")
        out["algorithm1_energy_stops"] = algorithm1_energy_stops(ope, torch)
        log("Table 1 on the finite-difference oscillator")
        out["paper_table1"] = paper_table1(ope, torch)
        out["paper_hydrogen"] = paper_hydrogen(ope, torch)
        log("batched workload (64 problems)")
        out["batched"] = batched_throughput(ope, torch)
        log("batch of small problems: eager steps and graph replays")
        out["small_batch"] = small_batch_graph(ope, torch)
        log("large mixed-precision workload (96^3, N=512)")
        out["large_mixed"] = large_mixed(ope, torch)
        log("network forward pass")
        out["net_forward"] = net_forward_rate(ope, torch)

    if not args.no_cpu_baseline:
        log(f"cpu baseline: {args.cpu_steps} oracle step(s)")
        out["cpu_baseline"] = cpu_baseline(p, args.tau, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
