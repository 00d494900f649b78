#!/usr/bin/env python3
"""Benchmark of the polarization-solve hot path on one MI355X.

One step = one pass of the whole path over one synthetic configuration:
pe_set_system (wrap, cell sort, bead-bead real-space operator), the
right-hand side (ion potential at the beads), the Krylov solve to a double
relative residual of 1e-6 (float operator inside double refinement, started
from the learned guess when a trained model is given), and the force pass
(forces, torques, energies).  Inputs are resident in HBM before timing.

Printed: one JSON line with the metric, the live roofline of the dominant
kernel class (HIP events around its launches in the timed region; which
class dominates, and the per-class breakdown, come from a few untimed steps
with events around every class), the FP64 arms for comparison, and the CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "polarization-solve time & PME matvec Mbeads/s, learned+FP32 vs plain FP64 at 1e-6"

WORKLOADS = {
    "cfg2": (2, "two level-3 icospheres (1284 beads, sigma 0.05) 2.5 apart + 2000 ions, L=30, mesh 64^3, P=8"),
    "cfg3": (3, "4^3 sc lattice of level-3 spheres (41088 beads, sigma 0.05, phi=0.2) + 40000 ions, "
                "L=11.03, mesh 128^3, P=8, split 1e-6"),
    "cfg4": (4, "128 rods + 128 cubes (~257k beads) + 100000 ions, L=32, mesh 192^3, P=8, split 1e-6"),
    "cfg5": (5, "512 level-3 spheres Q=+20 (328704 beads) + 1e6 ions, phi=0.1, mesh 256^3, P=8, split 1e-6"),
}
SPLIT_TOL = {"cfg2": 1e-8, "cfg3": 1e-6, "cfg4": 1e-6, "cfg5": 1e-6}

# HBM bytes per launch (profiler scope) of a kernel class on the default
# workload, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE passes over a short
# run of this script (the class's dispatches of five steps, averaged;
# FETCH_SIZE scaled by 2.0 and WRITE_SIZE by 1.0, the ratios a plain 256 MiB
# device copy reads on those counters).  Each entry
# records the source files of the kernels and of their launches with their
# sha1 at measurement; once one changes the figure is stale and `traffic` is
# reported null, as it is on any other workload.
TRAFFIC = {
    # two rocprofv3 --pmc passes (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0 after a
    # 256 MiB copy calibration) of the 512-sphere workload; one launch is one
    # profiler scope (right-hand side: 399 MB; force pass: 2351 MB)
    "pair_f32": {"workload": "cfg5", "bytes_per_launch": 1.375e9,
                 "sources": {"paper_2401_04865_amd/csrc/realspace.hip": "83ae5a528fd52d9ce40bfb5e8fe773457299762d",
                             "paper_2401_04865_amd/csrc/api.hip": "db2cf28a122a3411da773082a60831037809cb40"}},
}


def traffic_current(entry):
    """True while every source file the figure depends on (the kernels and
    the code that launches them) still has the sha1 recorded with it."""
    import hashlib
    for rel, sha in entry["sources"].items():
        try:
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha1(f.read()).hexdigest() != sha:
                    return False
        except OSError:
            return False
    return True


# Peaks of one MI355X: HBM bandwidth, dense matrix-core and vector rates.
MFMA_PEAK_TFLOPS = {False: 157.3, True: 78.6}     # fp32, fp64 dense matrix
VALU_PEAK_TFLOPS = {False: 157.3, True: 78.6}     # fp32, fp64 vector
PAIR_FLOP = 40   # one pair inside the cutoff: minimum image, r^2, kernel value and slope, field, sums


def kernel_model(cls, dbl, cnt, work, nb, G, Gc):
    """(bound, algorithmic amount over all launches, unit, peak) of a kernel class.

    cnt launches did `work` units (particles, pairs, stored entries or
    multiply-adds, as the library reports them).  Byte counts are the minimum
    HBM traffic: s = bytes per real; a particle record is position + width
    (32 B), index (4 B) and charge or output (8 B); a spread writes and a
    contraction reads the whole grid; the FFT passes read and write the half
    spectrum (or the real grid); the sparse product reads each stored entry
    once.  Dense per-shape products and pair evaluations are counted in
    floating-point operations.
    """
    s = 8 if dbl else 4
    if cls in ("spread", "gather"):
        return "hbm", work * (32 + 4 + 8) + cnt * G * s, "GB/s", HBM_PEAK_GBS
    if cls in ("fft_y_fwd", "fft_y_inv", "fft_x_scale"):
        return "hbm", cnt * 2 * Gc * 2 * s, "GB/s", HBM_PEAK_GBS
    if cls in ("fft_z_r2c", "fft_z_c2r"):
        return "hbm", cnt * (G * s + Gc * 2 * s), "GB/s", HBM_PEAK_GBS
    if cls == "spmv":
        return "hbm", work * (s + 4) + cnt * nb * (8 + 4 + 32 + 8 + 8 + 4 + 8), "GB/s", HBM_PEAK_GBS
    if cls in ("near", "precond"):
        return "mfma", 2.0 * work, "TFLOP/s", MFMA_PEAK_TFLOPS[dbl]
    if cls == "pair":
        return "alu", PAIR_FLOP * work, "TFLOP/s", VALU_PEAK_TFLOPS[dbl]
    return None


def cpu_baseline(system, budget_s=20.0):
    """The FP64 oracle (direct Ewald assembly of M + dense LU) on a bounded
    sample of the same workload, extrapolated to the full bead count."""
    import threadpoolctl
    from oracle import ewald
    n = system.n_bead
    rng = np.random.default_rng(0)
    ns = min(n, 1536)
    idx = np.sort(rng.choice(n, ns, replace=False))
    pos, sig = system.bead_pos[idx], system.bead_sigma[idx]
    xi = 1.0
    t0 = time.perf_counter()
    M = ewald.potential_matrix(pos, sig, system.box, xi)
    t_asm = time.perf_counter() - t0
    nl = min(n, 4096)
    A = np.random.default_rng(1).standard_normal((nl, nl)) + nl * np.eye(nl)
    b = np.ones(nl)
    t0 = time.perf_counter()
    np.linalg.solve(A, b)
    t_lu = time.perf_counter() - t0
    t_full = t_asm * (n / ns) ** 2 + t_lu * (n / nl) ** 3
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    return {
        "value": n / t_full / 1e6, "unit": "Mbeads/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"direct-Ewald assembly of M for {ns} of {n} beads ({t_asm:.2f} s, scaled by (n/ns)^2) "
                   f"+ dense LU of {nl}^2 ({t_lu:.2f} s, scaled by (n/nl)^3); solve time extrapolated "
                   f"{t_full:.3g} s"),
        "seconds_measured": t_asm + t_lu,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--train-systems", type=int, default=4,
                    help="independent configurations of the workload whose solves train the learned guess "
                         "(0: no learned guess)")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-arm", action="store_true")
    ap.add_argument("--fp64-solves", type=int, default=2)
    ap.add_argument("--matvec-reps", type=int, default=20)
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="untimed steps with events around every kernel class (per-class breakdown)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the solve runs on one GPU only (it is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import tempfile

    import torch
    from paper_2401_04865_amd import binding as B
    from paper_2401_04865_amd import inputs

    torch.cuda.set_device(0)
    k, desc = WORKLOADS[args.workload]
    bd_mode = args.workload == "cfg5"
    t0 = time.perf_counter()
    system = inputs.config(k)
    t_gen = time.perf_counter() - t0
    log(f"{args.workload}: {system.n_bead} beads, {system.n_body} bodies, {system.n_ion} ions, "
        f"mesh {system.mesh} (inputs {t_gen:.1f} s)")
    tol = SPLIT_TOL[args.workload]
    nb, nbody, ni = system.n_bead, system.n_body, system.n_ion
    off = system.body_offsets
    dt, kT, gamma, seed = 1e-4, 1.0, 1.0, 20240109

    def params(prec, learned=False, precond=1):
        return B.make_params(system.box, system.mesh, P=8, split_tol=tol, rel_tol=1e-6, precision=prec,
                             use_learned_guess=1 if learned else 0, precond=precond)

    q = torch.empty(nb, dtype=torch.float64, device="cuda")
    dpsi = torch.empty(nbody, dtype=torch.float64, device="cuda")
    S = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    F = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    L = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    U = torch.empty(nbody, dtype=torch.float64, device="cuda")
    fi = torch.empty((max(ni, 1), 3), dtype=torch.float64, device="cuda")
    counter = {"step": 0}

    def step(c, dev, record=False, move=bd_mode):
        tp = [time.perf_counter()]
        c.pe_set_system(off, dev["bead_pos"], dev["bead_sigma"], dev["body_center"], dev["body_quat"],
                        dev["body_charge"], dev["ion_pos"] if ni else None, dev["ion_charge"] if ni else None,
                        dev["ion_sigma"] if ni else None, system.E0)
        tp.append(time.perf_counter())
        st, info = c.pe_solve_polarization(None, q, dpsi, S)
        tp.append(time.perf_counter())
        if record:
            c.pe_guess_record(q)
        c.pe_forces_torques(F, L, U, fi if ni else None, None)
        tp.append(time.perf_counter())
        if move:
            c.pe_bd_step(dt, kT, gamma, seed, counter["step"], dev["bead_pos"], dev["body_center"],
                         dev["body_quat"], dev["ion_pos"] if ni else None)
            counter["step"] += 1
        tp.append(time.perf_counter())
        return info, np.diff(tp)

    # ---- learned guess: train on solves of the method from untimed steps
    learned = args.train_systems > 0
    train_info = None
    wfile = os.path.join(tempfile.mkdtemp(), "guess.bin")
    ctx = B.Context(params(B.PE_MIXED))
    if learned:
        ctx.pe_guess_init(1)
        ta = time.perf_counter()
        for t in range(args.train_systems):
            ts = inputs.config(k, seed=inputs.SEED_BASE + 1000 + t)
            ctx.load(ts)
            ctx.pe_guess_set_types(ts.body_type)
            st, _ = ctx.pe_solve_polarization(None, q, dpsi, S)
            ctx.pe_guess_record(q)
        tb = time.perf_counter()
        loss0 = ctx.pe_guess_train(1, 4096, 1e-3, 1)
        loss = ctx.pe_guess_train(args.epochs, 4096, 2e-3, 2)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        ctx.pe_guess_save(wfile)
        train_info = {"solves": args.train_systems, "rows": args.train_systems * nb, "epochs": args.epochs + 1,
                      "loss_first_epoch": loss0, "loss_last_epoch": loss, "generate_s": round(tb - ta, 2),
                      "train_s": round(tc - tb, 2)}
        log(f"learned guess: {train_info}")
        ctx.close()
        ctx = B.Context(params(B.PE_MIXED, learned=True))
        ctx.pe_guess_load(wfile)
        ctx.load(system)
        dev = ctx.sys_dev
        ctx.pe_set_system(off, dev["bead_pos"], dev["bead_sigma"], dev["body_center"], dev["body_quat"],
                          dev["body_charge"], dev["ion_pos"] if ni else None, dev["ion_charge"] if ni else None,
                          dev["ion_sigma"] if ni else None, system.E0)
        ctx.pe_guess_set_types(system.body_type)
    else:
        ctx.load(system)
        dev = ctx.sys_dev
    d = ctx.pe_get_derived()
    for _ in range(args.warmup):
        step(ctx, dev)
    G = int(np.prod(system.mesh))
    Gc = system.mesh[0] * system.mesh[1] * (system.mesh[2] // 2 + 1)

    def classes_of(prof):
        per = {}
        for name in B.PROF_CLASSES:
            for dbl in (False, True):
                cnt, ms, work = prof[name] if not dbl else prof[name + "_f64"]
                if cnt:
                    per[(name, dbl)] = (cnt, ms, work)
        return per

    # profiled steps (events around every kernel class; untimed): the
    # per-class breakdown, and which modeled class dominates
    torch.cuda.synchronize()
    ctx.pe_profile_enable(True)
    for _ in range(args.profile_steps):
        step(ctx, dev)
    torch.cuda.synchronize()
    per_class = classes_of(ctx.pe_profile_read())
    ctx.pe_profile_enable(False)
    ranked = sorted(per_class, key=lambda kk: -per_class[kk][1])
    modeled = [kk for kk in ranked
               if kernel_model(kk[0], kk[1], per_class[kk][0], per_class[kk][2], nb, G, Gc) is not None]
    dominant = modeled[0] if modeled else None

    # timed steps: events only around the dominant class's launches, so its
    # roofline is measured live while the rest runs undisturbed
    ctx.pe_profile_select([dominant[0]] if dominant else [])
    ctx.pe_profile_enable(True)
    infos, phases = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, ph = step(ctx, dev)
        infos.append(info)
        phases.append(ph)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed_class = classes_of(ctx.pe_profile_read())
    ctx.pe_profile_enable(False)
    ctx.pe_profile_select(None)
    solve_ms = [1e3 * i.t_total for i in infos]
    ph = 1e3 * np.median(np.array(phases), axis=0)
    log(f"timed {args.steps} steps: {elapsed:.3f} s; solve p50 {np.median(solve_ms):.2f} ms, iters "
        f"{[i.iters for i in infos]}, guess residual {infos[-1].rel_residual_guess:.3f}")

    # bead-only PME matvec throughput (the Krylov operator), both precisions, on the current configuration
    ctx.pe_set_system(off, dev["bead_pos"], dev["bead_sigma"], dev["body_center"], dev["body_quat"],
                      dev["body_charge"], dev["ion_pos"] if ni else None, dev["ion_charge"] if ni else None,
                      dev["ion_sigma"] if ni else None, system.E0)
    x = torch.randn(nb + nbody, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    matvec = {}
    for name, prec in (("fp32", B.PE_MIXED), ("fp64", B.PE_FP64)):
        for _ in range(3):
            ctx.pe_apply_saddle(x, y, prec)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(args.matvec_reps):
            ctx.pe_apply_saddle(x, y, prec)
        torch.cuda.synchronize()
        tm = (time.perf_counter() - ta) / args.matvec_reps
        matvec[name] = {"ms": round(1e3 * tm, 4), "mbeads_s": round(nb / tm / 1e6, 2)}

    # comparison arms on the same configuration, zero initial guess: the method as stated (double,
    # unpreconditioned GMRES), double with the block preconditioner, and mixed precision with the
    # preconditioner but without the learned guess
    fp64 = None
    if not args.no_fp64_arm:
        arms = {}
        for name, prec, pre in (("plain_fp64", B.PE_FP64, 0), ("fp64_precond", B.PE_FP64, 1),
                                ("mixed_precond_zero_guess", B.PE_MIXED, 1)):
            p = params(prec, precond=pre)
            p.max_iters = 4000
            c64 = B.Context(p)
            c64.sys_dev = dev
            ms, its = [], []
            for _ in range(args.fp64_solves):
                info, _ = step(c64, dev, move=False)
                ms.append(1e3 * info.t_total)
                its.append(info.iters)
            arms[name] = {"solve_ms_p50": round(float(np.median(ms)), 3), "iters": its,
                          "rel_residual": float(info.rel_residual)}
            c64.close()
        fp64 = arms

    # roofline of the dominant kernel class: live HIP-event timing of its
    # launches in the timed region; the other classes from the profiled steps
    total_ms = sum(v[1] for v in per_class.values())

    def roofline(name, dbl, source=per_class):
        cnt, ms, work = source[(name, dbl)]
        model = kernel_model(name, dbl, cnt, work, nb, G, Gc)
        if model is None:
            return None
        bound, amount, unit, peak = model
        achieved = amount / (ms * 1e-3) / (1e9 if unit == "GB/s" else 1e12)
        key = f"{name}_{'f64' if dbl else 'f32'}"
        tr = TRAFFIC.get(key)
        # a figure holds only for the workload it was counted on
        traffic = (tr["bytes_per_launch"] if tr and tr["workload"] == args.workload and traffic_current(tr)
                   else None)
        share = per_class[(name, dbl)][1] / total_ms
        return {"kernel": key, "bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "avg_launch_us": round(1e3 * ms / cnt, 2), "launches": int(cnt),
                "algorithmic_per_launch": amount / cnt, "share_of_kernel_time": round(share, 3)}

    roofs = [r for r in (roofline(n, db) for n, db in modeled) if r is not None]
    roof = None
    if dominant and dominant in timed_class:
        roof = roofline(*dominant, source=timed_class)
        roof["timing"] = "HIP events around this class's launches in the timed steps"
    breakdown = {f"{n}_{'f64' if db else 'f32'}": {"launches": int(c), "total_ms": round(m, 3),
                                                   "avg_us": round(1e3 * m / c, 2), "work": w}
                 for (n, db), (c, m, w) in sorted(per_class.items(), key=lambda kv: -kv[1][1])}

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(system)

    ms_per_step = 1e3 * elapsed / args.steps
    value = nb * args.steps / elapsed / 1e6
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "Mbeads/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}" + (", Brownian dynamics dt=1e-4" if bd_mode else ""),
                   "n_bead": nb, "n_body": nbody, "n_ion": ni, "mesh": list(system.mesh), "P": 8,
                   "xi": round(d["xi"], 5), "r_cut": round(d["r_cut"], 5), "eta": round(d["eta"], 5),
                   "bead_pairs_stored": d["nnz"], "rel_tol": 1e-6, "learned_guess": learned,
                   "precond": "block-Jacobi", "parallelism": "single GPU"},
        "step_phases_ms_p50": {"set_system": round(ph[0], 3), "solve": round(ph[1], 3), "forces": round(ph[2], 3),
                               "bd_update": round(ph[3], 3)},
        "steps_per_s": round(args.steps / elapsed, 3),
        "solve_ms_p50": round(float(np.median(solve_ms)), 3),
        "solve_ms_p99": round(float(np.percentile(solve_ms, 99)), 3),
        "iters": [int(i.iters) for i in infos],
        "outer_refinements": int(infos[-1].outer_refinements),
        "matvecs_fp32": int(infos[-1].matvecs_fp32),
        "matvecs_fp64": int(infos[-1].matvecs_fp64),
        "rel_residual": float(infos[-1].rel_residual),
        "rel_residual_guess": float(infos[-1].rel_residual_guess),
        "learned_guess_training": train_info,
        "matvec": matvec,
        "fp64_arms": fp64,
        "speedup_solve_vs_plain_fp64": (round(fp64["plain_fp64"]["solve_ms_p50"] / float(np.median(solve_ms)), 2)
                                        if fp64 else None),
        "roofline": roof,
        "roofline_by_class": roofs[1:6],
        "kernels": breakdown,
        "kernels_from": f"{args.profile_steps} profiled steps after the warmup (events around every class)",
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
