#!/usr/bin/env python3
"""Benchmark of the polarization-solve hot path on one MI355X.

One step = one pass of the whole path over one synthetic configuration:
pe_set_system (wrap, cell sort, bead-bead real-space operator), the
right-hand side (ion potential at the beads), the Krylov solve to a double
relative residual of 1e-6 (float operator inside double refinement, started
from the learned guess when a trained model is given), and the force pass
(forces, torques, energies).  Inputs are resident in HBM before timing.

Printed: one JSON line with the metric, the live per-kernel roofline of the
dominant kernel (HIP events around every launch in the timed region), the
plain-FP64 arm for comparison, and the CPU oracle timed on a bounded sample.
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


def algorithmic_bytes(cls, dbl, n_part, n_set_particles, G, Gc, nnz_stored):
    """Minimum HBM bytes one launch of a kernel class must move.

    s = bytes per real.  Particle records read by spread/gather: position
    (4 doubles incl. width), caller index (4 B), charge or output (8 B).
    """
    s = 8 if dbl else 4
    if cls == "spread":
        return n_set_particles * (32 + 4 + 8) + G * s            # particles in, grid out
    if cls == "gather":
        return n_set_particles * (32 + 4 + 8) + G * s            # grid in, potentials out
    if cls in ("fft_y_fwd", "fft_y_inv", "fft_x_scale"):
        return 2 * Gc * 2 * s                                     # complex half grid in and out
    if cls == "fft_z_r2c":
        return G * s + Gc * 2 * s
    if cls == "fft_z_c2r":
        return Gc * 2 * s + G * s
    if cls == "spmv":
        return nnz_stored * (s + 4) + n_part * (8 + 8 + 8 + 32)  # matrix + q, phi_wave, y, row data
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
    ap.add_argument("--workload", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--model", default=None, help="trained learned-guess weights (pe_guess_save format)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-arm", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=50)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (the solve is not sharded across GPUs); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2401_04865_amd import binding as B
    from paper_2401_04865_amd import inputs

    torch.cuda.set_device(0)
    k, desc = WORKLOADS[args.workload]
    t0 = time.perf_counter()
    system = inputs.config(k)
    t_gen = time.perf_counter() - t0
    print(f"[bench] {args.workload}: {system.n_bead} beads, {system.n_body} bodies, {system.n_ion} ions, "
          f"mesh {system.mesh} (inputs {t_gen:.1f} s)", file=sys.stderr, flush=True)
    tol = SPLIT_TOL[args.workload]

    def make_ctx(prec, learned=False):
        p = B.make_params(system.box, system.mesh, P=8, split_tol=tol, rel_tol=1e-6, precision=prec,
                          use_learned_guess=1 if learned else 0)
        ctx = B.Context(p)
        ctx.load(system)
        return ctx

    learned = False
    ctx = make_ctx(B.PE_MIXED)
    if args.model and os.path.exists(args.model):
        ctx.pe_guess_load(args.model)
        ctx.close()
        ctx = make_ctx(B.PE_MIXED, learned=True)
        ctx.pe_guess_load(args.model)
        learned = True
    d = ctx.pe_get_derived()
    dev = ctx.sys_dev
    off = system.body_offsets
    nb, nbody, ni = system.n_bead, system.n_body, system.n_ion
    q = torch.empty(nb, dtype=torch.float64, device="cuda")
    dpsi = torch.empty(nbody, dtype=torch.float64, device="cuda")
    S = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    F = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    L = torch.empty((nbody, 3), dtype=torch.float64, device="cuda")
    U = torch.empty(nbody, dtype=torch.float64, device="cuda")
    fi = torch.empty((max(ni, 1), 3), dtype=torch.float64, device="cuda")

    def step(c):
        c.pe_set_system(off, dev["bead_pos"], dev["bead_sigma"], dev["body_center"], dev["body_quat"],
                        dev["body_charge"], dev["ion_pos"] if ni else None, dev["ion_charge"] if ni else None,
                        dev["ion_sigma"] if ni else None, system.E0)
        st, info = c.pe_solve_polarization(None, q, dpsi, S)
        c.pe_forces_torques(F, L, U, fi if ni else None, None)
        return info

    for _ in range(args.warmup):
        step(ctx)
    torch.cuda.synchronize()
    ctx.pe_profile_enable(True)
    infos = []
    t_steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        info = step(ctx)
        t_steps.append(time.perf_counter() - ts)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.pe_profile_read()
    ctx.pe_profile_enable(False)
    solve_ms = [1e3 * i.t_total for i in infos]
    print(f"[bench] timed {args.steps} steps: {elapsed:.3f} s; solve p50 {np.median(solve_ms):.2f} ms, "
          f"iters {infos[-1].iters}, outer {infos[-1].outer_refinements}, rel {infos[-1].rel_residual:.2e}",
          file=sys.stderr, flush=True)

    # bead-only PME matvec throughput (the Krylov operator), both precisions
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
        matvec[name] = {"ms": 1e3 * tm, "mbeads_s": nb / tm / 1e6}

    # plain FP64 arm (zero guess)
    fp64 = None
    if not args.no_fp64_arm:
        c64 = make_ctx(B.PE_FP64)
        for _ in range(1):
            step(c64)
        torch.cuda.synchronize()
        i64 = []
        n64 = max(3, min(args.steps, 10))
        for _ in range(n64):
            i64.append(step(c64))
        ms64 = [1e3 * i.t_total for i in i64]
        fp64 = {"solve_ms_p50": float(np.median(ms64)), "iters": int(i64[-1].iters),
                "rel_residual": float(i64[-1].rel_residual), "solves": n64}
        c64.close()

    # roofline of the dominant kernel (live HIP-event timing of the timed region)
    G = int(np.prod(system.mesh))
    Gc = system.mesh[0] * system.mesh[1] * (system.mesh[2] // 2 + 1)
    nnz_stored = d["nnz"]
    classes = B.PROF_CLASSES
    per_class = {}
    for name in classes:
        for dbl in (False, True):
            cnt, ms = prof[name] if not dbl else prof[name + "_f64"]
            if cnt:
                per_class[(name, dbl)] = (cnt, ms)
    dom = max(per_class, key=lambda kk: per_class[kk][1])
    cnt, ms = per_class[dom]
    avg_ms = ms / cnt
    name, dbl = dom
    # spread/gather launches per matvec cover beads (solve) or beads+ions (RHS / forces):
    n_launch_particles = nb
    abytes = algorithmic_bytes(name, dbl, nb, n_launch_particles, G, Gc, nnz_stored)
    roof = None
    if abytes is not None:
        achieved = abytes / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": f"{name}_{'f64' if dbl else 'f32'}", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_us": round(1e3 * avg_ms, 2), "launches": int(cnt), "alg_bytes_per_launch": int(abytes)}
    breakdown = {f"{n}_{'f64' if db else 'f32'}": {"launches": int(c), "total_ms": round(m, 3),
                                                   "avg_us": round(1e3 * m / c, 2)}
                 for (n, db), (c, m) in sorted(per_class.items(), key=lambda kv: -kv[1][1])}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample ...", file=sys.stderr, flush=True)
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
        "config": {"workload": f"{args.workload}: {desc}", "n_bead": nb, "n_body": nbody, "n_ion": ni,
                   "mesh": list(system.mesh), "P": 8, "xi": round(d["xi"], 5), "r_cut": round(d["r_cut"], 5),
                   "eta": round(d["eta"], 5), "bead_pairs_stored": nnz_stored, "rel_tol": 1e-6,
                   "learned_guess": learned, "parallelism": "single GPU"},
        "solve_ms_p50": round(float(np.median(solve_ms)), 3),
        "solve_ms_p99": round(float(np.percentile(solve_ms, 99)), 3),
        "iters": int(infos[-1].iters),
        "outer_refinements": int(infos[-1].outer_refinements),
        "matvecs_fp32": int(infos[-1].matvecs_fp32),
        "matvecs_fp64": int(infos[-1].matvecs_fp64),
        "rel_residual": float(infos[-1].rel_residual),
        "matvec": matvec,
        "fp64_arm": fp64,
        "speedup_solve_vs_fp64": (round(fp64["solve_ms_p50"] / float(np.median(solve_ms)), 3) if fp64 else None),
        "roofline": roof,
        "kernels": breakdown,
        "cpu_baseline": cpu,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
