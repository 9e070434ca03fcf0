"""Benchmark of one implicit BDEM time step on one MI355X.

Workload: the paper-scale ceramic plate (117x117x16 close-packed layers =
219,024 particles, ~1.36M bonds, E = 5e10 Pa, dropped at 8 m/s onto the
ground, dt = 3.5e-5 s), seeded synthetic input resident in HBM.  A "step" is
one bdem_step: prediction, Newton iterations (bond evaluation, assembly,
block-Jacobi PCG, exp-map line search), velocity update and fracture test.

Prints one JSON line: Newton iterations per second of the mixed-precision
path (value), bond-Hessian evaluations per second, the plain FP64 path and the
ratio, the SpMV roofline and the oracle's CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton iters/s + bond Hessian evals/s, 219K particles, FP32-mixed vs FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "spmv_ceramic_plate_219k.md")


def spmv_source_digest():
    """sha256 of the SpMV kernel's source text (the k_spmv template and the
    SPMV_* tiling constants): HBM counter figures recorded for one digest are
    stale once it changes."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2308_10459_amd", "csrc")
    src = open(os.path.join(csrc, "k_solve.hip")).read()
    m = re.search(r"template <typename T, int NT, int U> __global__ __launch_bounds__\([^)]*\) void k_spmv.*?\n}\n",
                  src, re.S)
    consts = [ln for ln in open(os.path.join(csrc, "bdem_internal.hpp")) if "SPMV_" in ln]
    text = (m.group(0) if m else "") + "".join(consts)
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def recorded_traffic():
    """HBM bytes per SpMV launch from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    import re
    try:
        txt = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(r"TRAFFIC kernel=k_spmv<float> digest=(\w+) fetch_bytes=(\d+) write_bytes=(\d+)", txt)
    if not m or m.group(1) != spmv_source_digest():
        return None
    return int(m.group(2)) + int(m.group(3))


def spmv_algorithmic_bytes(n, nb_alive, elt):
    """Bytes one SpMV must move at least: every unique block once (one 6x6 per
    bond, the 21 packed values of each diagonal block), the bond's index pair,
    the input vector read once and the output written once (FP64)."""
    return nb_alive * 36 * elt + n * 21 * elt + nb_alive * 8 + 2 * 6 * n * 8


def bond_algorithmic_bytes(n, nb_alive, elt):
    """Bytes of one bond evaluation (both bond kernels): state read once
    (p, q: 64 B per particle), bond topology and rest data (8 + 64 B), unique
    Hessian blocks written (36 per bond, 21 per diagonal) and the FP64 gradient."""
    return n * 64 + nb_alive * 72 + nb_alive * 36 * elt + n * 21 * elt + n * 48


def run_path(scene, mixed, steps, warmup, profile, **opts):
    """Warm up, then time `steps` implicit steps with the library defaults.
    With profile, HIP events on the library's stream bracket every bond
    evaluation and every SpMV launch of the timed steps; PCG issues one
    iteration ahead of its convergence poll and the timings of the one
    iteration issued after convergence (whose kernels return at once) are
    dropped, so the SpMV average covers working launches only."""
    import torch
    from paper_2308_10459_amd import bdem as B
    prec = B.BDEM_PREC_MIXED if mixed else B.BDEM_PREC_FP64
    sim = B.Simulator(scene, precision=prec, **opts)
    tuning = sim.autotune([scene.dt])
    log(f"  autotuned: {tuning}")
    if profile:   # per-launch events need ungraphed launches; the poll interval stays tuned
        sim.set_tuning(use_graph=0)
    for k in range(warmup):
        st = sim.step(scene.dt)
        log(f"  warmup {k}: newton {st['newton_iters']} cg {st['cg_iters']} broken {st['bonds_broken']}")
    B.bdem_set_profiling(sim.ctx, profile)
    tot = dict(newton=0, cg=0, ls=0, bond_ms=0.0, spmv_ms=0.0, bond_launch=0, spmv_launch=0,
               broken=0, step_ms=[], step_newton=[])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        st = sim.step(scene.dt)
        nb_launch, sp_launch = B.bdem_profile_counts(sim.ctx)
        tot["newton"] += st["newton_iters"]
        tot["cg"] += st["cg_iters"]
        tot["ls"] += st["ls_backtracks"]
        tot["bond_ms"] += st["t_ms"][6]
        tot["spmv_ms"] += st["t_ms"][7]
        tot["bond_launch"] += nb_launch
        tot["spmv_launch"] += sp_launch
        tot["broken"] += st["bonds_broken"]
        tot["step_ms"].append(st["t_ms"][5])
        tot["step_newton"].append(st["newton_iters"])
        log(f"  step {k}: newton {st['newton_iters']} cg {st['cg_iters']} ls {st['ls_backtracks']} "
            f"broken {st['bonds_broken']} rc {st['rc']} {st['t_ms'][5]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    alive = int(sim.get_state()["alive"].sum())
    sim.close()
    tot["wall_s"] = wall
    tot["alive_bonds"] = alive
    tot["tuning"] = tuning
    return tot


def run_batch(steps, warmup):
    """The 64-scene batch (992,148 particles, seeded sizes 2K-50K, per-scene
    dt): aggregate particle-steps per second of the mixed path stepping all
    scenes in one batched call, of the FP64 path batched, and of the FP64
    path stepping the scenes one after another (each scene alone).  Every
    handle is autotuned on its own scenes first, as in the single-scene runs."""
    import torch
    from paper_2308_10459_amd import bdem as B
    from paper_2308_10459_amd import scenes as S
    sc = S.make_batch()
    out = {"workload": f"{sc.name}: {sc.n} particles, {sc.nb} bonds, 64 scenes of 2K-50K particles, "
                       "per-scene dt = 50 x the period estimate", "steps": steps}
    for label, prec in (("mixed_batched", B.BDEM_PREC_MIXED), ("fp64_batched", B.BDEM_PREC_FP64)):
        sim = B.Simulator(sc, precision=prec)
        tuning = sim.autotune(sc.dt_per_scene)
        log(f"  batch {label} autotuned: {tuning}")
        for _ in range(warmup):
            sim.step_batched(sc.dt_per_scene)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        newton = 0
        for _ in range(steps):
            rc, stats = sim.step_batched(sc.dt_per_scene)
            newton += sum(st["newton_iters"] for st in stats)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        out[label] = sc.n * steps / wall
        log(f"  batch {label}: {1e3 * wall / steps:.1f} ms/step, {newton} Newton iterations summed over scenes")
    wall = 0.0
    for s in range(len(sc.dt_per_scene)):
        m = S.subset_scenes(sc, [s])
        sim = B.Simulator(m, precision=B.BDEM_PREC_FP64)
        sim.autotune(m.dt_per_scene)
        for _ in range(warmup):
            sim.step_batched(m.dt_per_scene)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sim.step_batched(m.dt_per_scene)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        sim.close()
    out["fp64_sequential"] = sc.n * steps / wall
    out["unit"] = "particle-steps/s"
    out["mixed_batched_over_fp64_sequential"] = out["mixed_batched"] / out["fp64_sequential"]
    log(f"  batch fp64 one scene at a time: {1e3 * wall / steps:.1f} ms per step of all scenes")
    return out


def run_solver_comparison(max_first_order=20000, rtol=1e-6):
    """Algorithm 1 (first-order) against Algorithm 2 (second-order) on the
    1000-particle block (FP64): iterations and time of one step to the same
    relative gradient tolerance, the comparison the paper makes."""
    import torch
    from paper_2308_10459_amd import bdem as B
    from paper_2308_10459_amd import scenes as S
    sc = S.make_block()
    out = {"workload": f"{sc.name}: {sc.n} particles, {sc.nb} bonds, E=1e7, dt={sc.dt}, one step to "
                       f"|grad f| <= {rtol} |grad f_0|"}
    for label, solver, cap in (("second_order", B.BDEM_SOLVER_NEWTON, 200),
                               ("first_order", B.BDEM_SOLVER_FIRST_ORDER, max_first_order)):
        sim = B.Simulator(sc, precision=B.BDEM_PREC_FP64, solver=solver, newton_rtol=rtol, max_newton=cap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sim.step(sc.dt)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sim.close()
        out[label] = {"iterations": st["newton_iters"], "cg_iterations": st["cg_iters"],
                      "ms": 1e3 * wall, "grad_reduction": st["grad_final"] / st["grad0"],
                      "converged": st["status"] == 0}
        log(f"  {label}: {st['newton_iters']} iterations, {1e3 * wall:.1f} ms, "
            f"|z| {st['grad0']:.3e} -> {st['grad_final']:.3e}")
    return out


def run_integrator_comparison(scene, steps, warmup):
    """The variational midpoint form of Section 3.1 on the bench workload
    (mixed path), against the implicit-Euler form timed above: Newton
    iterations per second and per step, CG iterations per Newton iteration."""
    from paper_2308_10459_amd import bdem as B
    r = run_path(scene, True, steps, warmup, profile=False, integrator=B.BDEM_INTEGRATOR_MIDPOINT)
    return {"integrator": "midpoint", "steps": steps, "warmup": warmup,
            "newton_iters_per_s": r["newton"] / r["wall_s"],
            "ms_per_step": 1e3 * r["wall_s"] / steps,
            "newton_iters_per_step": r["newton"] / steps,
            "cg_iters_per_newton": r["cg"] / max(r["newton"], 1),
            "bonds_broken": r["broken"]}


def run_precond_comparison(scene, steps, warmup):
    """The bench workload (mixed path, same steps) with the aggregation
    multigrid preconditioner instead of block-Jacobi (Section 5.3 solves with
    AMG-PCG): Newton iterations per second, per step and CG iterations per
    Newton iteration."""
    from paper_2308_10459_amd import bdem as B
    r = run_path(scene, True, steps, warmup, profile=False, preconditioner=B.BDEM_PRECOND_AMG)
    return {"preconditioner": "aggregation multigrid", "steps": steps, "warmup": warmup,
            "newton_iters_per_s": r["newton"] / r["wall_s"],
            "ms_per_step": 1e3 * r["wall_s"] / steps,
            "newton_iters_per_step": r["newton"] / steps,
            "cg_iters_per_newton": r["cg"] / max(r["newton"], 1),
            "bonds_broken": r["broken"]}


def run_contact_comparison(scene, steps):
    """The bench workload (mixed path) from its initial state, with and
    without the element repulsion of Section 5.4 (k_ec = E_max r_max,
    candidates within r_i + r_j + r_max): per-step time, Newton and CG
    iterations, and the time per Newton iteration, which carries the cost of
    the per-step broad phase, the per-iteration repulsion terms and the extra
    PCG coupling kernel.  Steps are counted from the impact on, where the
    repulsion between the pairs of bonds broken at impact (jittered rest
    distances, so some overlap) changes the dynamics; the two columns are
    therefore different trajectories after the first step."""
    import torch
    from paper_2308_10459_amd import bdem as B
    out = {"k_self": "E_max r_max", "steps": steps}
    for label, opts in (("without", {}), ("with", {"k_self": -1.0})):
        sim = B.Simulator(scene, precision=B.BDEM_PREC_MIXED, **opts)
        sim.autotune([scene.dt])
        rows = []
        for _ in range(steps):
            st = sim.step(scene.dt)
            rows.append({"ms": st["t_ms"][5], "newton": st["newton_iters"], "cg": st["cg_iters"],
                         "broken": st["bonds_broken"], "rc": st["rc"]})
        pairs = len(sim.contact_pairs())
        sim.close()
        torch.cuda.synchronize()
        nw = sum(r["newton"] for r in rows)
        out[label] = {"per_step": rows, "ms_per_newton_iter": sum(r["ms"] for r in rows) / max(nw, 1),
                      "candidate_pairs_last_step": pairs}
        log(f"  {label}: " + ", ".join(f"{r['ms']:.1f} ms / {r['newton']} Newton / {r['cg']} CG" for r in rows))
    return out


def cpu_baseline(target_s=15.0):
    """The FP64 oracle on a bounded sample of the same workload: a 24x24x16
    sub-plate (9,216 particles) built like the ceramic plate, same material,
    velocity, ground and dt.  One oracle step; Newton iterations per second
    scaled to 219,024 particles by the particle ratio (optimistic for the
    oracle: its PCG iteration count would grow with size), and oracle bond
    Hessian evaluations per second (exact per-bond work)."""
    import numpy as np
    from oracle.oracle import Oracle
    from paper_2308_10459_amd import scenes as S
    full_n = 117 * 117 * 16
    sc = S.make_ceramic_plate(nx=24, ny=24, nl=16)
    o = Oracle(sc)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    st = o.step(sc.dt, tol_rel=1e-10, max_newton=20)
    t_step = time.perf_counter() - t0
    # bond Hessian evaluations: energy/gradient/projected Hessian of every bond
    t0 = time.perf_counter()
    reps = 0
    while True:
        o.energy_grad_hess(sc.dt)
        reps += 1
        if time.perf_counter() - t0 > min(5.0, target_s / 3):
            break
    t_egh = (time.perf_counter() - t0) / reps
    iters = max(st["newton_iters"], 1)
    return {
        "value": iters / t_step * sc.n / full_n, "unit": "Newton iters/s", "cores": threads,
        "kind": "oracle",
        "sample": f"one oracle step of a 24x24x16 sub-plate ({sc.n} particles, {sc.nb} bonds): "
                  f"{st['newton_iters']} Newton iterations, {st['cg_iters']} PCG iterations in "
                  f"{t_step:.1f} s, rate scaled by {sc.n}/{full_n} particles",
        "bond_hessian_evals_per_s": sc.nb / t_egh,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="ceramic_plate")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--mixed-only", action="store_true")
    ap.add_argument("--no-solver-comparison", action="store_true")
    ap.add_argument("--batch-steps", type=int, default=3,
                    help="steps of the 64-scene batch (0: skip)")
    ap.add_argument("--midpoint-steps", type=int, default=5,
                    help="steps of the bench workload with the midpoint integrator (0: skip)")
    ap.add_argument("--no-amg", action="store_true",
                    help="skip the multigrid-preconditioned run of the bench workload")
    ap.add_argument("--contact-steps", type=int, default=2,
                    help="steps of the bench workload from its initial state with and without "
                         "element repulsion (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the multi-GPU "
              "path of this method is a design, not a build", file=sys.stderr)
        sys.exit(2)
    from paper_2308_10459_amd import scenes as S
    scene = S.WORKLOADS[args.workload]()
    log(f"workload {scene.name}: n={scene.n} nb={scene.nb} dt={scene.dt}")
    log("mixed path:")
    mixed = run_path(scene, True, args.steps, args.warmup, profile=True)
    fsteps = args.steps if args.fp64_steps is None else args.fp64_steps
    if args.mixed_only:
        fsteps = 0
    fp64 = None
    if fsteps:
        log("fp64 path:")
        fp64 = run_path(scene, False, fsteps, args.warmup, profile=True)
    if args.copy_probe:
        import torch
        src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x 1 GiB device-to-device copies")

    def rates(r, elt, steps):
        if steps == 0:
            return None
        nwt = r["newton"] / r["wall_s"] if r["wall_s"] > 0 and r["newton"] else 0.0
        be = r["alive_bonds"] * r["bond_launch"] / (r["bond_ms"] * 1e-3) if r["bond_ms"] > 0 else 0.0
        spmv_avg_ms = r["spmv_ms"] / max(r["spmv_launch"], 1)
        bytes_spmv = spmv_algorithmic_bytes(scene.n, r["alive_bonds"], elt)
        bond_avg_ms = r["bond_ms"] / max(r["bond_launch"], 1)
        bytes_bond = bond_algorithmic_bytes(scene.n, r["alive_bonds"], elt)
        return dict(newton_iters_per_s=nwt, bond_hessian_evals_per_s=be,
                    bond_hessian_evals_per_wall_s=r["alive_bonds"] * r["newton"] / r["wall_s"],
                    ms_per_step=1e3 * r["wall_s"] / steps,
                    cg_iters_per_newton=r["cg"] / max(r["newton"], 1),
                    ls_backtracks_per_newton=r["ls"] / max(r["newton"], 1),
                    spmv_launches=r["spmv_launch"], spmv_avg_ms=spmv_avg_ms,
                    spmv_gbs=bytes_spmv / (spmv_avg_ms * 1e-3) / 1e9 if spmv_avg_ms > 0 else 0.0,
                    spmv_bytes=bytes_spmv, bond_launches=r["bond_launch"], bond_avg_ms=bond_avg_ms,
                    bond_gbs=bytes_bond / (bond_avg_ms * 1e-3) / 1e9 if bond_avg_ms > 0 else 0.0,
                    bond_bytes=bytes_bond,
                    newton_iters=r["newton"], cg_iters=r["cg"], bonds_broken=r["broken"],
                    alive_bonds=r["alive_bonds"], tuning=r["tuning"])

    rm, rf = rates(mixed, 4, args.steps), rates(fp64, 8, fsteps)
    out = {
        "metric": METRIC,
        "value": rm["newton_iters_per_s"],
        "unit": "Newton iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mixed["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 Hessian/SpMV, f64 state/gradient/reductions",
        "data": "synthetic",
        "config": {"workload": f"{scene.name}: {scene.n} particles, {scene.nb} bonds, E=5e10 Pa, "
                               f"v0=-8 m/s onto the ground, dt={scene.dt}",
                   "parallelism": "single GPU"},
        "bond_hessian_evals_per_s": rm["bond_hessian_evals_per_s"],
        "mixed": rm,
        "fp64": rf,
        "mixed_over_fp64_newton_iters_per_s": (rm["newton_iters_per_s"] / rf["newton_iters_per_s"]
                                               if rf and rf["newton_iters_per_s"] > 0 else None),
        "roofline": {"bound": "hbm", "kernel": "k_spmv<float>", "achieved": rm["spmv_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rm["spmv_gbs"] / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(),
                     "algorithmic_bytes_per_launch": rm["spmv_bytes"]},
    }
    if not args.no_amg:
        log("aggregation multigrid preconditioner (mixed path):")
        out["precond_comparison"] = run_precond_comparison(scene, args.steps, args.warmup)
        out["precond_comparison"]["block_jacobi"] = {
            "newton_iters_per_s": rm["newton_iters_per_s"], "ms_per_step": rm["ms_per_step"],
            "cg_iters_per_newton": rm["cg_iters_per_newton"]}
    if args.midpoint_steps > 0:
        log("midpoint integrator (mixed path):")
        out["integrator_comparison"] = run_integrator_comparison(scene, args.midpoint_steps, args.warmup)
        out["integrator_comparison"]["euler_newton_iters_per_step"] = mixed["newton"] / args.steps
    if args.contact_steps > 0:
        log("element repulsion on (mixed path):")
        out["contact_comparison"] = run_contact_comparison(scene, args.contact_steps)
    if not args.no_solver_comparison:
        log("first- vs second-order manifold optimisation:")
        out["solver_comparison"] = run_solver_comparison()
    if args.batch_steps > 0:
        log("64-scene batch:")
        out["batch"] = run_batch(args.batch_steps, 1)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle):")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
