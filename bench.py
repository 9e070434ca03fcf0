"""Benchmark of one implicit BDEM time step on one MI355X.

Workload: the paper-scale ceramic plate (117x117x16 close-packed layers =
219,024 particles, ~1.36M bonds, E = 5e10 Pa, dropped at 8 m/s onto the
ground, dt = 3.5e-5 s), seeded synthetic input resident in HBM.  A "step" is
one bdem_step: prediction, Newton iterations (bond evaluation, assembly,
PCG preconditioned with the aggregation multigrid of Section 5.3, or with
block-Jacobi under --precond block-jacobi, exp-map line search), velocity
update and fracture test.

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


# committed counter summaries, one per kernel
PROFILES = {"k_spmv<float>": os.path.join(ROOT, "profiles", "spmv_ceramic_plate_219k.md"),
            "k_rows_eval<float>": os.path.join(ROOT, "profiles", "rows_eval_ceramic_plate_219k.md")}


def source_digest(kernel="k_spmv<float>"):
    """sha256 of the kernel's source text: HBM counter figures recorded for one
    digest are stale once it changes.  k_spmv: its template and the SPMV_*
    tiling constants; k_rows_eval: its file and the headers it inlines (bond
    geometry, particle terms) and the ROWS_* tiling constant."""
    import hashlib
    import re
    csrc = os.path.join(ROOT, "paper_2308_10459_amd", "csrc")
    if kernel.startswith("k_rows_eval"):
        text = "".join(open(os.path.join(csrc, f)).read()
                       for f in ("k_rows.hip", "bdem_bond.hpp", "bdem_particle.hpp"))
        text += "".join(ln for ln in open(os.path.join(csrc, "bdem_internal.hpp")) if "ROWS_" in ln)
        return hashlib.sha256(text.encode()).hexdigest()[:16]
    src = open(os.path.join(csrc, "k_solve.hip")).read()
    m = re.search(r"template <typename T, int NT, int U> __global__ __launch_bounds__\([^)]*\) void k_spmv.*?\n}\n",
                  src, re.S)
    consts = [ln for ln in open(os.path.join(csrc, "bdem_internal.hpp")) if "SPMV_" in ln]
    text = (m.group(0) if m else "") + "".join(consts)
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def spmv_source_digest():
    return source_digest("k_spmv<float>")


def recorded_traffic(kernel="k_spmv<float>"):
    """HBM bytes per launch of `kernel` from the committed counter summary, if
    they were taken on the current source of the kernels; else None."""
    import re
    try:
        txt = open(PROFILES[kernel]).read()
    except (OSError, KeyError):
        return None
    pat = r"TRAFFIC kernel=" + re.escape(kernel) + r" digest=(\w+) fetch_bytes=(\d+) write_bytes=(\d+)"
    m = re.search(pat, txt)
    if not m or m.group(1) != source_digest(kernel):
        return None
    return int(m.group(2)) + int(m.group(3))


def recorded_valu(kernel):
    """VALU wave-instructions per launch of `kernel` from its committed counter
    summary (SQ_INSTS_VALU), if taken on the current source; else None."""
    import re
    try:
        txt = open(PROFILES[kernel]).read()
    except (OSError, KeyError):
        return None
    m = re.search(r"VALU kernel=" + re.escape(kernel) + r" digest=(\w+) insts_valu=(\d+)", txt)
    if not m or m.group(1) != source_digest(kernel):
        return None
    return int(m.group(2))


# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4


def spmv_algorithmic_bytes(n, nb_alive, elt):
    """Bytes one SpMV must move at least: every unique block once (one 6x6 per
    bond, the 21 packed values of each diagonal block), the bond's index pair,
    the input vector read once and the output written once (FP64).  Both
    launches of a multigrid PCG iteration (the cycle's fine product and the
    PCG's own) are such products."""
    return nb_alive * 36 * elt + n * 21 * elt + nb_alive * 8 + 2 * 6 * n * 8


def bond_algorithmic_bytes(n, nb_alive, elt, inverse=False):
    """Bytes one bond evaluation must move at least (the K1 figure of the
    measurement plan): the state read once (p, q: 56 B per particle), each
    bond's topology and rest data (i, j, l0, d0: 24 B), the unique Hessian
    blocks written (36 values per bond, 21 per diagonal block) and the FP64
    reduced gradient (48 B per particle).  The row-parallel evaluation also
    writes the block-Jacobi inverse (21 values per particle): inverse=True
    counts it."""
    b = n * 56 + nb_alive * 24 + nb_alive * 36 * elt + n * 21 * elt + n * 48
    return b + (n * 21 * elt if inverse else 0)


def run_path(scene, mixed, steps, warmup, profile, **opts):
    """Warm up, then time `steps` implicit steps in the autotuned launch
    configuration.  With profile, HIP events on the library's stream bracket
    every bond-evaluation launch of the timed steps, and every SpMV launch too
    when the tuned PCG mode issues plain launches; when it replays captured
    graphs (whose launches cannot be bracketed) the SpMV average comes from
    three further steps with plain launches, and the result says so.  PCG
    issues one iteration ahead of its convergence poll; the timings of the one
    iteration issued after convergence (whose kernels return at once) are
    dropped, so the SpMV average covers working launches only."""
    import torch
    from paper_2308_10459_amd import bdem as B
    prec = B.BDEM_PREC_MIXED if mixed else B.BDEM_PREC_FP64
    sim = B.Simulator(scene, precision=prec, **opts)
    tuning = sim.autotune([scene.dt])
    log(f"  autotuned: {tuning}")
    plain = not tuning["use_graph"]
    for k in range(warmup):
        st = sim.step(scene.dt)
        log(f"  warmup {k}: newton {st['newton_iters']} cg {st['cg_iters']} broken {st['bonds_broken']}")
    B.bdem_set_profiling(sim.ctx, (1 if plain else 2) if profile else 0)
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
    tot["spmv_timing"] = "timed steps"
    if profile and not plain:
        B.bdem_set_profiling(sim.ctx, 1)
        for k in range(3):
            st = sim.step(scene.dt)
            tot["spmv_ms"] += st["t_ms"][7]
            tot["spmv_launch"] += B.bdem_profile_counts(sim.ctx)[1]
        tot["spmv_timing"] = ("3 steps after the timed ones with plain launches (the tuned PCG mode "
                              "replays captured graphs)")
    alive = int(sim.get_state()["alive"].sum())
    sim.close()
    tot["wall_s"] = wall
    tot["alive_bonds"] = alive
    tot["tuning"] = tuning
    return tot


def run_batch(steps, warmup, amg=True):
    """The 64-scene batch (992,148 particles, seeded sizes 2K-50K, per-scene
    dt): aggregate particle-steps per second of the mixed path stepping all
    scenes in one batched call, of the FP64 path batched, and of the FP64
    path stepping the scenes one after another (each scene alone), all with
    the headline legs' preconditioner; then the mixed batched call with the
    other preconditioner.  Every handle is autotuned on its own scenes first,
    as in the single-scene runs."""
    import torch
    from paper_2308_10459_amd import bdem as B
    from paper_2308_10459_amd import scenes as S
    sc = S.make_batch()
    pc, other = ((B.BDEM_PRECOND_AMG, B.BDEM_PRECOND_BLOCK_JACOBI) if amg else
                 (B.BDEM_PRECOND_BLOCK_JACOBI, B.BDEM_PRECOND_AMG))
    out = {"workload": f"{sc.name}: {sc.n} particles, {sc.nb} bonds, 64 scenes of 2K-50K particles, "
                       "per-scene dt = 50 x the period estimate", "steps": steps,
           "preconditioner": "aggregation multigrid" if amg else "block-Jacobi (6x6)"}
    other_label = "mixed_batched_block_jacobi" if amg else "mixed_batched_multigrid"
    for label, prec, p in (("mixed_batched", B.BDEM_PREC_MIXED, pc), ("fp64_batched", B.BDEM_PREC_FP64, pc),
                           (other_label, B.BDEM_PREC_MIXED, other)):
        sim = B.Simulator(sc, precision=prec, preconditioner=p)
        tuning = sim.autotune(sc.dt_per_scene)
        log(f"  batch {label} autotuned: {tuning}")
        if label == "mixed_batched":
            # the batched SpMV's roofline: the autotuner times the tuned SpMV
            # shape with every scene active (back-to-back launches on the
            # batch's initial matrix, all bonds alive)
            nbytes = spmv_algorithmic_bytes(sc.n, sc.nb, 4)
            us = tuning["spmv_us"]
            out["roofline_spmv"] = {
                "bound": "hbm", "kernel": "k_spmv<float> (all 64 scenes in one launch)",
                "achieved": nbytes / (us * 1e-6) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "launch_us": us,
                "algorithmic_bytes_per_launch": nbytes,
                "timing": "autotuner: mean of back-to-back launches, every scene active"}
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
        sim = B.Simulator(m, precision=B.BDEM_PREC_FP64, preconditioner=pc)
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


def run_precond_comparison(scene, steps, warmup, amg):
    """The bench workload (mixed path, same steps) with the other
    preconditioner than the headline legs' (6x6 block-Jacobi, or the
    aggregation multigrid with which Section 5.3 solves): Newton iterations
    per second, per step and CG iterations per Newton iteration."""
    from paper_2308_10459_amd import bdem as B
    r = run_path(scene, True, steps, warmup, profile=False,
                 preconditioner=B.BDEM_PRECOND_AMG if amg else B.BDEM_PRECOND_BLOCK_JACOBI)
    return {"preconditioner": "aggregation multigrid" if amg else "block-Jacobi (6x6)",
            "steps": steps, "warmup": warmup,
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


def _omp_threads(n=None):
    """OpenMP threads of this process (the oracle's runtime); with n, set them."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cg_per_newton=None):
    """The FP64 oracle on the bench workload itself (the 219,024-particle
    plate, its own initial state), on the host cores:
      * one Newton iteration of the oracle's Algorithm 3 step (its evaluation
        with the eigen-clamped Hessian, PCG with the Section 5.3 forcing
        min(0.5, sqrt|grad f|), line search): the step limited to one
        iteration, minus the closing evaluation of the new iterate, timed
        separately;
      * one evaluation (energy, gradient, projected Hessian of every bond) at
        all threads and at one thread (the oracle parallelises its bond and
        particle loops; its PCG is sequential);
      * 20 PCG iterations on that Hessian, for the seconds per iteration.
    value: Newton iterations per second of the first iteration of the impact
    step (the oracle's first PCG solve stops at half the residual, so few
    iterations); modelled_at_bench_cg_per_newton: one evaluation plus the GPU
    run's CG iterations per Newton iteration at the measured cost each."""
    import numpy as np
    from oracle.oracle import Oracle, lib
    from paper_2308_10459_amd import scenes as S
    lib()
    threads = _omp_threads()
    sc = S.make_ceramic_plate()
    o = Oracle(sc)
    t0 = time.perf_counter()
    phi, z, hd, ho = o.energy_grad_hess(sc.dt)
    t_eval = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, it, _ = o.pcg(hd, ho, -z, rtol=0.0, max_iter=20)
    t_cg = (time.perf_counter() - t0) / max(it, 1)
    del hd, ho
    t0 = time.perf_counter()
    st = o.step(sc.dt, max_newton=1, tol_rel=1e-8, cg_rtol=0.5, cg_forcing=1, break_bonds=0)
    t_step = time.perf_counter() - t0
    t_iter = max(t_step - t_eval, 1e-9)
    t_eval1 = None
    if threads and threads > 1:
        _omp_threads(1)
        try:
            t0 = time.perf_counter()
            o.energy_grad_hess(sc.dt, hess=True)
            t_eval1 = time.perf_counter() - t0
        finally:
            _omp_threads(threads)
    nb = sc.nb
    out = {
        "value": 1.0 / t_iter, "unit": "Newton iters/s", "cores": threads, "kind": "oracle",
        "cpu_model": _cpu_model(),
        "sample": (f"the bench workload itself ({sc.n} particles, {nb} bonds): the first Newton "
                   f"iteration of the oracle's impact step ({st['cg_iters']} PCG iterations, forcing "
                   f"min(0.5, sqrt|grad f|)) in {t_iter:.1f} s = step limited to one iteration "
                   f"({t_step:.1f} s) minus one evaluation ({t_eval:.1f} s)"),
        "seconds_per_evaluation": t_eval,
        "seconds_per_pcg_iteration": t_cg,
        "bond_hessian_evals_per_s": nb / t_eval,
    }
    if t_eval1 is not None:
        out["seconds_per_evaluation_1_thread"] = t_eval1
        out["bond_hessian_evals_per_s_1_thread"] = nb / t_eval1
    if cg_per_newton:
        out["modelled_at_bench_cg_per_newton"] = {
            "cg_per_newton": cg_per_newton,
            "newton_iters_per_s": 1.0 / (t_eval + cg_per_newton * t_cg)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="ceramic_plate")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--mixed-only", action="store_true")
    ap.add_argument("--no-solver-comparison", action="store_true")
    ap.add_argument("--no-hessian-comparison", action="store_true",
                    help="skip the run with eigen-clamped bond Hessians")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the 64-scene batch (0: skip)")
    ap.add_argument("--midpoint-steps", type=int, default=5,
                    help="steps of the bench workload with the midpoint integrator (0: skip)")
    ap.add_argument("--precond", choices=("amg", "block-jacobi"), default="amg",
                    help="preconditioner of the headline legs (the comparison leg runs the other)")
    ap.add_argument("--no-precond-comparison", "--no-amg", dest="no_precond_comparison",
                    action="store_true",
                    help="skip the run of the bench workload with the other preconditioner")
    ap.add_argument("--contact-steps", type=int, default=2,
                    help="steps of the bench workload from its initial state with and without "
                         "element repulsion (0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}); the multi-GPU "
              "path of this method is a design, not a build", file=sys.stderr)
        sys.exit(2)
    from paper_2308_10459_amd import bdem as B
    from paper_2308_10459_amd import scenes as S
    scene = S.WORKLOADS[args.workload]()
    log(f"workload {scene.name}: n={scene.n} nb={scene.nb} dt={scene.dt}")
    # the headline legs: Section 5.3's multigrid-preconditioned CG by default
    head_amg = args.precond == "amg"
    amg = dict(preconditioner=B.BDEM_PRECOND_AMG if head_amg else B.BDEM_PRECOND_BLOCK_JACOBI)
    log(f"mixed path (Gauss-Newton bond Hessians, {args.precond} PCG):")
    mixed = run_path(scene, True, args.steps, args.warmup, profile=True, **amg)
    fsteps = args.steps if args.fp64_steps is None else args.fp64_steps
    if args.mixed_only:
        fsteps = 0
    fp64 = None
    if fsteps:
        log("fp64 path:")
        fp64 = run_path(scene, False, fsteps, args.warmup, profile=True, **amg)
    eig = None
    if not args.no_hessian_comparison:
        log("mixed path, eigen-clamped bond Hessians:")
        eig = run_path(scene, True, args.steps, args.warmup, profile=True,
                       hessian=B.BDEM_HESS_EIGEN_CLAMP, **amg)
    if args.copy_probe:
        import torch
        src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x 1 GiB device-to-device copies")

    def rates(r, elt, steps, rows):
        if steps == 0 or r is None:
            return None
        nwt = r["newton"] / r["wall_s"] if r["wall_s"] > 0 and r["newton"] else 0.0
        be = r["alive_bonds"] * r["bond_launch"] / (r["bond_ms"] * 1e-3) if r["bond_ms"] > 0 else 0.0
        spmv_avg_ms = r["spmv_ms"] / max(r["spmv_launch"], 1)
        bytes_spmv = spmv_algorithmic_bytes(scene.n, r["alive_bonds"], elt)
        bond_avg_ms = r["bond_ms"] / max(r["bond_launch"], 1)
        bytes_bond = bond_algorithmic_bytes(scene.n, r["alive_bonds"], elt, inverse=rows)
        return dict(newton_iters_per_s=nwt, bond_hessian_evals_per_s=be,
                    bond_hessian_evals_per_wall_s=r["alive_bonds"] * r["newton"] / r["wall_s"],
                    ms_per_step=1e3 * r["wall_s"] / steps,
                    newton_iters_per_step=r["newton"] / steps,
                    cg_iters_per_newton=r["cg"] / max(r["newton"], 1),
                    ls_backtracks_per_newton=r["ls"] / max(r["newton"], 1),
                    spmv_launches=r["spmv_launch"], spmv_avg_ms=spmv_avg_ms,
                    spmv_gbs=bytes_spmv / (spmv_avg_ms * 1e-3) / 1e9 if spmv_avg_ms > 0 else 0.0,
                    spmv_bytes=bytes_spmv, spmv_timing=r["spmv_timing"],
                    bond_kernels=("k_rows_eval (row-parallel, Gauss-Newton blocks, assembly and "
                                  "block-Jacobi inverse)" if rows else
                                  "k_bond_eval + k_bond_project (bond-parallel, eigen-clamp)"),
                    bond_launches=r["bond_launch"], bond_avg_ms=bond_avg_ms,
                    bond_gbs=bytes_bond / (bond_avg_ms * 1e-3) / 1e9 if bond_avg_ms > 0 else 0.0,
                    bond_bytes=bytes_bond,
                    newton_iters=r["newton"], cg_iters=r["cg"], bonds_broken=r["broken"],
                    alive_bonds=r["alive_bonds"], tuning=r["tuning"])

    rm, rf = rates(mixed, 4, args.steps, True), rates(fp64, 8, fsteps, True)
    re_ = rates(eig, 4, args.steps, False)
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
                   "parallelism": "single GPU",
                   "hessian": "Gauss-Newton bond Hessians (PSD by construction)",
                   "preconditioner": ("aggregation multigrid V(1,1) cycle (PCG, Section 5.3)" if head_amg
                                      else "block-Jacobi (6x6)")},
        "bond_hessian_evals_per_s": rm["bond_hessian_evals_per_s"],
        "mixed": rm,
        "fp64": rf,
        "mixed_over_fp64_newton_iters_per_s": (rm["newton_iters_per_s"] / rf["newton_iters_per_s"]
                                               if rf and rf["newton_iters_per_s"] > 0 else None),
        "mixed_over_fp64_ms_per_step": (rf["ms_per_step"] / rm["ms_per_step"] if rf else None),
        "roofline": {"bound": "hbm",
                     "kernel": ("k_spmv<float> (every launch: the multigrid cycle's and the PCG's)"
                                if head_amg else "k_spmv<float>"),
                     "achieved": rm["spmv_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rm["spmv_gbs"] / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(),
                     "algorithmic_bytes_per_launch": rm["spmv_bytes"]},
        "roofline_bond_eval": {"bound": "hbm", "kernel": "k_rows_eval<float>",
                               "achieved": rm["bond_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": rm["bond_gbs"] / HBM_PEAK_GBS,
                               "traffic": recorded_traffic("k_rows_eval<float>"),
                               "algorithmic_bytes_per_launch": rm["bond_bytes"]},
    }
    valu = recorded_valu("k_rows_eval<float>")
    if valu and rm["bond_avg_ms"] > 0:
        rate = valu / (rm["bond_avg_ms"] * 1e-3)
        out["roofline_bond_eval"]["valu_issue"] = {
            "insts_valu_per_launch": valu, "achieved": rate, "peak": VALU_ISSUE_PEAK,
            "unit": "wave64 VALU instructions/s", "frac": rate / VALU_ISSUE_PEAK}
    if re_:
        out["hessian_comparison"] = {
            "hessian": "eigen-clamped exact bond Hessians (bond-parallel evaluation + projection)",
            **{k: re_[k] for k in ("newton_iters_per_s", "ms_per_step", "newton_iters_per_step",
                                   "cg_iters_per_newton", "bond_avg_ms", "bond_gbs",
                                   "bond_hessian_evals_per_s", "bond_kernels")}}
    if not args.no_precond_comparison:
        log("other preconditioner (mixed path):")
        out["precond_comparison"] = run_precond_comparison(scene, args.steps, args.warmup, not head_amg)
        out["precond_comparison"]["headline"] = {
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
        out["batch"] = run_batch(args.batch_steps, 1, amg=head_amg)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle):")
        out["cpu_baseline"] = cpu_baseline(cg_per_newton=rm["cg_iters_per_newton"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
