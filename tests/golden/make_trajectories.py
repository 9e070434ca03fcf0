"""Writes the stored oracle trajectories the full-size step tests compare with.

    OMP_NUM_THREADS=8 python tests/golden/make_trajectories.py plate_drop
    OMP_NUM_THREADS=8 python tests/golden/make_trajectories.py ceramic_plate

Only the FP64 CPU oracle (`oracle/`) and the seeded scene generators are
called.  Each workload is stepped from its generated initial state with the
oracle's own Algorithm 3 step: Newton run to the FP64 rounding floor
(tol_rel = 0), each linear solve to the relative residual
min(0.5, sqrt|grad f|) of Section 5.3 (the fixed point does not depend on
that choice, only the path), fracture tested after every step (Section 3.3).

Stored for every step k = 1..K of the trajectory:
  * s{k}_pos, s{k}_quat: the oracle's state after step k at a seeded sample
    of particles (`sample`, the same for every step);
  * s{k}_phi: the objective Phi(x_k) of step k at the state Newton stopped at;
  * s{k}_broken: indices of the bonds that broke at the end of step k;
  * s{k}_uncert: indices of the bonds alive before step k whose stresses at
    x_k lie within 1e-3 (relative) of a threshold: there the broken-set
    decision is not decidable from a state known only to the step
    tolerance, and a test compares the decision on every other bond;
  * meta: the oracle's per-step statistics (Newton / PCG iterations, wall
    time, |grad f| before and after) and the options used.
Steps finished so far are kept in a resume file next to the output, so an
interrupted run continues where it stopped.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.oracle import Oracle  # noqa: E402
from paper_2308_10459_amd import scenes as S  # noqa: E402

# workload -> (number of steps stored, sample size)
STEPS = {"ceramic_plate": (10, 2048), "plate_drop": (3, 2048)}
MARGIN = 1e-3
ORACLE_OPTS = dict(tol_rel=0.0, max_newton=300, cg_rtol=0.5, cg_forcing=1)
SAMPLE_SEED = 20230821


def out_path(name):
    return os.path.join(HERE, f"{name}_steps.npz")


def uncertified(o, sc, state_after, alive_before):
    """bonds alive before the step whose stress at the new state is within
    MARGIN (relative) of a threshold"""
    sig, tau = o.stresses(state_after["pos"], state_after["quat"])
    m = sc.materials[0]
    near = np.zeros(sc.nb, dtype=bool)
    if m["sigma_c"] > 0:
        near |= np.abs(sig / m["sigma_c"] - 1.0) < MARGIN
    if m["tau_c"] > 0:
        near |= np.abs(tau / m["tau_c"] - 1.0) < MARGIN
    return np.nonzero(near & (alive_before != 0))[0].astype(np.int32)


def sample_of(sc, size):
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    return np.sort(rng.choice(sc.n, size=size, replace=False)).astype(np.int32)


def main(name):
    nsteps, nsample = STEPS[name]
    sc = getattr(S, "make_" + name)()
    sample = sample_of(sc, nsample)
    resume = out_path(name) + ".partial.npz"
    data = {}
    meta = {"workload": sc.name, "n": sc.n, "nb": sc.nb, "dt": sc.dt, "steps_stored": nsteps,
            "oracle_options": ORACLE_OPTS, "margin": MARGIN, "sample_seed": SAMPLE_SEED,
            "steps": {}, "threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}
    o = Oracle(sc)
    done = 0
    if os.path.exists(resume):
        z = np.load(resume)
        data = {k: z[k] for k in z.files if k != "meta" and not k.startswith("cur_")}
        meta = json.loads(str(z["meta"]))
        done = int(meta["done"])
        o.set_state(pos=z["cur_pos"], quat=z["cur_quat"], vel=z["cur_vel"], qvel=z["cur_qvel"],
                    alive=np.unpackbits(z["cur_alive"])[:sc.nb])
        print(f"resuming after step {done}", flush=True)
    data["sample"] = sample
    for k in range(done + 1, nsteps + 1):
        before = o.get_state()
        t0 = time.time()
        st = o.step(sc.dt, **ORACLE_OPTS)
        wall = time.time() - t0
        after = o.get_state()
        broken = np.nonzero((before["alive"] != 0) & (after["alive"] == 0))[0].astype(np.int32)
        unc = uncertified(o, sc, after, before["alive"])
        meta["steps"][str(k)] = dict(st, wall_s=wall, uncertified=int(len(unc)))
        print(f"step {k}: rc {st['rc']} newton {st['newton_iters']} cg {st['cg_iters']} "
              f"ls {st['ls_backtracks']} |z| {st['grad0']:.3e} -> {st['grad_final']:.3e} "
              f"broken {st['bonds_broken']} uncertified {len(unc)} phi {st['phi']:.15e} "
              f"({wall:.0f} s)", flush=True)
        data[f"s{k}_pos"] = after["pos"][sample]
        data[f"s{k}_quat"] = after["quat"][sample]
        data[f"s{k}_phi"] = np.float64(st["phi"])
        data[f"s{k}_broken"] = broken
        data[f"s{k}_uncert"] = unc
        meta["done"] = k
        np.savez(resume, meta=json.dumps(meta), **data,
                 **{f"cur_{f}": after[f] for f in ("pos", "quat", "vel", "qvel")},
                 cur_alive=np.packbits(after["alive"]))
    meta.pop("done", None)
    np.savez_compressed(out_path(name), meta=json.dumps(meta), **data)
    os.remove(resume)
    print("wrote", out_path(name), flush=True)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "ceramic_plate")
