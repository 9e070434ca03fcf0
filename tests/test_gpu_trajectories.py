"""Full-size workloads stepped from their generated initial state and compared
with the oracle's own trajectory (Algorithm 3 step by step, fracture of
Section 3.3 at the end of every step), stored by
tests/golden/make_trajectories.py, which calls only the oracle:

  * the 219,024-particle ceramic plate (the benchmark workload), steps 1-10,
    on the mixed path the benchmark runs, with either preconditioner;
  * the 32,768-particle plate drop, steps 1-3, on both paths (and with the
    multigrid preconditioner on the mixed one).

Per step: positions and orientations of 2,048 seeded sample particles against
the oracle's (relative to the step's own displacement / rotation at the
sample), the objective Phi(x_k) at the state Newton stopped at, and the broken
bond set bit-exact on every bond whose oracle stress is certified at least
1e-3 (relative) away from both thresholds.  A bond inside that margin may be
decided either way from a state known only to the step tolerance; the run
then carries on with the oracle's decision for it (counted and reported), so
that one undecidable bond does not fork the two trajectories."""
import json
import os

import numpy as np
import pytest

from paper_2308_10459_amd import scenes as S
from tests.gpu_helpers import log, make_sim, quat_angle_err, record_bound

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TIGHT = dict(newton_rtol=0.0, newton_tol=0.0, max_newton=120)


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_10459_amd import bdem
    return bdem


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}_steps.npz")
    assert os.path.exists(path), f"{path} missing (tests/golden/make_trajectories.py {name} writes it)"
    z = np.load(path, allow_pickle=False)
    return z, json.loads(str(z["meta"]))


@pytest.mark.parametrize("name,mixed,precond", [("ceramic_plate", True, "block_jacobi"),
                                                ("ceramic_plate", True, "amg"),
                                                ("plate_drop", True, "block_jacobi"),
                                                ("plate_drop", False, "block_jacobi"),
                                                ("plate_drop", True, "amg")])
def test_full_size_trajectory_matches_the_oracle(B, name, mixed, precond):
    """precond: the PCG's preconditioner (the multigrid one is the benchmark's
    headline configuration); the fixed point of each step does not depend on
    it."""
    z, meta = _golden(name)
    sc = getattr(S, "make_" + name)()
    assert (sc.n, sc.nb, sc.dt) == (meta["n"], meta["nb"], meta["dt"])
    sample = z["sample"]
    nsteps = int(meta["steps_stored"])
    log(f"[trajectory] {name} mixed={mixed} precond={precond}: n={sc.n} nb={sc.nb}, {nsteps} steps, "
        f"{len(sample)} sample particles")
    pc = B.BDEM_PRECOND_AMG if precond == "amg" else B.BDEM_PRECOND_BLOCK_JACOBI
    sim = make_sim(sc, mixed=mixed, preconditioner=pc, **TIGHT)
    tol = 1e-5 if mixed else 1e-9
    ptol = 1e-6 if mixed else 1e-12
    prev_p, prev_q = sc.pos[sample], sc.quat[sample]
    alive = np.ones(sc.nb, dtype=np.uint8)
    adopted = 0
    for k in range(1, nsteps + 1):
        sg = sim.step(sc.dt)
        got = sim.get_state()
        assert sg["rc"] == 0, sg
        # broken set: bit-exact on the certified bonds alive before the step
        broken = np.zeros(sc.nb, dtype=bool)
        broken[z[f"s{k}_broken"]] = True
        cert = alive != 0
        cert[z[f"s{k}_uncert"]] = False
        newly = (alive != 0) & (got["alive"] == 0)
        np.testing.assert_array_equal(newly[cert], broken[cert])
        expect = alive.copy()
        expect[broken] = 0
        diff = int(np.count_nonzero(got["alive"] != expect))
        if diff:
            adopted += diff
            sim.set_state(alive=expect)
        alive = expect
        # sampled state against the oracle's
        ref_p, ref_q = z[f"s{k}_pos"], z[f"s{k}_quat"]
        disp = np.linalg.norm(ref_p - prev_p)
        perr = np.linalg.norm(got["pos"][sample] - ref_p) / disp
        rot = quat_angle_err(ref_q, prev_q)
        qerr = quat_angle_err(got["quat"][sample], ref_q)
        qrel = np.linalg.norm(qerr) / max(np.linalg.norm(rot), 1e-300)
        phi_o = float(z[f"s{k}_phi"])
        eerr = abs(sg["phi"] - phi_o) / abs(phi_o)
        tag = f"{name} mixed={mixed} {precond} step {k}"
        log(f"  step {k}: newton {sg['newton_iters']} cg {sg['cg_iters']} broken {sg['bonds_broken']} "
            f"(oracle {int(broken.sum())}, uncertified {len(z[f's{k}_uncert'])}, adopted {diff}) "
            f"pos {perr:.2e} rot {qrel:.2e} phi {eerr:.2e}")
        record_bound(f"{tag}: sampled positions / displacement", perr, tol)
        record_bound(f"{tag}: sampled rotation error / step rotation", qrel, tol)
        record_bound(f"{tag}: objective at the new state, relative", eerr, ptol)
        assert perr <= tol
        assert qrel <= tol or np.abs(qerr).max() <= 1e-12
        assert eerr <= ptol
        assert np.abs(np.linalg.norm(got["quat"], axis=1) - 1.0).max() <= 4.5e-16
        prev_p, prev_q = ref_p, ref_q
    sim.close()
    log(f"  undecidable bonds taken over from the oracle: {adopted}")
