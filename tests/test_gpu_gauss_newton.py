"""The Gauss-Newton form of the bond Hessians (bdem_options.hessian =
BDEM_HESS_GAUSS_NEWTON, the PSD matrix the Newton steps solve with by
default; Section 5.2 asks only that the matrix be positive semi-definite)
against the oracle's exact reduced Hessian (Sections 4.1-4.2):

  * at a rigidly moved rest lattice every term the form drops vanishes
    (shear residual, bend/twist moment, Weingarten share, stretch below rest
    length), so it must equal the oracle's unprojected Hessian;
  * at perturbed states it must be symmetric positive semi-definite, with the
    objective and reduced gradient (computed exactly) equal to the oracle's;
  * the terms it drops are first order in the strain: the difference from the
    exact Hessian must shrink in proportion to the perturbation amplitude.

Whole steps with the Gauss-Newton form are checked against the oracle's
fixed points by the step tests of test_gpu_parity.py (it is the default),
and with the eigen-clamp there too (parametrised)."""
import numpy as np
import pytest

from paper_2308_10459_amd import scenes as S
from tests.gpu_helpers import log, make_sim, oracle_for, record_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2308_10459_amd import bdem
    return bdem


def _full(hd, ho, ij, n, alive=None):
    H = np.zeros((6 * n, 6 * n))
    for i in range(n):
        H[6 * i:6 * i + 6, 6 * i:6 * i + 6] = hd[i]
    for b, (i, j) in enumerate(ij):
        if alive is not None and not alive[b]:
            continue
        H[6 * i:6 * i + 6, 6 * j:6 * j + 6] += ho[b]
        H[6 * j:6 * j + 6, 6 * i:6 * i + 6] += ho[b].T
    return H


def _rotation(axis, angle):
    axis = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K, \
        np.concatenate([np.sin(angle / 2) * axis, [np.cos(angle / 2)]])


def _qmul(a, b):
    av, aw = a[..., :3], a[..., 3:]
    bv, bw = b[..., :3], b[..., 3:]
    v = aw * bv + bw * av + np.cross(av, bv)
    w = aw * bw - np.sum(av * bv, axis=-1, keepdims=True)
    return np.concatenate([v, w], axis=-1)


def _gn_what(B):
    return B.BDEM_EGH_E | B.BDEM_EGH_G | B.BDEM_EGH_H | B.BDEM_EGH_GN


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("ground", [False, True])
def test_gauss_newton_equals_exact_hessian_at_rest(B, mixed, ground):
    """Rest lattice moved rigidly (rotation by 0.7 rad about a skew axis plus a
    translation): V = 0 and every dropped term vanishes."""
    sc = S.make_block(nx=5, ny=4, nz=3, rot_angle=0.0)
    sc.gravity = (0.0, 0.0, 0.0)
    R, qr = _rotation([1.0, -2.0, 0.5], 0.7)
    pos = sc.pos @ R.T + np.array([0.1, -0.2, 0.3])
    quat = _qmul(np.broadcast_to(qr, sc.quat.shape), sc.quat)
    if ground:
        sc.k_contact = -1.0
        sc.ground_offset = pos[:, 2].min() - 0.01 + 2e-4   # the lowest spheres penetrate
    st = dict(pos=pos, quat=quat, vel=np.zeros_like(pos), qvel=np.zeros_like(quat))
    o = oracle_for(sc, st)
    phio, zo, hdo, hoo = o.energy_grad_hess(1e-3, psd=False)
    sim = make_sim(sc, mixed=mixed)
    sim.set_state(**st)
    phi, z, hd, ho = sim.energy_grad_hess(1e-3, _gn_what(B))
    sim.close()
    H, Ho = _full(hd, ho, sc.ij, sc.n), _full(hdo, hoo, sc.ij, sc.n)
    err = np.abs(H - Ho).max() / np.abs(Ho).max()
    tol = 1e-6 if mixed else 1e-12
    log(f"[gn at rest] mixed={mixed} ground={ground}: max |H_gn - H_exact| / max |H| = {err:.2e}")
    record_bound(f"Gauss-Newton vs exact Hessian at a rigidly moved rest state, mixed={mixed} ground={ground}",
                 err, tol)
    assert err <= tol
    assert abs(phi - phio) <= 1e-12 * max(abs(phio), 1e-300) + 1e-18


@pytest.mark.parametrize("mixed", [False, True])
def test_gauss_newton_is_psd_with_exact_gradient(B, mixed):
    """Perturbed states of a free block (positions 2e-4 m, rotations 0.03 rad,
    compressed and stretched bonds, ground contact) with dt = 1 s, where the
    inertia term (m/dt^2) no longer hides the bond Hessians: the exact
    reduced Hessian is indefinite, the Gauss-Newton matrix is symmetric and
    positive semi-definite, and the objective and reduced gradient (which do
    not depend on the Hessian form) equal the oracle's."""
    dt = 1.0
    indefinite = []
    for seed in (11, 12, 13):
        sc = S.make_block(nx=5, ny=4, nz=3, rot_angle=0.02)
        sc.flags[:] = 0
        sc.gravity = (0.0, 0.0, 0.0)
        sc.k_contact = -1.0
        sc.ground_offset = 0.01 + 2e-4
        pos, quat, _, _ = S.perturb_state(sc, seed, 2e-4, 0.03)
        st = dict(pos=pos, quat=quat, vel=np.zeros_like(pos), qvel=np.zeros_like(quat))
        o = oracle_for(sc, st)
        phio, zo, hdo, hoo = o.energy_grad_hess(dt, psd=False)
        sim = make_sim(sc, mixed=mixed)
        sim.set_state(**st)
        phi, z, hd, ho = sim.energy_grad_hess(dt, _gn_what(B))
        sim.close()
        H = _full(hd, ho, sc.ij, sc.n)
        Hx = _full(hdo, hoo, sc.ij, sc.n)
        ev = np.linalg.eigvalsh(0.5 * (H + H.T))
        ex = np.linalg.eigvalsh(Hx)
        scale = np.abs(H).max()
        log(f"[gn psd] seed {seed} mixed={mixed}: min eig {ev.min():.3e} (exact Hessian's {ex.min():.3e}), "
            f"scale {scale:.3e}")
        assert np.abs(H - H.T).max() <= 1e-14 * scale
        # PSD up to the rounding of the block values (FP32 blocks on the mixed path)
        tol = (1e-6 if mixed else 1e-12) * scale
        record_bound(f"Gauss-Newton Hessian, most negative eigenvalue / scale, seed {seed} mixed={mixed}",
                     max(-ev.min(), 0.0) / scale, tol / scale)
        assert ev.min() >= -tol
        indefinite.append(ex.min() < -1e-8 * scale)
        assert abs(phi - phio) <= 1e-12 * abs(phio)
        assert np.abs(z - zo).max() <= 1e-11 * np.abs(zo).max()
    # at least one of the states makes the exact Hessian indefinite
    assert any(indefinite)


def test_gauss_newton_differs_by_first_order_terms(B):
    """The dropped terms are proportional to the strain: scaling the
    perturbation of a rest lattice by 1/4 scales |H_gn - H_exact| by about
    1/4 (a term that did not vanish with the strain, e.g. a wrong Jacobian,
    would leave the difference flat; a missing first-order term of the exact
    form would show as a difference that does not vanish at rest)."""
    sc = S.make_block(nx=4, ny=3, nz=3, rot_angle=0.0)
    sc.gravity = (0.0, 0.0, 0.0)
    diffs = []
    for amp in (1.0, 0.25, 0.0625):
        pos, quat, _, _ = S.perturb_state(sc, 7, 2e-4 * amp, 0.02 * amp)
        st = dict(pos=pos, quat=quat, vel=np.zeros_like(pos), qvel=np.zeros_like(quat))
        o = oracle_for(sc, st)
        _, _, hdo, hoo = o.energy_grad_hess(1e-3, psd=False, hess=True)
        sim = make_sim(sc, mixed=False)
        sim.set_state(**st)
        _, _, hd, ho = sim.energy_grad_hess(1e-3, _gn_what(B))
        sim.close()
        H, Hx = _full(hd, ho, sc.ij, sc.n), _full(hdo, hoo, sc.ij, sc.n)
        # the inertia diagonal cancels in the difference; scale by the bond stiffness part
        Hb = Hx - np.diag(np.diag(Hx))
        diffs.append(np.abs(H - Hx).max() / np.abs(Hb).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    log(f"[gn first order] relative differences {diffs}, ratios {r1:.2f} {r2:.2f}")
    assert diffs[0] > 1e-6
    assert 3.0 <= r1 <= 5.3 and 3.0 <= r2 <= 5.3
