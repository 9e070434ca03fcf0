"""Shared helpers of the GPU parity tests (test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np

from oracle.oracle import Oracle


# (test, comparison, error, bound) of every bounded comparison made in this
# process; printed in the terminal summary, so that a run's log shows how far
# each result was from its bound even when every test passes
BOUNDS = []


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def record_bound(what, err, bound):
    import os
    test = os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]
    BOUNDS.append((test, what, float(err), float(bound)))


def make_sim(scene, mixed=False, **opts):
    from paper_2308_10459_amd import bdem as B
    prec = B.BDEM_PREC_MIXED if mixed else B.BDEM_PREC_FP64
    return B.Simulator(scene, precision=prec, **opts)


def oracle_for(scene, state=None):
    o = Oracle(scene)
    if state is not None:
        o.set_state(**{k: state[k] for k in ("pos", "quat", "vel", "qvel", "alive") if k in state})
    return o


def subsystem(scene, sample):
    """Scene holding the sampled particles, every bond incident to one of them and
    the other endpoints of those bonds (created at the rest positions).
    Returns (sub_scene, particle index map, bond mask)."""
    sample = np.unique(np.asarray(sample))
    ij = scene.ij
    bmask = np.isin(ij[:, 0], sample) | np.isin(ij[:, 1], sample)
    parts = np.unique(np.concatenate([sample, ij[bmask].ravel()]))
    sub = scene.copy()
    sub.pos, sub.quat = scene.pos[parts].copy(), scene.quat[parts].copy()
    sub.vel, sub.qvel = scene.vel[parts].copy(), scene.qvel[parts].copy()
    sub.radius, sub.pmat, sub.flags = scene.radius[parts].copy(), scene.pmat[parts].copy(), \
        scene.flags[parts].copy()
    sub.ij = np.searchsorted(parts, ij[bmask]).astype(np.int32)
    sub.scene_id = None
    if sub.bmat is not None:
        sub.bmat = scene.bmat[bmask].copy()
    return sub, parts, bmask


def sampled_oracle_egh(scene, state, eval_pos, eval_quat, dt, sample, psd=True, alive=None,
                       midpoint=False):
    """Oracle reduced gradient / diagonal blocks of the sampled particles and the
    off-diagonal blocks of their bonds, at full-system values.  The subsystem
    holds every bond of a sampled particle, so the midpoint form's z_hat of the
    sampled particles is the full system's too."""
    sub, parts, bmask = subsystem(scene, sample)
    o = Oracle(sub)
    st = {k: state[k][parts] for k in ("pos", "quat", "vel", "qvel")}
    if alive is not None:
        st["alive"] = alive[bmask]
    o.set_state(**st)
    _, z, hd, ho = o.energy_grad_hess(dt, eval_pos[parts], eval_quat[parts], psd=psd,
                                      midpoint=midpoint)
    pos_in_sub = np.searchsorted(parts, np.unique(sample))
    return z[pos_in_sub], hd[pos_in_sub], ho, np.nonzero(bmask)[0]


def row_scale(hd, ho, ij, n):
    """Frobenius scale of each block row: max of the diagonal block and the
    off-diagonal blocks touching the particle."""
    s = np.linalg.norm(hd.reshape(n, -1), axis=1)
    if len(ho):
        nb = np.linalg.norm(ho.reshape(len(ho), -1), axis=1)
        np.maximum.at(s, ij[:, 0], nb)
        np.maximum.at(s, ij[:, 1], nb)
    return s


def quat_angle_err(qa, qb):
    """rotation angle between two orientations (sign-insensitive)"""
    sgn = np.where(np.sum(qa * qb, axis=1) < 0, -1.0, 1.0)[:, None]
    chord = np.linalg.norm(qa - sgn * qb, axis=1)
    return 4.0 * np.arcsin(np.clip(0.5 * chord, 0.0, 1.0))
