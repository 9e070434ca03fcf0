"""Seeded synthetic scene generators.

This module only places particles, builds the bond graph and fills in the
material / environment tables.  It holds none of the method's arithmetic
(no rest data, no energies, no derivatives): both the HIP path and the CPU
oracle derive everything else from these raw inputs on their own.

The scenes stand in for the paper's experiments (Section 6, Table 1): a
simple-cubic block, dropping close-packed plates (the paper packs its
elements by hexagonal close packing, Section 3.4), a one-layer sheet that
is pulled apart, and a batch of uneven scenes.  Particle orientations start
at identity unless stated; the rest orientation is always identity.

Conventions shared with the C interface:
  * quaternions are (x, y, z, w) with the scalar last (Appendix A);
  * flags: 0 = free, 1 = fixed, 2 = kinematic (moves with its own velocity);
  * bonds are (i, j) pairs with i < j, sorted, unique, no self pairs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
from scipy.spatial import cKDTree

FREE, FIXED, KINEMATIC = 0, 1, 2


def material(young, poisson=0.3, density=1000.0, sigma_c=0.0, tau_c=0.0,
             stiff_scale=(1.0, 1.0, 1.0, 1.0), shear_mode=0, tension_only=0):
    """One row of the material table.  sigma_c / tau_c <= 0 means unbreakable.
    stiff_scale multiplies (stretch, shear, twist, bend) stiffness."""
    return dict(young=float(young), poisson=float(poisson), density=float(density),
                sigma_c=float(sigma_c), tau_c=float(tau_c),
                stiff_scale=tuple(float(s) for s in stiff_scale),
                shear_mode=int(shear_mode), tension_only=int(tension_only))


@dataclasses.dataclass
class Scene:
    name: str
    pos: np.ndarray          # (n,3) float64
    quat: np.ndarray         # (n,4) float64, scalar last
    vel: np.ndarray          # (n,3)
    qvel: np.ndarray         # (n,4)
    radius: np.ndarray       # (n,)
    pmat: np.ndarray         # (n,) int32 material index
    flags: np.ndarray        # (n,) uint8
    ij: np.ndarray           # (nb,2) int32
    materials: List[Dict]
    gravity: tuple = (0.0, 0.0, -9.81)
    ground_normal: tuple = (0.0, 0.0, 1.0)
    ground_offset: float = 0.0
    k_contact: float = 0.0   # <0: E_max * r_max ; 0: no ground ; >0: value
    k_self: float = 0.0      # element repulsion: <0: E_max * r_max ; 0: off ; >0: value
    contact_margin: float = -1.0   # candidate reach beyond r_i + r_j (<0: r_max)
    mu_s: float = 0.0        # sliding friction coefficient
    mu_r: float = 0.0        # rolling friction coefficient
    dt: float = 1e-3
    steps: int = 1
    scene_id: Optional[np.ndarray] = None   # (n,) int32, non-decreasing (batches)
    dt_per_scene: Optional[np.ndarray] = None
    bmat: Optional[np.ndarray] = None       # (nb,) int32 or None (= material of i)

    @property
    def n(self):
        return int(self.pos.shape[0])

    @property
    def nb(self):
        return int(self.ij.shape[0])

    @property
    def n_scenes(self):
        return 1 if self.scene_id is None else int(self.scene_id.max()) + 1

    def copy(self):
        return dataclasses.replace(
            self, pos=self.pos.copy(), quat=self.quat.copy(), vel=self.vel.copy(),
            qvel=self.qvel.copy(), radius=self.radius.copy(), pmat=self.pmat.copy(),
            flags=self.flags.copy(), ij=self.ij.copy(),
            materials=[dict(m) for m in self.materials],
            scene_id=None if self.scene_id is None else self.scene_id.copy(),
            dt_per_scene=None if self.dt_per_scene is None else self.dt_per_scene.copy(),
            bmat=None if self.bmat is None else self.bmat.copy())


# ----------------------------------------------------------------------------
# lattices and bond graphs
# ----------------------------------------------------------------------------

def sc_lattice(nx, ny, nz, spacing, origin=(0.0, 0.0, 0.0)):
    """Simple-cubic points, x fastest, then y, then z."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * spacing
    return p + np.asarray(origin, dtype=np.float64)


def fcc111_layers(nx, ny, nlayers, a):
    """Close-packed (111) layers in ABC stacking, nearest-neighbour distance a.
    Within a layer: triangular rows along x; row j is offset by a/2 when odd."""
    h = a * math.sqrt(2.0 / 3.0)
    out = []
    for L in range(nlayers):
        sx, sy = (L % 3) * 0.5 * a, (L % 3) * a / (2.0 * math.sqrt(3.0))
        j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        x = i * a + (j % 2) * 0.5 * a + sx
        y = j * (math.sqrt(3.0) / 2.0) * a + sy
        z = np.full_like(x, L * h, dtype=np.float64)
        out.append(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    return np.concatenate(out, axis=0).astype(np.float64)


def square_sheet(nx, ny, spacing):
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    return np.stack([i.ravel() * spacing, j.ravel() * spacing, np.zeros(nx * ny)],
                    axis=1).astype(np.float64)


def _canon_pairs(pairs):
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    lo = np.minimum(pairs[:, 0], pairs[:, 1])
    hi = np.maximum(pairs[:, 0], pairs[:, 1])
    keep = lo != hi
    key = np.unique(lo[keep] * (1 << 32) + hi[keep])
    out = np.stack([key >> 32, key & ((1 << 32) - 1)], axis=1)
    return out.astype(np.int32)


def bonds_cutoff(pos, cutoff):
    """All pairs closer than cutoff."""
    tree = cKDTree(pos)
    pairs = tree.query_pairs(r=cutoff, output_type="ndarray")
    return _canon_pairs(pairs)


def bonds_knn_union(pos, k):
    """Union of each particle's k nearest neighbours (i in kNN(j) or j in kNN(i))."""
    tree = cKDTree(pos)
    _, idx = tree.query(pos, k=k + 1)
    src = np.repeat(np.arange(pos.shape[0]), k)
    dst = idx[:, 1:].ravel()
    return _canon_pairs(np.stack([src, dst], axis=1))


def random_small_rotations(n, max_angle, rng):
    """Unit quaternions exp of a rotation with uniform axis on S^2 and angle U[0, max_angle]."""
    axis = rng.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.uniform(0.0, max_angle, size=n)
    q = np.empty((n, 4))
    q[:, :3] = axis * np.sin(0.5 * ang)[:, None]
    q[:, 3] = np.cos(0.5 * ang)
    return q


def period_estimate(young, radius, density, n_lap):
    """Time-step rule of Section 5.1: T = 2/sqrt(lambda), lambda = (k/m) N with
    k ~ (pi/2) E r and N the largest bond-graph Laplacian eigenvalue.  Used only
    to choose the dt of a generated scene."""
    m = density * 4.0 / 3.0 * math.pi * radius ** 3
    k = 0.5 * math.pi * young * radius
    return 2.0 / math.sqrt(k / m * n_lap)


def _identity(n):
    q = np.zeros((n, 4))
    q[:, 3] = 1.0
    return q


def _scene(name, pos, radius, ij, materials, **kw):
    n = pos.shape[0]
    return Scene(name=name, pos=np.ascontiguousarray(pos, dtype=np.float64),
                 quat=kw.pop("quat", _identity(n)),
                 vel=kw.pop("vel", np.zeros((n, 3))), qvel=kw.pop("qvel", np.zeros((n, 4))),
                 radius=np.broadcast_to(np.asarray(radius, dtype=np.float64), (n,)).copy(),
                 pmat=kw.pop("pmat", np.zeros(n, dtype=np.int32)),
                 flags=kw.pop("flags", np.zeros(n, dtype=np.uint8)),
                 ij=np.ascontiguousarray(ij, dtype=np.int32), materials=materials, **kw)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def make_block(nx=10, ny=10, nz=10, seed=1, rot_angle=1e-3, dt=1e-3, steps=10,
               young=1e7):
    """Plain FP64 workload: simple-cubic block of nx*ny*nz particles, r = 0.01 m,
    spacing 0.02 m, 6-neighbour bonds, E = 1e7 Pa, density 1000, gravity, the
    bottom layer fixed, seeded random initial rotations up to rot_angle rad,
    no contact, no fracture.  (10x10x10: 1000 particles, 2700 bonds.)"""
    a, r = 0.02, 0.01
    pos = sc_lattice(nx, ny, nz, a)
    ij = bonds_cutoff(pos, 1.1 * a)
    flags = np.zeros(pos.shape[0], dtype=np.uint8)
    flags[pos[:, 2] < 0.5 * a] = FIXED
    rng = np.random.Generator(np.random.PCG64(seed))
    quat = random_small_rotations(pos.shape[0], rot_angle, rng)
    return _scene(f"sc_block_{nx}x{ny}x{nz}", pos, r, ij, [material(young)],
                  quat=quat, flags=flags, k_contact=0.0, dt=dt, steps=steps)


def _plate(name, nx, ny, nl, r, seed, young, density, v0, sigma_c, tau_c, dt, steps,
           jitter=0.01, knn=12):
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = fcc111_layers(nx, ny, nl, 2.0 * r)
    pos += rng.uniform(-jitter * r, jitter * r, size=pos.shape)
    pos[:, 2] += r - pos[:, 2].min()          # lowest sphere touches the ground z = 0
    ij = bonds_knn_union(pos, knn)
    vel = np.zeros_like(pos)
    vel[:, 2] = -abs(v0)
    mats = [material(young, 0.3, density, sigma_c, tau_c)]
    return _scene(name, pos, r, ij, mats, vel=vel, k_contact=-1.0, dt=dt, steps=steps)


def make_plate_drop(nx=128, ny=128, nl=2, seed=2, sigma_c=6.5e4, tau_c=2.0e4, dt=1e-3,
                    steps=100):
    """Close-packed plate, 128x128x2 (32768 particles), r = 2.5 mm, 1 % jitter,
    12-nearest-neighbour bond union, E = 1e9, dropping at 5 m/s onto the ground
    plane with penalty contact, bond breaking by stress thresholds.  The
    thresholds sit near the 95th percentiles of the oracle's bond stresses
    after the impact step (sigma: 6.2e4, tau: 1.9e4 Pa), so a few percent of
    the bonds break on impact."""
    return _plate(f"plate_drop_{nx}x{ny}x{nl}", nx, ny, nl, 2.5e-3, seed, 1e9, 1000.0,
                  5.0, sigma_c, tau_c, dt, steps)


def make_ceramic_plate(nx=117, ny=117, nl=16, seed=3, sigma_c=1.3e7, tau_c=5e6,
                       dt=3.5e-5, steps=200):
    """Paper-scale plate: 117x117x16 close-packed layers = 219,024 particles,
    r = 2.5 mm, E = 5e10, density 2400, ~1.36M bonds, dropped at 8 m/s onto
    the ground, dt = 3.5e-5 (Table 1's plate step).  Brittle thresholds near
    the 99th percentiles of the bond stresses after the impact step (sigma:
    1.26e7, tau: 4.9e6 Pa; peaks 4.2e7 and 1.7e7), so about 1 % of the bonds
    break on impact."""
    return _plate(f"ceramic_plate_{nx}x{ny}x{nl}", nx, ny, nl, 2.5e-3, seed, 5e10, 2400.0,
                  8.0, sigma_c, tau_c, dt, steps)


def make_textile(nx=300, ny=300, seed=4, sigma_c=1e8, tau_c=1e8, dt=5e-5, steps=500,
                 pull_speed=2.0, notch=0.1):
    """One-layer sheet, 300x300 square grid (90K particles), spacing 2 mm, r = 1 mm,
    4 axial + 4 diagonal neighbour bonds, E = 1e9, low bending/twisting
    stiffness (x1e-2), no gravity, the x-min and x-max columns pulled apart at
    pull_speed m/s as kinematic particles.  A notch (bonds crossing the middle
    column line over the lowest `notch` fraction of the height are left out)
    seeds the tear: with dt = 5e-5 (about 60 x the period estimate of Section
    5.1, inside the range the paper recommends) the first bonds break at its
    tip after ~60 steps and a crack runs across the sheet over the next ~150."""
    a, r = 2e-3, 1e-3
    pos = square_sheet(nx, ny, a)
    ij = bonds_cutoff(pos, 1.5 * a)
    if notch > 0.0:
        xm = 0.5 * (nx - 1) * a
        yc = notch * (ny - 1) * a
        xi, xj = pos[ij[:, 0], 0], pos[ij[:, 1], 0]
        ymax = np.maximum(pos[ij[:, 0], 1], pos[ij[:, 1], 1])
        cross = (np.minimum(xi, xj) < xm) & (np.maximum(xi, xj) > xm) & (ymax <= yc + 1e-12)
        ij = ij[~cross]
    flags = np.zeros(pos.shape[0], dtype=np.uint8)
    vel = np.zeros_like(pos)
    left = pos[:, 0] < 0.5 * a
    right = pos[:, 0] > (nx - 1.5) * a
    flags[left | right] = KINEMATIC
    vel[left, 0] = -pull_speed
    vel[right, 0] = pull_speed
    mats = [material(1e9, 0.3, 1000.0, sigma_c, tau_c, stiff_scale=(1.0, 1.0, 1e-2, 1e-2))]
    return _scene(f"textile_{nx}x{ny}", pos, r, ij, mats, vel=vel, flags=flags,
                  gravity=(0.0, 0.0, 0.0), k_contact=0.0, dt=dt, steps=steps)


def _batch_member(s, rng, r=5e-3):
    """One scene of the uneven batch: shape cycles box / beam / plate."""
    n_target = int(round(math.exp(rng.uniform(math.log(2000), math.log(50000)))))
    young = math.exp(rng.uniform(math.log(1e6), math.log(1e10)))
    a = 2.0 * r
    shape = ("box", "beam", "plate")[s % 3]
    if shape == "box":
        side = max(2, int(round(n_target ** (1.0 / 3.0))))
        pos = sc_lattice(side, side, side, a, origin=(0.0, 0.0, 1.0))
        ij = bonds_cutoff(pos, 1.1 * a)
        flags = np.zeros(pos.shape[0], dtype=np.uint8)
        flags[pos[:, 2] < 1.0 + 0.5 * a] = FIXED
        vel = np.zeros_like(pos)
        n_lap = 12.0
    elif shape == "beam":
        k = max(2, int(round((n_target / 8.0) ** (1.0 / 3.0))))
        pos = sc_lattice(8 * k, k, k, a, origin=(0.0, 0.0, 1.0))
        ij = bonds_cutoff(pos, 1.1 * a)
        flags = np.zeros(pos.shape[0], dtype=np.uint8)
        flags[pos[:, 0] < 0.5 * a] = FIXED
        vel = np.zeros_like(pos)
        n_lap = 12.0
    else:
        nl = 2 + s % 3
        side = max(4, int(round(math.sqrt(n_target / nl))))
        pos = fcc111_layers(side, side, nl, a)
        pos += rng.uniform(-0.01 * r, 0.01 * r, size=pos.shape)
        pos[:, 2] += r - pos[:, 2].min()
        ij = bonds_knn_union(pos, 12)
        flags = np.zeros(pos.shape[0], dtype=np.uint8)
        vel = np.zeros_like(pos)
        vel[:, 2] = -5.0
        n_lap = 16.0
    dt = 50.0 * period_estimate(young, r, 1000.0, n_lap)
    return shape, pos, ij, flags, vel, young, dt


def make_batch(n_scenes=64, seed0=0, steps=20, r=5e-3):
    """Batch of n_scenes independent scenes with seeded sizes 2K-50K particles
    (boxes, beams, plates), E log-uniform in [1e6, 1e10], each with its own dt
    (50 x the Section 5.1 period).  Concatenated into one particle / bond list
    with non-decreasing scene ids; one material per scene."""
    pos_l, ij_l, fl_l, v_l, sid_l, mats, dts = [], [], [], [], [], [], []
    off = 0
    for s in range(n_scenes):
        rng = np.random.Generator(np.random.PCG64(seed0 + s))
        shape, pos, ij, flags, vel, young, dt = _batch_member(s, rng, r)
        pos_l.append(pos)
        ij_l.append(ij + off)
        fl_l.append(flags)
        v_l.append(vel)
        sid_l.append(np.full(pos.shape[0], s, dtype=np.int32))
        mats.append(material(young, 0.3, 1000.0))
        dts.append(dt)
        off += pos.shape[0]
    pos = np.concatenate(pos_l)
    sid = np.concatenate(sid_l)
    sc = _scene(f"batch_{n_scenes}", pos, r, np.concatenate(ij_l), mats,
                vel=np.concatenate(v_l), flags=np.concatenate(fl_l), pmat=sid.copy(),
                k_contact=-1.0, dt=float(dts[0]), steps=steps)
    sc.scene_id = sid
    sc.dt_per_scene = np.asarray(dts, dtype=np.float64)
    return sc


def subset_scenes(batch: Scene, keep):
    """The given member scenes of a batch, renumbered 0..len(keep)-1."""
    keep = list(keep)
    sel = np.isin(batch.scene_id, keep)
    old = np.nonzero(sel)[0]
    remap = -np.ones(batch.n, dtype=np.int64)
    remap[old] = np.arange(old.size)
    bsel = sel[batch.ij[:, 0]] & sel[batch.ij[:, 1]]
    ij = remap[batch.ij[bsel]].astype(np.int32)
    sid_map = {s: k for k, s in enumerate(keep)}
    sid = np.array([sid_map[s] for s in batch.scene_id[sel]], dtype=np.int32)
    out = batch.copy()
    out.pos, out.quat, out.vel, out.qvel = (batch.pos[sel].copy(), batch.quat[sel].copy(),
                                            batch.vel[sel].copy(), batch.qvel[sel].copy())
    out.radius, out.flags = batch.radius[sel].copy(), batch.flags[sel].copy()
    out.pmat = sid.copy()
    out.materials = [dict(batch.materials[s]) for s in keep]
    out.ij, out.scene_id = ij, sid
    out.dt_per_scene = batch.dt_per_scene[keep].copy()
    out.dt = float(out.dt_per_scene[0])
    return out


WORKLOADS = {
    "sc_block": make_block,
    "plate_drop": make_plate_drop,
    "ceramic_plate": make_ceramic_plate,
    "textile": make_textile,
    "batch": make_batch,
}


# ----------------------------------------------------------------------------
# tiny hand-built systems used by tests
# ----------------------------------------------------------------------------

def make_pair(axis=(1.0, 0.0, 0.0), length=0.02, r=0.01, young=1e7, density=1000.0,
              gravity=(0.0, 0.0, 0.0), **matkw):
    """Two particles bonded along `axis`, at rest."""
    d = np.asarray(axis, dtype=np.float64)
    d /= np.linalg.norm(d)
    pos = np.stack([np.zeros(3), length * d])
    ij = np.array([[0, 1]], dtype=np.int32)
    return _scene("pair", pos, r, ij, [material(young, density=density, **matkw)],
                  gravity=gravity, k_contact=0.0)


def make_chain(n=3, spacing=0.02, r=0.01, young=1e7, gravity=(0.0, 0.0, 0.0), **matkw):
    pos = np.zeros((n, 3))
    pos[:, 0] = np.arange(n) * spacing
    ij = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).astype(np.int32)
    return _scene(f"chain_{n}", pos, r, ij, [material(young, **matkw)], gravity=gravity,
                  k_contact=0.0)


def make_triangle(side=0.02, r=0.01, young=1e7, gravity=(0.0, 0.0, 0.0), **matkw):
    """Three particles bonded pairwise, an equilateral triangle in the xy plane
    centred on the origin, at rest."""
    pos = np.array([[0.0, 0.0, 0.0], [side, 0.0, 0.0], [0.5 * side, 0.5 * math.sqrt(3.0) * side, 0.0]])
    pos -= pos.mean(axis=0)
    ij = np.array([[0, 1], [1, 2], [0, 2]], dtype=np.int32)
    return _scene("triangle", pos, r, ij, [material(young, **matkw)], gravity=gravity,
                  k_contact=0.0)


def perturb_state(sc: Scene, seed, pos_scale, rot_angle, vel_scale=0.0, qvel_scale=0.0):
    """Seeded random displacement / rotation / velocity of a scene's free particles.
    Returns (pos, quat, vel, qvel); quaternions stay unit."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = sc.pos + rng.uniform(-pos_scale, pos_scale, size=sc.pos.shape)
    # a random 4-vector of size ~rot_angle/2 added to q, then renormalised:
    # a seeded small rotation away from the scene's orientation
    quat = sc.quat + rng.uniform(-0.5 * rot_angle, 0.5 * rot_angle, size=sc.quat.shape)
    quat /= np.linalg.norm(quat, axis=1, keepdims=True)
    vel = sc.vel + rng.uniform(-vel_scale, vel_scale, size=sc.vel.shape)
    qvel = sc.qvel + rng.uniform(-qvel_scale, qvel_scale, size=sc.qvel.shape)
    fixed = sc.flags != FREE
    pos[fixed], quat[fixed] = sc.pos[fixed], sc.quat[fixed]
    vel[fixed], qvel[fixed] = sc.vel[fixed], sc.qvel[fixed]
    return pos, quat, vel, qvel
