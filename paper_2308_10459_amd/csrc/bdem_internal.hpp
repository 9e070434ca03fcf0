// Internal layout of a bdem_ctx on the device, shared by the host driver and
// the kernel launchers.  Not part of the public ABI.
//
// Layout in HBM (internal order; scenes are padded to multiples of TILE
// particles and TILE bonds so every kernel block belongs to one scene):
//   particles : double4 per particle for p_n, q_n, v_n, qdot_n, p_hat, q_hat,
//               iterate p, q and trial p, q;  double4 (m, c, r, 0) constants;
//               uint8 flags; int scene id.
//   bonds     : int2 (i, j);  double4 (d0, l0);  double4 (k_n, k_t L^2,
//               GJ/l0, EI/l0);  double4 (S, r0/I, r0/J, tension_only);
//               double2 (sigma_c, tau_c); uint8 alive; int2 slot of the bond in rows i and j.
//   Hessian   : diagonal blocks, 21 packed values per particle (T);
//               off-diagonal blocks stored once per bond, 36 values (T), the
//               block (i, j) of the bond's own (i, j) order; the block-CSR
//               pattern has two slots per bond, each naming the bond's block
//               and whether its row reads it transposed; per-slot halves of the diagonal block
//               (21 T) and of the reduced gradient (6 double) written by the
//               bond kernel and summed in a fixed order by the particle kernel.
//   solver    : 6 doubles per particle for z, CG x, r, s (= M^-1 r), p, Ap;
//               block-Jacobi inverse, 21 packed values per particle (T).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bdem {

constexpr int TILE = 256;       // particles / bonds per scene-aligned tile
constexpr int SPMV_ROWS = 32;     // block rows per SpMV workgroup
constexpr int SPMV_CAP = 512;     // slot products held in LDS per pass of an SpMV workgroup (~400 per 32 rows of a close-packed solid)
constexpr int DOT_GROUP = 64;     // SpMV blocks whose (r, u), (r, r) partials one SpMV wavefront merges
constexpr int CMAXC = 32;         // element-repulsion candidates per particle
constexpr int ROWS_RT = 64;       // block rows per workgroup of the row-parallel evaluation

// per-scene control block, device resident; every decision of the Newton /
// PCG / line-search loops is taken on the device from these values
struct SceneCtl {
  double dt, inv_dt2;
  double kc;   // ground penalty stiffness of the scene (0: no ground)
  double gnorm, gnorm0, phi, phi_trial, slope, alpha_ls;
  double rz, rz_new, rr, pAp, alpha, beta, cg_tol;
  double last_move, xmax;
  int newton_active, cg_active, ls_active, ls_accept;
  int newton_it, cg_it, ls_it, status;
  int cg_total, ls_total, nonfinite;
  int ndegen;   // alive bonds with |q_i + q_j| < 1e-6 at the last evaluated iterate
  int unresolved, stall;   // rounding-floor detection (see k_newton_check)
  double gnorm_prev;
  double alpha_prev;       // last accepted line-search step
  double kself;            // element-repulsion stiffness of the scene (0: off)
  double cmargin;          // candidate reach beyond r_i + r_j
  double ccell;            // broad-phase cell size (>= 2 r_max + margin)
};

enum { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_LS_FAILED = 2, ST_NONFINITE = 3 };

struct Params {
  // environment
  double gx, gy, gz;
  double gnx, gny, gnz, gh;
  double newton_tol, newton_rtol, armijo_c, cg_rtol_max;
  int max_newton, max_cg, max_ls;
  int n_scenes;
  int first_order;   // Algorithm 1 instead of Algorithm 2
  int midpoint;      // variational midpoint objective of Section 3.1
  int contact;       // element repulsion enabled in some scene
  double mu_s, mu_r; // friction coefficients (Section 5.4)
};

struct DevPtrs {
  int n_pad, nb_pad, n_slots;
  int one_scene;                     // 1: every row is scene 0 (no scene lookup needed)
  // particles
  double4 *pn, *qn, *vn, *wn;        // state x_n and rates
  double4 *ph, *qh;                  // prediction
  double4 *px, *qx;                  // Newton iterate
  double4 *pt, *qt;                  // line-search trial
  double4 *pconst;                   // (m, c, r, 0)
  uint8_t *flags;                    // FREE / FIXED / KINEMATIC ; 255 = padding
  int *psid;                         // scene id per particle
  int *row_ptr;                      // n_pad + 1, off-diagonal slots per row
  int *col;                          // n_slots: neighbour row of each off-diagonal slot
  int *sblk;                         // n_slots: 2 * bond + (1 when the row is the bond's j end:
                                     // its block is the transpose of the stored one)
  // bonds
  int2 *bij;
  double4 *brest_a, *brest_b, *brest_c;
  double2 *bstrength;
  uint8_t *alive;
  int2 *bslot;
  int *bsid;
  // Hessian / gradient (T = float or double, typed at the launch)
  void *hdiag;   // n_pad * 21
  void *hoff;    // nb_pad * 36: the (i, j) block of every bond (at least 64 bytes per slot)
  void *hhalf;   // n_slots * 21
  void *h9;      // nb_pad * 45: per-bond packed reduced 9x9 before projection
  double *ghalf; // n_slots * 6
  void *dinv;    // n_pad * 21
  double *z;     // 6 n_pad
  // CG
  double *cx, *cr, *cs, *cp, *cAp, *cq;
  double *amg_t0;                     // multigrid only: the CG update writes the cycle's pre-smoothed
                                      // start omega D^-1 r here in place of u (null otherwise)
  // reductions
  double2 *part_a, *part_b, *part_c;  // per-block compensated partials
  double2 *part_ag, *part_cg;         // part_a, part_c merged per DOT_GROUP SpMV blocks (one slot per TILE rows)
  double *part_max;                   // per-block maxima (2 per block)
  int *part_cnt;                      // per-block integer counts
  SceneCtl *ctl;                      // n_scenes
  int *scene_pbeg;                    // n_scenes + 1 (particle index, multiple of TILE)
  int *scene_bbeg;                    // n_scenes + 1 (bond index, multiple of TILE)
  int *counters_ws;                   // 2 slots x 4 ints in the workspace (the counters of a handle
                                      // created in the static scratch, which has no pinned host memory)
  int *counters;                      // device address of 2 slots x 4 ints in mapped pinned host memory
                                      // (or counters_ws):
                                      // [0] newton active, [1] cg active, [2] ls active, [3] degenerate bonds
  int *degenerate;                    // bonds with |q_i + q_j| below the threshold
  // element repulsion (Section 5.4); allocated only when enabled
  int *cand, *ncand;                  // CMAXC candidates per particle (sorted), their count
  int *cact, *nact;                   // overlapping candidates at the last evaluation
  int *gcnt, *gbeg, *gitem;           // broad-phase hash grid: counts, starts, items
  int n_bucket;                       // power of two
  int *cand_over;                     // particles with more than CMAXC candidates
  double2 *part_d;                    // per-tile partial of the repulsion's w.u in PCG
};

// the scene of a row (of a tile: every row of a tile is one scene's); with
// one scene, no load
__device__ __forceinline__ int row_scene(const DevPtrs &d, int row) { return d.one_scene ? 0 : d.psid[row]; }

// ----- launchers (kernels in the .hip files) -----
// bond kernels
void launch_bond_eval(const DevPtrs &d, bool mixed, bool psd, bool hess, bool midpoint,
                      hipStream_t s);
void launch_bond_energy(const DevPtrs &d, bool trial, bool midpoint, hipStream_t s);
void launch_bond_force(const DevPtrs &d, hipStream_t s);
void launch_bond_fracture(const DevPtrs &d, hipStream_t s);
// particle kernels
void launch_predict(const DevPtrs &d, bool write_iterate, hipStream_t s);
void launch_copy_state_to_iterate(const DevPtrs &d, hipStream_t s);
void launch_restart_from_state(const DevPtrs &d, hipStream_t s);
void launch_particle_eval(const DevPtrs &d, const Params &P, bool mixed, bool hess,
                          bool potential_only, hipStream_t s);
// row-parallel evaluation with the Gauss-Newton bond Hessian (gradient,
// diagonal and off-diagonal blocks, block-Jacobi inverse, |z|^2 per ROWS_RT
// rows), and the particle part of the objective at the iterate
void launch_rows_eval(const DevPtrs &d, const Params &P, bool mixed, bool midpoint,
                      bool potential_only, hipStream_t s);
void launch_particle_energy(const DevPtrs &d, const Params &P, bool potential_only, hipStream_t s);
void launch_midpoint_target(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_ls_trial(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_ls_accept(const DevPtrs &d, hipStream_t s);
// element repulsion and friction
void launch_contact_broad_phase(const DevPtrs &d, hipStream_t s);
void launch_contact_spmv(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_contact_trial_energy(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_friction(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_finish_step(const DevPtrs &d, hipStream_t s);
// per-scene decisions
// rows: the iterate was evaluated by the row-parallel kernel (|z|^2 partials
// per ROWS_RT rows; Phi of later iterates is the accepted line-search trial's)
void launch_newton_check(const DevPtrs &d, const Params &P, int first, bool rows, hipStream_t s);
void launch_count_active(const DevPtrs &d, int n_scenes, int slot, hipStream_t s);
void launch_ls_decide(const DevPtrs &d, const Params &P, hipStream_t s);
// PCG
void launch_cg_init(const DevPtrs &d, bool mixed, hipStream_t s);
// dots: SPMV_DOTS_ALL forms the (r, u), (w, u) and (r, r) partials;
// SPMV_DOTS_WU leaves (r, u) and (r, r) to the kernel that produced u (the CG
// update with rdots = true, or the multigrid cycle's last kernel) and
// merges theirs; SPMV_DOTS_NONE writes w only (the cycle's fine product)
enum SpmvDots { SPMV_DOTS_WU = 0, SPMV_DOTS_ALL = 1, SPMV_DOTS_NONE = 2 };
// reverse: workgroups take the row blocks of each XCD's range from its end
// (consecutive products alternate, so that the rows a product reads first
// are the ones the product before read last, still in the caches); the
// results do not depend on it
void launch_spmv(const DevPtrs &d, bool mixed, int variant, hipStream_t s, int dots = SPMV_DOTS_ALL,
                 bool reverse = false);
int spmv_variants();
void spmv_shape(int variant, int *threads, int *trips);
void launch_cg_scalars(const DevPtrs &d, const Params &P, hipStream_t s, bool grouped);
void launch_cg_update(const DevPtrs &d, bool mixed, int variant, hipStream_t s, bool rdots = false);
int update_variants();
int update_rows(int variant);
void launch_cg_slope(const DevPtrs &d, const Params &P, hipStream_t s);
void launch_steepest(const DevPtrs &d, hipStream_t s);

}  // namespace bdem
