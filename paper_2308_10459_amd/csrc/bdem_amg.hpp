// Aggregation multigrid preconditioner for the block-CSR reduced Hessian
// (Section 5.3 solves with AMG-PCG; the variant is this project's choice).
//
// Aggregates are cells of side h0 = AMG_CELL r_max of the scene, counted
// from the corner of the scene's initial bounding box; a coarser level groups the
// cells of the level below by doubling the side.  The hierarchy (which nodes
// belong together, every coarse sparsity pattern and the list of fine blocks
// that sum into each coarse block) is built once on the host at create; the
// numbers are recomputed on the device at the first Newton iteration of each
// step (or at every one, bdem_options.amg_refresh = 0):
//   P_i = [[I, -[x_i - c_a]x], [0, S_i]]  (rigid-body modes t, w of the
//         aggregate a: dp = t + w x (x_i - c_a), y = S_i w; S_i = 1/2 R(q_i)^T
//         for particles, I above), zero for particles that are not unknowns;
//   A_{l+1} = P^T A_l P (Galerkin), identity on nodes without unknowns;
//   smoothing: omega = 0.9 block Jacobi before and after the coarse
//   correction; an exact dense solve per scene on the last level (at most
//   AMG_COARSE_MAX nodes per scene, in LDS).
// The fine level's post-smoothing needs H t for t = t0 + P e (e the level-1
// correction).  It is formed as H t0 (the cycle's first fine product) plus
// (H P) e: the fine coupling H P, one 6x6 block per fine row and level-1
// aggregate that the row's blocks reach (about 2.7 per row on close-packed
// solids against ~13 Hessian blocks per row), is recomputed whenever the
// Hessian changes, so the cycle runs one fine product instead of two.
#pragma once
#include <cstdint>
#include <vector>

#include "bdem_internal.hpp"

namespace bdem {

// cell side in units of the largest radius: 8 r_max holds about 4 x 4 x 4
// lattice sites of a close-packed solid.  On the 219K plate cells of 4, 5, 6
// and 8 r_max all need ~22.6 CG iterations per Newton iteration, and the
// larger cells make every level smaller (8 r_max fastest; past 10 r_max the
// first level's restriction and Galerkin sums grow long)
constexpr double AMG_CELL = 8.0;
constexpr int AMG_COARSE_MAX = 16;
constexpr double AMG_OMEGA = 0.9;
// the tail: the first level Lt at which every scene has at most
// AMG_DENSE_MAX nodes.  Everything the cycle does from that level's b on
// (its pre- and post-smoothing, the coarser levels, the dense solve) is
// linear in b: one symmetric matrix N per scene, formed at setup from
// N_L = A_L^-1 and N_l = S + (I - S A)(S + P N_{l+1} P^T (I - A S)),
// S = omega D^-1 of level l.  Per PCG iteration the tail is e = N b,
// AMG_DENSE_NODES tail nodes per workgroup, prolonged one level down.
constexpr int AMG_DENSE_MAX = 64;
constexpr int AMG_DENSE_NODES = 2;

// device view of one coarse level (level >= 1)
struct AmgLevel {
  int n = 0, nslots = 0;
  int *row_ptr = nullptr, *col = nullptr, *slot_row = nullptr, *dslot = nullptr;
  void *val = nullptr;              // 36 T per slot (rows of the row node)
  void *dinv = nullptr;             // 36 T per node
  int *gptr = nullptr, *gsrc = nullptr;   // contributions per slot, sources in the finer level
  int *mbeg = nullptr, *mlist = nullptr;  // children (finer-level nodes) of each node
  int *active = nullptr, *scene = nullptr;
  double *cen = nullptr;            // 3 per node
  double *pd = nullptr;             // 3 per node: x_node - c_parent (towards the next level)
  int *parent = nullptr;            // node of the next level
  double *b = nullptr, *t = nullptr, *e = nullptr;   // 6 per node
};

// device view of the whole hierarchy
struct AmgDev {
  int L = 0;                        // coarse levels (>= 1)
  int Lt = 0;                       // the tail's level (1 <= Lt <= L)
  int tmax[16] = {};                // most nodes of a scene on each tail level Lt..L
  int *tbeg = nullptr;              // (L - Lt + 1) x (n_scenes + 1): node range per scene on the
                                    // tail levels, level l at (l - Lt) * (n_scenes + 1)
  int64_t *noff = nullptr;          // n_scenes + 1: offset of the scene's (6 n_Lt)^2 tail matrix
  void *nmat = nullptr;             // the tail matrices N (T)
  double *nwork = nullptr;          // 4 x the tail matrices' size: setup work (FP64), per scene
                                    // four slots of (6 n_Lt)^2 at 4 noff[s]
  // fine level (particles, internal order)
  int *slot_row0 = nullptr;         // row of each fine off-diagonal slot
  int *parent0 = nullptr;           // level-1 node of each particle (-1: padding)
  void *pd0 = nullptr;              // 12 T per particle: x_i - c_a (3), S_i (9)
  double *t0 = nullptr, *r0 = nullptr;   // 6 per particle
  const AmgLevel *lv = nullptr;     // device array lv[0..L] (lv[0] unused)
  // fine coupling H P: per fine row its level-1 aggregates in ascending order
  // (hp_ptr over rows, hp_agg per entry, 36 T per entry, row-major); per
  // row the entry its diagonal block adds to (hp_self, -1: none), first;
  // per entry its off-diagonal blocks, in slot order (hp_gptr; per source
  // hp_src: the slot's block code, (bond block << 1) | transposed; hp_col:
  // the block's column j)
  int nhp = 0;
  int *hp_ptr = nullptr, *hp_agg = nullptr, *hp_self = nullptr, *hp_gptr = nullptr, *hp_src = nullptr,
      *hp_col = nullptr;
  void *hp_val = nullptr;
  // coarsest level: dense inverse per scene
  int *cbeg = nullptr;              // n_scenes + 1: node range per scene on level L
  int64_t *coff = nullptr;          // n_scenes: offset of the scene's (6m)^2 block
  double *cmat = nullptr;           // dense operator, then its inverse
  double *cwork = nullptr;          // Gauss-Jordan work
};

// host-side symbolic hierarchy
struct AmgHostLevel {
  int n = 0;
  std::vector<int> row_ptr, col, slot_row, dslot, gptr, gsrc, mbeg, mlist, active, scene, parent;
};
struct AmgHost {
  int L = 0;
  int Lt = 0;
  std::vector<int> tbeg;
  std::vector<int> parent0, slot_row0;
  // fine coupling pattern (AmgDev); hp_gsrc per source: the slot
  std::vector<int> hp_ptr, hp_agg, hp_self, hp_gptr, hp_gsrc;
  std::vector<AmgHostLevel> lv;     // lv[1..L]
  std::vector<int> cbeg;
  std::vector<int64_t> coff;
  int64_t cdense = 0;               // total doubles of the dense blocks
  std::vector<int> tmax;            // per level (Lt..L at index l): most nodes of a scene
  std::vector<int64_t> noff;        // n_scenes + 1 (tail matrices)
};

// Morton (Z-order) key of an aggregation cell (x, y, z >= 0): the order of
// the nodes of every level within a scene
uint64_t amg_cell_key(int64_t x, int64_t y, int64_t z);

// Builds the symbolic hierarchy.  pos: 4 doubles per internal row (initial
// positions), flags per row (255 = padding), psid per row, scene_pbeg,
// fine CSR (row_ptr over rows, col per slot), per-scene box corner and h0.
void amg_build(int n_pad, int n_scenes, const std::vector<double> &pos4,
               const std::vector<uint8_t> &flags, const std::vector<int> &psid,
               const std::vector<int> &scene_pbeg, const std::vector<int> &row_ptr,
               const std::vector<int> &col, const std::vector<double> &lo3,
               const std::vector<double> &h0, AmgHost &H);

// kernels (k_amg.hip)
// hl: host copy of the level array (sizes for the launches)
void launch_amg_setup(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, bool mixed,
                      hipStream_t s);
// the fine coupling H P from the current Hessian blocks and the prolongator
// of the last setup: after every setup and every Hessian evaluation that
// the cycle will use
void launch_amg_couple(const DevPtrs &d, const AmgDev &a, bool mixed, hipStream_t s);
// t0_ready: the CG update already wrote t0 = omega D^-1 r (DevPtrs::amg_t0);
// the cycle writes u = M^-1 r into d.cs and the (r, u), (r, r) partials of
// each SPMV_ROWS-row block
// mark (optional): called with true before and false after the cycle's
// fine SpMV launch (the profiler's event brackets)
struct SpmvMark {
  void (*fn)(void *arg, bool start) = nullptr;
  void *arg = nullptr;
};
// rev: the block order of the cycle's fine SpMV
void launch_amg_vcycle(const DevPtrs &d, const AmgDev &a, const AmgLevel *hl, int n_scenes, bool mixed,
                       int spmv_variant, bool t0_ready, bool rev, hipStream_t s, SpmvMark mark = SpmvMark());

}  // namespace bdem
