// Host side of the C ABI declared in include/bdem.h: validation, rest data
// (Section 3.2), the block-sparse pattern of the reduced Hessian, workspace
// layout, and the driver of one implicit step (Algorithm 3 with Algorithm 2
// inside).  Every numeric decision of the Newton / PCG / line-search loops is
// taken by device kernels from per-scene control blocks; the host only polls
// how many scenes are still iterating.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/bdem.h"
#include "bdem_amg.hpp"
#include "bdem_internal.hpp"

using namespace bdem;

namespace {

thread_local std::string g_create_error;

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct Sizes {
  int n = 0, n_pad = 0, n_scenes = 1;
  int64_t nb = 0;
  int nb_pad = 0, n_slots = 0;
  bool mixed = false;
  bool contact = false;   // element repulsion on: candidate lists and hash grid
  int n_bucket = 0;
};

// ordered list of device buffers carved out of one allocation
struct Layout {
  size_t total = 0;
  std::vector<std::pair<void **, size_t>> items;
  void add(void **p, size_t bytes) { items.push_back({p, bytes}); total += align_up(bytes); }
  void bind(char *base) const {
    size_t off = 0;
    for (auto &it : items) {
      *it.first = base + off;
      off += align_up(it.second);
    }
  }
};

void make_layout(const Sizes &S, DevPtrs &d, Layout &L) {
  const size_t np = S.n_pad, nbp = S.nb_pad, ns = std::max(S.n_slots, 1);
  const size_t T = S.mixed ? 4 : 8;
  const size_t ntile_p = np / TILE, ntile_b = std::max<size_t>(nbp / TILE, 1);
  const size_t nspmv = np / SPMV_ROWS;
  const size_t npart = std::max(std::max(ntile_p, ntile_b), nspmv);
  for (double4 **p : {&d.pn, &d.qn, &d.vn, &d.wn, &d.ph, &d.qh, &d.px, &d.qx, &d.pt, &d.qt, &d.pconst})
    L.add(reinterpret_cast<void **>(p), np * sizeof(double4));
  L.add(reinterpret_cast<void **>(&d.flags), np);
  L.add(reinterpret_cast<void **>(&d.psid), np * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.row_ptr), (np + 1) * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.col), ns * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.sblk), ns * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.bij), std::max<size_t>(nbp, 1) * sizeof(int2));
  for (double4 **p : {&d.brest_a, &d.brest_b, &d.brest_c})
    L.add(reinterpret_cast<void **>(p), std::max<size_t>(nbp, 1) * sizeof(double4));
  L.add(reinterpret_cast<void **>(&d.bstrength), std::max<size_t>(nbp, 1) * sizeof(double2));
  L.add(reinterpret_cast<void **>(&d.alive), std::max<size_t>(nbp, 1));
  L.add(reinterpret_cast<void **>(&d.bslot), std::max<size_t>(nbp, 1) * sizeof(int2));
  L.add(reinterpret_cast<void **>(&d.bsid), std::max<size_t>(nbp, 1) * sizeof(int));
  L.add(&d.hdiag, np * 21 * T);
  // one block per bond; k_bond_force also parks 8 doubles per slot here
  L.add(&d.hoff, std::max(std::max<size_t>(nbp, 1) * 36 * T, ns * 8 * sizeof(double)));
  L.add(&d.hhalf, ns * 21 * T);
  L.add(&d.h9, std::max<size_t>(nbp, 1) * 45 * T);
  L.add(reinterpret_cast<void **>(&d.ghalf), ns * 6 * sizeof(double));
  L.add(&d.dinv, np * 21 * T);
  for (double **p : {&d.z, &d.cx, &d.cr, &d.cs, &d.cp, &d.cAp, &d.cq})
    L.add(reinterpret_cast<void **>(p), np * 6 * sizeof(double));
  for (double2 **p : {&d.part_a, &d.part_b, &d.part_c})
    L.add(reinterpret_cast<void **>(p), npart * sizeof(double2));
  L.add(reinterpret_cast<void **>(&d.part_max), 2 * npart * sizeof(double));
  L.add(reinterpret_cast<void **>(&d.part_cnt), npart * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.ctl), S.n_scenes * sizeof(SceneCtl));
  L.add(reinterpret_cast<void **>(&d.scene_pbeg), (S.n_scenes + 1) * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.scene_bbeg), (S.n_scenes + 1) * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.degenerate), sizeof(int));
  L.add(reinterpret_cast<void **>(&d.counters_ws), 8 * sizeof(int));
  const size_t npc = S.contact ? np : 1;
  for (int **p : {&d.cand, &d.cact}) L.add(reinterpret_cast<void **>(p), npc * CMAXC * sizeof(int));
  for (int **p : {&d.ncand, &d.nact, &d.gitem}) L.add(reinterpret_cast<void **>(p), npc * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.gcnt), std::max(S.n_bucket, 1) * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.gbeg), (std::max(S.n_bucket, 1) + 1) * sizeof(int));
  L.add(reinterpret_cast<void **>(&d.cand_over), sizeof(int));
  L.add(reinterpret_cast<void **>(&d.part_d), std::max<size_t>(ntile_p, 1) * sizeof(double2));
  for (double2 **p : {&d.part_ag, &d.part_cg}) L.add(reinterpret_cast<void **>(p), std::max<size_t>(ntile_p, 1) * sizeof(double2));
}

// scene sizes from the particle and bond arrays (no validation beyond what
// sizing needs)
bool scene_sizes(const bdem_particles *p, const bdem_bonds *b, std::vector<int> &pcnt,
                 std::vector<int64_t> &bcnt, std::string &err) {
  const int n = p->n;
  int S = 1;
  if (p->scene) {
    for (int i = 0; i < n; ++i) {
      if (p->scene[i] < 0 || (i > 0 && p->scene[i] < p->scene[i - 1])) {
        err = "scene ids must be non-negative and non-decreasing";
        return false;
      }
    }
    S = p->scene[n - 1] + 1;
  }
  pcnt.assign(S, 0);
  bcnt.assign(S, 0);
  for (int i = 0; i < n; ++i) pcnt[p->scene ? p->scene[i] : 0]++;
  for (int s = 0; s < S; ++s)
    if (pcnt[s] == 0) { err = "empty scene id"; return false; }
  for (int64_t k = 0; k < b->nb; ++k) {
    const int i = b->ij[2 * k], j = b->ij[2 * k + 1];
    if (i < 0 || j < 0 || i >= n || j >= n) { err = "bond index out of range"; return false; }
    const int si = p->scene ? p->scene[i] : 0, sj = p->scene ? p->scene[j] : 0;
    if (si != sj) { err = "bond joins two scenes"; return false; }
    bcnt[si]++;
  }
  return true;
}

Sizes compute_sizes(const std::vector<int> &pcnt, const std::vector<int64_t> &bcnt, int n,
                    int64_t nb, bool mixed) {
  Sizes S;
  S.n = n;
  S.nb = nb;
  S.n_scenes = (int)pcnt.size();
  S.mixed = mixed;
  int64_t np = 0, nbp = 0;
  for (size_t s = 0; s < pcnt.size(); ++s) {
    np += (pcnt[s] + TILE - 1) / TILE * TILE;
    nbp += (bcnt[s] + TILE - 1) / TILE * TILE;
  }
  S.n_pad = (int)np;
  S.nb_pad = (int)nbp;
  S.n_slots = (int)(2 * nb);
  return S;
}

// element repulsion on (bdem_options.k_self != 0): hash-grid size, a power
// of two of at least twice the padded particle count
void enable_contact(Sizes &S, const bdem_options &o) {
  S.contact = o.k_self != 0.0;
  S.n_bucket = 0;
  if (!S.contact) return;
  int nb = 1024;
  while (nb < 2 * S.n_pad) nb <<= 1;
  S.n_bucket = nb;
}

}  // namespace

struct bdem_ctx {
  hipStream_t stream = nullptr;
  void *mem = nullptr;
  bool own_mem = false;
  Sizes S;
  DevPtrs d{};
  Params P{};
  bdem_options opt{};
  std::string err;
  // host copies of the mapping
  std::vector<int> p_int;        // user particle -> internal row
  std::vector<int64_t> b_int;    // user bond -> internal bond
  std::vector<int2> bslot_h;     // internal bond -> slots
  std::vector<int> scene_pbeg, scene_bbeg;
  std::vector<double> scene_kc;  // ground penalty stiffness per scene
  std::vector<double> scene_kself, scene_cmargin, scene_ccell;   // element repulsion per scene
  // pinned host mirrors
  int *h_counters = nullptr;     // 2 polling slots x 4
  // created by bdem_create_in_scratch: workspace = the device's static scratch,
  // counters in the workspace (copied to h_counters_local), host mirrors unpinned
  bool in_scratch = false;       // holds the claim on the device's scratch (set once created)
  bool host_pinned = false;      // h_counters / h_ctl are pinned allocations
  int scratch_dev = -1;
  int h_counters_local[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<SceneCtl> h_ctl_local;
  int prof_cnt[2] = {0, 0};      // profiled launches in the last step (bond, SpMV)
  SceneCtl *h_ctl = nullptr;
  hipEvent_t ev_slot[2] = {nullptr, nullptr};
  // graph of one CG iteration (+ counter copy), one per polling slot
  int spmv_variant = 0, upd_variant = 0;   // launch shapes (see bdem_autotune)
  double tune_us[3] = {0.0, 0.0, 0.0};      // measured SpMV, update, PCG-iteration times
  hipGraphExec_t cg_exec[2] = {nullptr, nullptr};
  hipGraph_t cg_graph[2] = {nullptr, nullptr};
  // profiling: 1 = events around the bond and SpMV kernels, 2 = around the bond kernels only
  int profiling = 0;
  int trace = 0;                 // BDEM_TRACE=1: one line per Newton iteration of scene 0
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;   // (kind, index of start event)
  std::vector<int> ev_iter;     // PCG iteration of each mark (-1: outside the iterations)
  bool spmv_rev = false;        // block order of the next PCG iteration's first SpMV
  int prof_iter = -1;           // the PCG iteration being issued
  // aggregation multigrid preconditioner (bdem_options.preconditioner)
  bool amg = false;
  AmgDev amg_d;
  std::vector<AmgLevel> amg_hl;   // host copy of the level array (device pointers)
  void *amg_mem = nullptr;
};

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t _e = (expr);                                                           \
    if (_e != hipSuccess) {                                                           \
      ctx->err = std::string("HIP error: ") + hipGetErrorString(_e) + " at " #expr;   \
      return BDEM_E_HIP;                                                              \
    }                                                                                 \
  } while (0)

static int fail(bdem_ctx *ctx, int code, const std::string &m) {
  if (ctx) ctx->err = m;
  else g_create_error = m;
  return code;
}

extern "C" void bdem_default_options(bdem_options *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->gravity[2] = -9.81;
  o->ground_normal[2] = 1.0;
  o->k_contact = 0.0;
  o->newton_tol = 0.0;
  o->newton_rtol = 1e-8;
  o->armijo_c = 1e-4;
  o->cg_rtol_max = 0.5;
  o->max_newton = 50;
  o->max_cg = 2000;
  o->max_ls = 30;
  o->precision = BDEM_PREC_FP64;
  o->break_each_step = 1;
  o->cg_chunk = 16;
  o->use_graph = 0;
  o->solver = BDEM_SOLVER_NEWTON;
  o->integrator = BDEM_INTEGRATOR_EULER;
  o->k_self = 0.0;
  o->contact_margin = -1.0;
  o->preconditioner = BDEM_PRECOND_BLOCK_JACOBI;
  o->hessian = BDEM_HESS_GAUSS_NEWTON;
  o->amg_refresh = 1;
}

extern "C" size_t bdem_workspace_bytes(const bdem_particles *p, const bdem_bonds *b,
                                       const bdem_options *opt) {
  if (!p || !b || p->n <= 0 || b->nb < 0 || (b->nb > 0 && !b->ij)) return 0;
  std::vector<int> pcnt;
  std::vector<int64_t> bcnt;
  std::string err;
  if (!scene_sizes(p, b, pcnt, bcnt, err)) return 0;
  bdem_options o;
  if (opt) o = *opt;
  else bdem_default_options(&o);
  Sizes S = compute_sizes(pcnt, bcnt, p->n, b->nb, o.precision == BDEM_PREC_MIXED);
  enable_contact(S, o);
  DevPtrs d{};
  Layout L;
  make_layout(S, d, L);
  return L.total + ALIGN;
}

// ---------------------------------------------------------------------------
// Static scratch of bdem_create_in_scratch: a file-scope device array (every
// GPU the library runs on holds one until the process ends).  Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device with that device current, and is kept
// per device.  One handle per device may live in it at a time.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_BYTES = BDEM_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES == size_t(64) << 20, "64 MiB");
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
static bool g_scratch_used[SCRATCH_MAX_DEVICES] = {};

static void scratch_release(int dev) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  g_scratch_used[dev] = false;
}

static void destroy_resources(bdem_ctx *ctx) {
  for (int k = 0; k < 2; ++k) {
    if (ctx->cg_exec[k]) (void)hipGraphExecDestroy(ctx->cg_exec[k]);
    if (ctx->cg_graph[k]) (void)hipGraphDestroy(ctx->cg_graph[k]);
    if (ctx->ev_slot[k]) (void)hipEventDestroy(ctx->ev_slot[k]);
  }
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->host_pinned) {
    if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
    if (ctx->h_ctl) (void)hipHostFree(ctx->h_ctl);
  }
  if (ctx->own_mem && ctx->mem) (void)hipFree(ctx->mem);
  if (ctx->amg_mem) (void)hipFree(ctx->amg_mem);
  if (ctx->in_scratch) scratch_release(ctx->scratch_dev);
}

extern "C" void bdem_destroy(bdem_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  destroy_resources(ctx);
  delete ctx;
}

extern "C" const char *bdem_last_error(const bdem_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

extern "C" int bdem_sizes(const bdem_ctx *ctx, int32_t *n, int64_t *nb, int32_t *ns) {
  if (!ctx) return BDEM_E_INVALID;
  if (n) *n = ctx->S.n;
  if (nb) *nb = ctx->S.nb;
  if (ns) *ns = ctx->S.n_scenes;
  return BDEM_OK;
}

// Symbolic multigrid hierarchy: built on the host, uploaded into one
// allocation owned by the handle (freed by bdem_destroy).
static int amg_upload(bdem_ctx *ctx, const std::vector<double> &pos4, const std::vector<uint8_t> &flags,
                      const std::vector<int> &psid, const std::vector<int> &rp,
                      const std::vector<int> &col, const std::vector<int> &sblk,
                      const std::vector<double> &lo3, const std::vector<double> &h0) {
  const Sizes &S = ctx->S;
  const int NP = S.n_pad, NS = S.n_scenes;
  const size_t T = S.mixed ? 4 : 8;
  AmgHost H;
  amg_build(NP, NS, pos4, flags, psid, ctx->scene_pbeg, rp, col, lo3, h0, H);
  for (int sc = 0; sc < NS; ++sc)
    if (H.cbeg[sc + 1] - H.cbeg[sc] > AMG_COARSE_MAX) {
      ctx->err = "multigrid: a scene does not coarsen to 16 aggregates within 15 levels";
      return BDEM_E_INVALID;
    }
  for (int l = 1; l <= H.L; ++l)
    for (int v : H.lv[l].dslot)
      if (v < 0) { ctx->err = "multigrid: a coarse row without a diagonal block"; return BDEM_E_INVALID; }
  {   // the level-1 restriction reads an aggregate's members as consecutive rows
    const AmgHostLevel &l1 = H.lv[1];
    for (int A = 0; A < l1.n; ++A)
      for (int k = l1.mbeg[A]; k < l1.mbeg[A + 1]; ++k)
        if (l1.mlist[k] != l1.mlist[l1.mbeg[A]] + (k - l1.mbeg[A])) {
          ctx->err = "multigrid: the members of a first-level aggregate are not consecutive rows";
          return BDEM_E_INVALID;
        }
  }
  // one allocation carved into the arrays
  Layout L;
  AmgDev &a = ctx->amg_d;
  a = AmgDev();
  a.L = H.L;
  a.Lt = H.Lt;
  ctx->amg_hl.assign(H.L + 1, AmgLevel());
  auto addi = [&](int **p, size_t n) { L.add(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(int)); };
  auto addd = [&](double **p, size_t n) { L.add(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(double)); };
  addi(&a.slot_row0, H.slot_row0.size());
  addi(&a.parent0, NP);
  L.add(&a.pd0, 12 * (size_t)NP * T);
  addd(&a.t0, 6 * (size_t)NP);
  addd(&a.r0, 6 * (size_t)NP);
  // the coupling's sources as the kernel reads them: block code and column
  std::vector<int> hp_src(H.hp_gsrc.size()), hp_col(H.hp_gsrc.size());
  for (size_t m = 0; m < H.hp_gsrc.size(); ++m) {
    hp_src[m] = sblk[H.hp_gsrc[m]];
    hp_col[m] = col[H.hp_gsrc[m]];
  }
  a.nhp = (int)H.hp_agg.size();
  addi(&a.hp_ptr, H.hp_ptr.size());
  addi(&a.hp_agg, H.hp_agg.size());
  addi(&a.hp_self, H.hp_self.size());
  addi(&a.hp_gptr, H.hp_gptr.size());
  addi(&a.hp_src, hp_src.size());
  addi(&a.hp_col, hp_col.size());
  L.add(&a.hp_val, std::max<size_t>(H.hp_agg.size(), 1) * 36 * T);
  for (int l = 1; l <= H.L; ++l) {
    AmgLevel &V = ctx->amg_hl[l];
    const AmgHostLevel &h = H.lv[l];
    V.n = h.n;
    V.nslots = (int)h.col.size();
    addi(&V.row_ptr, h.row_ptr.size());
    addi(&V.col, h.col.size());
    addi(&V.slot_row, h.slot_row.size());
    addi(&V.dslot, h.dslot.size());
    L.add(&V.val, std::max<size_t>(h.col.size(), 1) * 36 * T);
    L.add(&V.dinv, std::max<size_t>(h.n, 1) * 36 * T);
    addi(&V.gptr, h.gptr.size());
    addi(&V.gsrc, h.gsrc.size());
    addi(&V.mbeg, h.mbeg.size());
    addi(&V.mlist, h.mlist.size());
    addi(&V.active, h.n);
    addi(&V.scene, h.n);
    addi(&V.parent, h.n);
    addd(&V.cen, 3 * (size_t)h.n);
    addd(&V.pd, 3 * (size_t)h.n);
    for (double **v : {&V.b, &V.t, &V.e}) addd(v, 6 * (size_t)h.n);
  }
  addi(&a.cbeg, NS + 1);
  addi(&a.tbeg, H.tbeg.size());
  L.add(reinterpret_cast<void **>(&a.coff), NS * sizeof(int64_t));
  addd(&a.cmat, (size_t)H.cdense);
  addd(&a.cwork, (size_t)H.cdense);
  for (int l = H.Lt; l <= H.L; ++l) a.tmax[l] = H.tmax[l];
  L.add(reinterpret_cast<void **>(&a.noff), (NS + 1) * sizeof(int64_t));
  L.add(&a.nmat, std::max<size_t>((size_t)H.noff[NS], 1) * T);
  addd(&a.nwork, 4 * std::max<size_t>((size_t)H.noff[NS], 1));
  AmgLevel *lvdev = nullptr;
  L.add(reinterpret_cast<void **>(&lvdev), (H.L + 1) * sizeof(AmgLevel));
  if (hipMalloc(&ctx->amg_mem, L.total + ALIGN) != hipSuccess) {
    ctx->amg_mem = nullptr;
    ctx->err = "hipMalloc failed for the multigrid hierarchy";
    return BDEM_E_NOMEM;
  }
  char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ctx->amg_mem) + ALIGN - 1) / ALIGN * ALIGN);
  L.bind(base);
  a.lv = lvdev;
  hipStream_t st = ctx->stream;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  auto upi = [&](int *dst, const std::vector<int> &v) {
    if (!v.empty()) chk(hipMemcpyAsync(dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, st));
  };
  upi(a.slot_row0, H.slot_row0);
  upi(a.parent0, H.parent0);
  upi(a.hp_ptr, H.hp_ptr);
  upi(a.hp_agg, H.hp_agg);
  upi(a.hp_self, H.hp_self);
  upi(a.hp_gptr, H.hp_gptr);
  upi(a.hp_src, hp_src);
  upi(a.hp_col, hp_col);
  for (int l = 1; l <= H.L; ++l) {
    const AmgLevel &V = ctx->amg_hl[l];
    const AmgHostLevel &h = H.lv[l];
    upi(V.row_ptr, h.row_ptr); upi(V.col, h.col); upi(V.slot_row, h.slot_row); upi(V.dslot, h.dslot);
    upi(V.gptr, h.gptr); upi(V.gsrc, h.gsrc); upi(V.mbeg, h.mbeg); upi(V.mlist, h.mlist);
    upi(V.active, h.active); upi(V.scene, h.scene); upi(V.parent, h.parent);
    for (double *v : {V.b, V.t, V.e, V.cen, V.pd}) chk(hipMemsetAsync(v, 0, std::max<size_t>(6 * (size_t)h.n, 1) * sizeof(double) / (v == V.cen || v == V.pd ? 2 : 1), st));
  }
  upi(a.cbeg, H.cbeg);
  upi(a.tbeg, H.tbeg);
  chk(hipMemcpyAsync(a.coff, H.coff.data(), NS * sizeof(int64_t), hipMemcpyHostToDevice, st));
  chk(hipMemcpyAsync(a.noff, H.noff.data(), (NS + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  chk(hipMemcpyAsync(lvdev, ctx->amg_hl.data(), (H.L + 1) * sizeof(AmgLevel), hipMemcpyHostToDevice, st));
  chk(hipMemsetAsync(a.pd0, 0, 12 * (size_t)NP * T, st));
  for (double *v : {a.t0, a.r0}) chk(hipMemsetAsync(v, 0, 6 * (size_t)NP * sizeof(double), st));
  chk(hipStreamSynchronize(st));
  if (e != hipSuccess) { ctx->err = std::string("HIP error during multigrid setup: ") + hipGetErrorString(e); return BDEM_E_HIP; }
  ctx->amg = true;
  ctx->d.amg_t0 = a.t0;   // the CG update writes the cycle's first step there
  return BDEM_OK;
}

// scratch_dev >= 0: the workspace is that device's static scratch (the
// caller holds its claim): no pinned host memory, no events, no multigrid
static int create_impl(const bdem_particles *p, const bdem_bonds *b, const bdem_material *mats,
                       int32_t n_mats, const bdem_options *opt, void *hip_stream,
                       void *workspace_dev, size_t workspace_bytes, int scratch_dev, bdem_ctx **out) {
  if (!out) return fail(nullptr, BDEM_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!p || !b || !mats || n_mats <= 0) return fail(nullptr, BDEM_E_INVALID, "NULL argument");
  const int n = p->n;
  if (n <= 0 || !p->pos || !p->quat || !p->radius || !p->material)
    return fail(nullptr, BDEM_E_INVALID, "particles: n <= 0 or a required array is NULL");
  if (b->nb < 0 || (b->nb > 0 && !b->ij)) return fail(nullptr, BDEM_E_INVALID, "bonds: bad nb / ij");
  if (b->nb > (int64_t)1 << 30) return fail(nullptr, BDEM_E_INVALID, "too many bonds");
  bdem_options o;
  if (opt) o = *opt;
  else bdem_default_options(&o);
  if (o.precision != BDEM_PREC_FP64 && o.precision != BDEM_PREC_MIXED)
    return fail(nullptr, BDEM_E_INVALID, "unknown precision");
  if (!(o.mu_s >= 0.0) || !(o.mu_r >= 0.0) || !std::isfinite(o.mu_s) || !std::isfinite(o.mu_r))
    return fail(nullptr, BDEM_E_INVALID, "friction coefficients must be finite and >= 0");
  if (!std::isfinite(o.k_self) || !std::isfinite(o.contact_margin))
    return fail(nullptr, BDEM_E_INVALID, "k_self and contact_margin must be finite");
  if (o.solver != BDEM_SOLVER_NEWTON && o.solver != BDEM_SOLVER_FIRST_ORDER)
    return fail(nullptr, BDEM_E_INVALID, "solver must be BDEM_SOLVER_NEWTON or BDEM_SOLVER_FIRST_ORDER");
  if (o.preconditioner != BDEM_PRECOND_BLOCK_JACOBI && o.preconditioner != BDEM_PRECOND_AMG)
    return fail(nullptr, BDEM_E_INVALID, "preconditioner must be BDEM_PRECOND_BLOCK_JACOBI or BDEM_PRECOND_AMG");
  if (o.integrator != BDEM_INTEGRATOR_EULER && o.integrator != BDEM_INTEGRATOR_MIDPOINT)
    return fail(nullptr, BDEM_E_INVALID, "integrator must be BDEM_INTEGRATOR_EULER or BDEM_INTEGRATOR_MIDPOINT");
  if (o.hessian != BDEM_HESS_EIGEN_CLAMP && o.hessian != BDEM_HESS_GAUSS_NEWTON)
    return fail(nullptr, BDEM_E_INVALID, "hessian must be BDEM_HESS_EIGEN_CLAMP or BDEM_HESS_GAUSS_NEWTON");
  if (o.amg_refresh != 0 && o.amg_refresh != 1)
    return fail(nullptr, BDEM_E_INVALID, "amg_refresh must be 0 or 1");
  if (o.max_newton < 0 || o.max_cg <= 0 || o.max_ls < 0 || o.cg_chunk <= 0)
    return fail(nullptr, BDEM_E_INVALID, "bad iteration limits");
  // ---- validation ----
  for (int i = 0; i < n; ++i) {
    const double *q = p->quat + 4 * i;
    const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!std::isfinite(qn) || std::fabs(qn - 1.0) > 1e-6) return fail(nullptr, BDEM_E_INVALID, "non-unit quaternion");
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(p->pos[3 * i + k])) return fail(nullptr, BDEM_E_NONFINITE, "non-finite position");
    if (!(p->radius[i] > 0.0)) return fail(nullptr, BDEM_E_INVALID, "radius must be > 0");
    if (p->material[i] < 0 || p->material[i] >= n_mats) return fail(nullptr, BDEM_E_INVALID, "bad material index");
    if (p->flags && p->flags[i] > 2) return fail(nullptr, BDEM_E_INVALID, "bad particle flag");
  }
  for (int k = 0; k < n_mats; ++k) {
    const bdem_material &m = mats[k];
    if (!(m.young > 0.0) || !(m.density > 0.0) || !(m.poisson > -1.0) || m.poisson >= 0.5)
      return fail(nullptr, BDEM_E_INVALID, "bad material constants");
    if (m.shear_mode != 0 && m.shear_mode != 1) return fail(nullptr, BDEM_E_INVALID, "bad shear_mode");
    for (int c = 0; c < 4; ++c)
      if (!(m.stiff_scale[c] >= 0.0)) return fail(nullptr, BDEM_E_INVALID, "bad stiff_scale");
  }
  std::vector<int> pcnt;
  std::vector<int64_t> bcnt;
  std::string err;
  if (!scene_sizes(p, b, pcnt, bcnt, err)) return fail(nullptr, BDEM_E_INVALID, err);
  {
    std::vector<uint64_t> keys(b->nb);
    for (int64_t k = 0; k < b->nb; ++k) {
      uint32_t i = b->ij[2 * k], j = b->ij[2 * k + 1];
      if (i == j) return fail(nullptr, BDEM_E_INVALID, "bond with i == j");
      if (b->material && (b->material[k] < 0 || b->material[k] >= n_mats))
        return fail(nullptr, BDEM_E_INVALID, "bad bond material");
      keys[k] = ((uint64_t)std::min(i, j) << 32) | std::max(i, j);
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
      return fail(nullptr, BDEM_E_INVALID, "duplicate bond");
  }
  if (scratch_dev >= 0 && o.preconditioner == BDEM_PRECOND_AMG)
    return fail(nullptr, BDEM_E_INVALID, "the multigrid preconditioner allocates its hierarchy: not available "
                                         "in the static scratch");
  bdem_ctx *ctx = new bdem_ctx();
  ctx->stream = (hipStream_t)hip_stream;
  ctx->scratch_dev = scratch_dev;
  {
    const char *tr = std::getenv("BDEM_TRACE");
    ctx->trace = (tr && tr[0] == '1') ? 1 : 0;
  }
  ctx->opt = o;
  ctx->S = compute_sizes(pcnt, bcnt, n, b->nb, o.precision == BDEM_PREC_MIXED);
  enable_contact(ctx->S, o);
  Sizes &S = ctx->S;
  const int NS = S.n_scenes;
  // ---- internal order: scenes padded to TILE particles / bonds ----
  ctx->scene_pbeg.assign(NS + 1, 0);
  ctx->scene_bbeg.assign(NS + 1, 0);
  for (int s = 0; s < NS; ++s) {
    ctx->scene_pbeg[s + 1] = ctx->scene_pbeg[s] + (pcnt[s] + TILE - 1) / TILE * TILE;
    ctx->scene_bbeg[s + 1] = ctx->scene_bbeg[s] + (int)((bcnt[s] + TILE - 1) / TILE * TILE);
  }
  // internal particle order: within each scene, by the multigrid's
  // first-level aggregation cell (side AMG_CELL r_max from the scene's
  // initial box corner, cells in the hierarchy's Morton order), and inside a
  // cell along a Morton (Z-order) curve of the initial positions.  Bonded
  // particles sit in nearby rows (locality of the bond gathers, the
  // assembly and the symmetric SpMV), and the members of an aggregate are
  // one contiguous range of rows (the restriction and prolongation read
  // them with unit stride).
  ctx->p_int.resize(n);
  {
    std::vector<uint64_t> code(n), cell(n);
    int i0 = 0;
    while (i0 < n) {
      const int s = p->scene ? p->scene[i0] : 0;
      int i1 = i0;
      while (i1 < n && (p->scene ? p->scene[i1] : 0) == s) ++i1;
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int i = i0; i < i1; ++i)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], p->pos[3 * i + k]);
          hi[k] = std::max(hi[k], p->pos[3 * i + k]);
        }
      const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
      double rmax = 0.0;
      for (int i = i0; i < i1; ++i) rmax = std::max(rmax, p->radius[i]);
      const double h0 = AMG_CELL * std::max(rmax, 1e-300);
      for (int i = i0; i < i1; ++i) {
        int64_t ck[3];
        for (int k = 0; k < 3; ++k) ck[k] = (int64_t)std::floor((p->pos[3 * i + k] - lo[k]) / h0);
        cell[i] = amg_cell_key(ck[0], ck[1], ck[2]);
        uint64_t c = 0;
        uint32_t q[3];
        for (int k = 0; k < 3; ++k)
          q[k] = (uint32_t)std::min(2097151.0, std::floor((p->pos[3 * i + k] - lo[k]) / ext * 2097151.0));
        for (int bit = 20; bit >= 0; --bit)
          for (int k = 0; k < 3; ++k) c = (c << 1) | ((q[k] >> bit) & 1u);
        code[i] = c;
      }
      std::vector<int> idx(i1 - i0);
      std::iota(idx.begin(), idx.end(), i0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
        return cell[a] != cell[c] ? cell[a] < cell[c] : code[a] < code[c];
      });
      for (int k = 0; k < (int)idx.size(); ++k) ctx->p_int[idx[k]] = ctx->scene_pbeg[s] + k;
      i0 = i1;
    }
  }
  const int NP = S.n_pad, NB = S.nb_pad;
  std::vector<double4> h_pn(NP, make_double4(0, 0, 0, 0)), h_qn(NP, make_double4(0, 0, 0, 1)),
      h_vn(NP, make_double4(0, 0, 0, 0)), h_wn(NP, make_double4(0, 0, 0, 0)),
      h_pc(NP, make_double4(0, 0, 1, 0));
  std::vector<uint8_t> h_flags(NP, 255);
  std::vector<int> h_psid(NP, 0);
  for (int s = 0; s < NS; ++s)
    for (int r = ctx->scene_pbeg[s]; r < ctx->scene_pbeg[s + 1]; ++r) h_psid[r] = s;
  // ground stiffness: the caller's value, or per scene E_max r_max over the
  // scene's own particle and bond materials (Section 5.4)
  std::vector<double> s_emax(NS, 0.0), s_rmax(NS, 0.0);
  for (int i = 0; i < n; ++i) {
    const int r = ctx->p_int[i];
    h_pn[r] = make_double4(p->pos[3 * i], p->pos[3 * i + 1], p->pos[3 * i + 2], 0.0);
    h_qn[r] = make_double4(p->quat[4 * i], p->quat[4 * i + 1], p->quat[4 * i + 2], p->quat[4 * i + 3]);
    if (p->vel) h_vn[r] = make_double4(p->vel[3 * i], p->vel[3 * i + 1], p->vel[3 * i + 2], 0.0);
    if (p->qvel) h_wn[r] = make_double4(p->qvel[4 * i], p->qvel[4 * i + 1], p->qvel[4 * i + 2], p->qvel[4 * i + 3]);
    const double rad = p->radius[i], rho = mats[p->material[i]].density;
    // solid sphere; extended mass M_s = diag(m I3, (8/5) m r^2 I4)  (Section 3.1)
    const double m = rho * 4.0 / 3.0 * M_PI * rad * rad * rad;
    h_pc[r] = make_double4(m, 8.0 / 5.0 * m * rad * rad, rad, 0.0);
    h_flags[r] = p->flags ? p->flags[i] : 0;
    const int si = p->scene ? p->scene[i] : 0;
    s_rmax[si] = std::max(s_rmax[si], rad);
    s_emax[si] = std::max(s_emax[si], mats[p->material[i]].young);
  }
  for (int64_t k = 0; k < b->nb; ++k)
    if (b->material) {
      const int si = p->scene ? p->scene[b->ij[2 * k]] : 0;
      s_emax[si] = std::max(s_emax[si], mats[b->material[k]].young);
    }
  ctx->scene_kc.assign(NS, 0.0);
  for (int s = 0; s < NS; ++s) ctx->scene_kc[s] = o.k_contact < 0.0 ? s_emax[s] * s_rmax[s] : o.k_contact;
  // element repulsion: k_ec (default E_max r_max of the scene, the order
  // Section 5.4 recommends), candidate margin (default r_max), grid cell
  ctx->scene_kself.assign(NS, 0.0);
  ctx->scene_cmargin.assign(NS, 0.0);
  ctx->scene_ccell.assign(NS, 1.0);
  for (int s = 0; s < NS; ++s) {
    ctx->scene_kself[s] = o.k_self < 0.0 ? s_emax[s] * s_rmax[s] : o.k_self;
    ctx->scene_cmargin[s] = o.contact_margin < 0.0 ? s_rmax[s] : o.contact_margin;
    ctx->scene_ccell[s] = 2.0 * s_rmax[s] + ctx->scene_cmargin[s];
  }
  // ---- bonds: per scene, sorted by (min row, max row) ----
  std::vector<int64_t> order(b->nb);
  std::iota(order.begin(), order.end(), 0);
  auto key = [&](int64_t k) {
    const int ri = ctx->p_int[b->ij[2 * k]], rj = ctx->p_int[b->ij[2 * k + 1]];
    return ((uint64_t)std::min(ri, rj) << 32) | (uint32_t)std::max(ri, rj);
  };
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t c) { return key(a) < key(c); });
  ctx->b_int.assign(b->nb, 0);
  std::vector<int2> h_bij(std::max(NB, 1), make_int2(0, 0));
  std::vector<double4> h_ra(std::max(NB, 1), make_double4(1, 0, 0, 1)), h_rb(std::max(NB, 1), make_double4(0, 0, 0, 0)),
      h_rc(std::max(NB, 1), make_double4(1, 0, 0, 0));
  std::vector<double2> h_str(std::max(NB, 1), make_double2(0, 0));
  std::vector<uint8_t> h_alive(std::max(NB, 1), 0);
  std::vector<int> h_bsid(std::max(NB, 1), 0);
  for (int s = 0; s < NS; ++s)
    for (int k = ctx->scene_bbeg[s]; k < ctx->scene_bbeg[s + 1]; ++k) h_bsid[k] = s;
  {
    std::vector<int> fill(NS, 0);
    for (int64_t k : order) {
      const int i = b->ij[2 * k], j = b->ij[2 * k + 1];
      const int s = p->scene ? p->scene[i] : 0;
      const int bi = ctx->scene_bbeg[s] + fill[s]++;
      ctx->b_int[k] = bi;
      const int ri = ctx->p_int[i], rj = ctx->p_int[j];
      h_bij[bi] = make_int2(ri, rj);
      const double u[3] = {p->pos[3 * j] - p->pos[3 * i], p->pos[3 * j + 1] - p->pos[3 * i + 1],
                           p->pos[3 * j + 2] - p->pos[3 * i + 2]};
      const double l0 = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      if (!(l0 > 0.0) || !std::isfinite(l0)) {
        destroy_resources(ctx);
        delete ctx;
        return fail(nullptr, BDEM_E_INVALID, "bonded particles coincide");
      }
      const bdem_material &m = mats[b->material ? b->material[k] : p->material[i]];
      const double E = m.young, G = E / (2.0 * (1.0 + m.poisson));
      const double r0 = 0.5 * (p->radius[i] + p->radius[j]);
      const double Sa = M_PI * r0 * r0, I = M_PI * r0 * r0 * r0 * r0 / 4.0, J = 2.0 * I;
      const double L2 = m.shear_mode == BDEM_SHEAR_LITERAL ? 1.0 : l0 * l0;
      h_ra[bi] = make_double4(u[0] / l0, u[1] / l0, u[2] / l0, l0);
      h_rb[bi] = make_double4(E * Sa / l0 * m.stiff_scale[0], G * Sa / l0 * m.stiff_scale[1] * L2,
                              G * J / l0 * m.stiff_scale[2], E * I / l0 * m.stiff_scale[3]);
      h_rc[bi] = make_double4(Sa, r0 / I, r0 / J, m.tension_only ? 1.0 : 0.0);
      h_str[bi] = make_double2(m.sigma_c, m.tau_c);
      h_alive[bi] = 1;
    }
  }
  // ---- block-CSR pattern: row r lists its bonds sorted by neighbour ----
  std::vector<int> rp(NP + 1, 0);
  for (int bi = 0; bi < NB; ++bi) {
    if (!h_alive[bi]) continue;   // padding (all real bonds start alive)
    rp[h_bij[bi].x + 1]++;
    rp[h_bij[bi].y + 1]++;
  }
  for (int r = 0; r < NP; ++r) rp[r + 1] += rp[r];
  std::vector<std::vector<std::pair<int, int>>> adj(NP);   // (neighbour, bond*2 + end)
  for (int bi = 0; bi < NB; ++bi) {
    if (!h_alive[bi]) continue;
    adj[h_bij[bi].x].push_back({h_bij[bi].y, 2 * bi});
    adj[h_bij[bi].y].push_back({h_bij[bi].x, 2 * bi + 1});
  }
  std::vector<int> h_col(std::max(S.n_slots, 1), 0), h_sb(std::max(S.n_slots, 1), 0);
  ctx->bslot_h.assign(std::max(NB, 1), make_int2(-1, -1));
  for (int r = 0; r < NP; ++r) {
    std::sort(adj[r].begin(), adj[r].end());
    for (size_t k = 0; k < adj[r].size(); ++k) {
      const int slot = rp[r] + (int)k;
      const int bi = adj[r][k].second >> 1, end = adj[r][k].second & 1;
      h_col[slot] = adj[r][k].first;
      h_sb[slot] = 2 * bi + end;
      if (end == 0) ctx->bslot_h[bi].x = slot;
      else ctx->bslot_h[bi].y = slot;
    }
  }
  adj.clear();
  adj.shrink_to_fit();
  // ---- device memory ----
  Layout L;
  make_layout(S, ctx->d, L);
  const size_t need = L.total + ALIGN;
  if (workspace_dev) {
    if (workspace_bytes < need) {
      destroy_resources(ctx);
      delete ctx;
      if (scratch_dev >= 0)
        return fail(nullptr, BDEM_E_NOMEM, "the problem needs " + std::to_string(need) +
                                           " bytes of workspace; the static scratch holds " +
                                           std::to_string(workspace_bytes));
      return fail(nullptr, BDEM_E_NOMEM, "workspace too small");
    }
    ctx->mem = workspace_dev;
  } else {
    if (hipMalloc(&ctx->mem, need) != hipSuccess) {
      destroy_resources(ctx);
      delete ctx;
      return fail(nullptr, BDEM_E_NOMEM, "hipMalloc failed");
    }
    ctx->own_mem = true;
  }
  char *base = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(ctx->mem) + ALIGN - 1) / ALIGN * ALIGN);
  L.bind(base);
  DevPtrs &d = ctx->d;
  d.n_pad = NP;
  d.nb_pad = NB;
  d.one_scene = NS == 1 ? 1 : 0;
  d.n_slots = S.n_slots;
  d.n_bucket = S.n_bucket;
  // ---- params ----
  Params &P = ctx->P;
  P.gx = o.gravity[0]; P.gy = o.gravity[1]; P.gz = o.gravity[2];
  {
    const double gn = std::sqrt(o.ground_normal[0] * o.ground_normal[0] + o.ground_normal[1] * o.ground_normal[1] +
                                o.ground_normal[2] * o.ground_normal[2]);
    if (o.k_contact != 0.0 && !(gn > 0.0)) {
      destroy_resources(ctx);
      delete ctx;
      return fail(nullptr, BDEM_E_INVALID, "ground normal is zero");
    }
    P.gnx = gn > 0 ? o.ground_normal[0] / gn : 0.0;
    P.gny = gn > 0 ? o.ground_normal[1] / gn : 0.0;
    P.gnz = gn > 0 ? o.ground_normal[2] / gn : 0.0;
  }
  P.gh = o.ground_offset;
  P.newton_tol = o.newton_tol;
  P.newton_rtol = o.newton_rtol;
  P.armijo_c = o.armijo_c;
  P.cg_rtol_max = o.cg_rtol_max;
  P.max_newton = o.max_newton;
  P.max_cg = o.max_cg;
  P.max_ls = o.max_ls;
  P.n_scenes = NS;
  P.first_order = o.solver == BDEM_SOLVER_FIRST_ORDER ? 1 : 0;
  P.midpoint = o.integrator == BDEM_INTEGRATOR_MIDPOINT ? 1 : 0;
  P.contact = S.contact ? 1 : 0;
  P.mu_s = o.mu_s;
  P.mu_r = o.mu_r;
  // ---- upload ----
  hipStream_t st = ctx->stream;
  auto up = [&](void *dst, const void *src, size_t bytes) { return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st); };
  std::vector<SceneCtl> ctl0(NS);
  std::memset(ctl0.data(), 0, sizeof(SceneCtl) * NS);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (e == hipSuccess) e = x; };
  chk(up(d.pn, h_pn.data(), NP * sizeof(double4)));
  chk(up(d.qn, h_qn.data(), NP * sizeof(double4)));
  chk(up(d.vn, h_vn.data(), NP * sizeof(double4)));
  chk(up(d.wn, h_wn.data(), NP * sizeof(double4)));
  chk(up(d.pconst, h_pc.data(), NP * sizeof(double4)));
  chk(up(d.flags, h_flags.data(), NP));
  chk(up(d.psid, h_psid.data(), NP * sizeof(int)));
  chk(up(d.row_ptr, rp.data(), (NP + 1) * sizeof(int)));
  chk(up(d.col, h_col.data(), h_col.size() * sizeof(int)));
  chk(up(d.sblk, h_sb.data(), h_sb.size() * sizeof(int)));
  chk(up(d.bij, h_bij.data(), h_bij.size() * sizeof(int2)));
  chk(up(d.brest_a, h_ra.data(), h_ra.size() * sizeof(double4)));
  chk(up(d.brest_b, h_rb.data(), h_rb.size() * sizeof(double4)));
  chk(up(d.brest_c, h_rc.data(), h_rc.size() * sizeof(double4)));
  chk(up(d.bstrength, h_str.data(), h_str.size() * sizeof(double2)));
  chk(up(d.alive, h_alive.data(), h_alive.size()));
  chk(up(d.bslot, ctx->bslot_h.data(), ctx->bslot_h.size() * sizeof(int2)));
  chk(up(d.bsid, h_bsid.data(), h_bsid.size() * sizeof(int)));
  chk(up(d.ctl, ctl0.data(), NS * sizeof(SceneCtl)));
  chk(up(d.scene_pbeg, ctx->scene_pbeg.data(), (NS + 1) * sizeof(int)));
  chk(up(d.scene_bbeg, ctx->scene_bbeg.data(), (NS + 1) * sizeof(int)));
  if (S.contact) {
    chk(hipMemsetAsync(d.ncand, 0, NP * sizeof(int), st));
    chk(hipMemsetAsync(d.nact, 0, NP * sizeof(int), st));
  }
  // iterate / trial / prediction start as the state; solver buffers zero
  chk(hipMemcpyAsync(d.px, d.pn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  chk(hipMemcpyAsync(d.qx, d.qn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  chk(hipMemcpyAsync(d.ph, d.pn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  chk(hipMemcpyAsync(d.qh, d.qn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  chk(hipMemcpyAsync(d.pt, d.pn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  chk(hipMemcpyAsync(d.qt, d.qn, NP * sizeof(double4), hipMemcpyDeviceToDevice, st));
  for (double *v : {d.z, d.cx, d.cr, d.cs, d.cp, d.cAp, d.cq}) chk(hipMemsetAsync(v, 0, (size_t)NP * 6 * sizeof(double), st));
  const size_t T = S.mixed ? 4 : 8;
  chk(hipMemsetAsync(d.hoff, 0, (size_t)std::max(NB, 1) * 36 * T, st));
  chk(hipMemsetAsync(d.hhalf, 0, (size_t)std::max(S.n_slots, 1) * 21 * T, st));
  chk(hipMemsetAsync(d.ghalf, 0, (size_t)std::max(S.n_slots, 1) * 6 * sizeof(double), st));
  chk(hipMemsetAsync(d.hdiag, 0, (size_t)NP * 21 * T, st));
  chk(hipMemsetAsync(d.dinv, 0, (size_t)NP * 21 * T, st));
  chk(hipMemsetAsync(d.degenerate, 0, sizeof(int), st));
  // counters: written by the decision kernels straight into mapped host
  // memory, read by the host once an event or the stream has passed them
  if (scratch_dev >= 0) {
    // counters in the workspace, copied to the host after the stream drains
    ctx->h_counters = ctx->h_counters_local;
    ctx->d.counters = d.counters_ws;
    chk(hipMemsetAsync(d.counters_ws, 0, 8 * sizeof(int), st));
    ctx->h_ctl_local.assign(NS, SceneCtl{});
    ctx->h_ctl = ctx->h_ctl_local.data();
  } else {
    ctx->host_pinned = true;
    chk(hipHostMalloc((void **)&ctx->h_counters, 8 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent));
    if (e == hipSuccess) {
      std::memset(ctx->h_counters, 0, 8 * sizeof(int));
      chk(hipHostGetDevicePointer((void **)&ctx->d.counters, ctx->h_counters, 0));
    }
    chk(hipHostMalloc((void **)&ctx->h_ctl, NS * sizeof(SceneCtl), hipHostMallocDefault));
    for (int k = 0; k < 2; ++k) chk(hipEventCreateWithFlags(&ctx->ev_slot[k], hipEventDisableTiming));
  }
  chk(hipStreamSynchronize(st));
  if (e != hipSuccess) {
    const std::string m = std::string("HIP error during create: ") + hipGetErrorString(e);
    destroy_resources(ctx);
    delete ctx;
    return fail(nullptr, BDEM_E_HIP, m);
  }
  if (o.preconditioner == BDEM_PRECOND_AMG) {
    // aggregation cells of side AMG_CELL r_max from each scene's initial box corner
    std::vector<double> pos4((size_t)NP * 4), lo3(3 * NS, 1e300), h0(NS);
    for (int r = 0; r < NP; ++r) {
      pos4[4 * (size_t)r] = h_pn[r].x; pos4[4 * (size_t)r + 1] = h_pn[r].y; pos4[4 * (size_t)r + 2] = h_pn[r].z;
      if (h_flags[r] == 255) continue;
      const int sc = h_psid[r];
      lo3[3 * sc] = std::min(lo3[3 * sc], h_pn[r].x);
      lo3[3 * sc + 1] = std::min(lo3[3 * sc + 1], h_pn[r].y);
      lo3[3 * sc + 2] = std::min(lo3[3 * sc + 2], h_pn[r].z);
    }
    for (int sc = 0; sc < NS; ++sc) h0[sc] = AMG_CELL * s_rmax[sc];
    const int rc = amg_upload(ctx, pos4, h_flags, h_psid, rp, h_col, h_sb, lo3, h0);
    if (rc) {
      const std::string m = ctx->err;
      destroy_resources(ctx);
      delete ctx;
      return fail(nullptr, rc, m);
    }
  }
  ctx->in_scratch = scratch_dev >= 0;
  *out = ctx;
  return BDEM_OK;
}

extern "C" int bdem_create(const bdem_particles *p, const bdem_bonds *b, const bdem_material *mats,
                           int32_t n_mats, const bdem_options *opt, void *hip_stream,
                           void *workspace_dev, size_t workspace_bytes, bdem_ctx **out) {
  return create_impl(p, b, mats, n_mats, opt, hip_stream, workspace_dev, workspace_bytes, -1, out);
}

extern "C" int bdem_create_in_scratch(const bdem_particles *p, const bdem_bonds *b,
                                      const bdem_material *mats, int32_t n_mats,
                                      const bdem_options *opt, void *hip_stream, bdem_ctx **out) {
  if (!out) return fail(nullptr, BDEM_E_INVALID, "out is NULL");
  *out = nullptr;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES)
    return fail(nullptr, BDEM_E_HIP, "no current HIP device");
  void *ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_used[dev])
      return fail(nullptr, BDEM_E_STATE, "another handle on this device lives in the static scratch "
                                         "(bdem_destroy it first)");
    if (!g_scratch_ptr[dev]) {
      void *ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return fail(nullptr, BDEM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch_ptr[dev] = ptr;
    }
    g_scratch_used[dev] = true;
    ws = g_scratch_ptr[dev];
  }
  const int rc = create_impl(p, b, mats, n_mats, opt, hip_stream, ws, SCRATCH_BYTES, dev, out);
  if (rc != BDEM_OK) scratch_release(dev);
  return rc;
}

// ---------------------------------------------------------------------------
// helpers for the step driver
// ---------------------------------------------------------------------------

// the counter slot written by the last decision kernel is valid once the
// stream has drained
// inertia target of a step: the prediction x_hat that k_predict wrote,
// replaced for the free particles by z_hat in the midpoint form
static void launch_step_target(const DevPtrs &d, const Params &P, hipStream_t st) {
  if (!P.midpoint) return;
  launch_bond_force(d, st);
  launch_midpoint_target(d, P, st);
}

// element-repulsion candidates of a step, at the predicted positions (before
// the midpoint form replaces the prediction by z_hat); fails when a particle
// has more candidates than the per-particle capacity
static int contact_candidates(bdem_ctx *ctx) {
  if (!ctx->P.contact) return BDEM_OK;
  hipStream_t st = ctx->stream;
  launch_contact_broad_phase(ctx->d, st);
  int over = 0;
  HIP_TRY(hipMemcpyAsync(&over, ctx->d.cand_over, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (over > 0)
    return fail(ctx, BDEM_E_CAPACITY, std::to_string(over) +
                " particles have more than 32 element-repulsion candidates (reduce contact_margin)");
  return BDEM_OK;
}

static int read_counters(bdem_ctx *ctx) {
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  // a handle in the static scratch keeps its counters in device memory
  if (ctx->in_scratch)
    HIP_TRY(hipMemcpy(ctx->h_counters, ctx->d.counters, 8 * sizeof(int), hipMemcpyDeviceToHost));
  return BDEM_OK;
}

// with profiling, the SpMV launches of one PCG iteration in this many are
// bracketed by events (and the initial product of every solve)
constexpr int PROF_SPMV_EVERY = 8;

static void prof_mark(bdem_ctx *ctx, int kind, bool start) {
  if (!ctx->profiling) return;
  if (ctx->ev_used + 1 >= ctx->ev_pool.size()) {
    const size_t add = 1024;
    for (size_t k = 0; k < add; ++k) {
      hipEvent_t ev;
      (void)hipEventCreate(&ev);
      ctx->ev_pool.push_back(ev);
    }
  }
  if (start) {
    ctx->ev_marks.push_back({kind, ctx->ev_used});
    ctx->ev_iter.push_back(ctx->prof_iter);
  }
  (void)hipEventRecord(ctx->ev_pool[ctx->ev_used++], ctx->stream);
}

// the multigrid cycle's SpMV launches, bracketed like the PCG's own
static void prof_mark_spmv(void *arg, bool start) { prof_mark(static_cast<bdem_ctx *>(arg), 1, start); }
static SpmvMark cycle_marks(bdem_ctx *ctx, bool on) {
  SpmvMark m;
  if (on) {
    m.fn = prof_mark_spmv;
    m.arg = ctx;
  }
  return m;
}

static void prof_collect(bdem_ctx *ctx, double *ms_kind, int *cnt_kind) {
  for (auto &m : ctx->ev_marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev_pool[m.second], ctx->ev_pool[m.second + 1]) == hipSuccess) {
      ms_kind[m.first] += ms;
      cnt_kind[m.first] += 1;
    }
  }
  ctx->ev_marks.clear();
  ctx->ev_iter.clear();
  ctx->ev_used = 0;
}

// Gradient (and Hessian) of every active scene at the Newton iterate, and the
// partials the Newton check reads.  With the Gauss-Newton Hessian one
// row-parallel kernel forms gradient, blocks and inverse; the objective of a
// step's first iterate then comes from the energy pass (later iterates take
// the value of the line-search trial they accepted).  Otherwise the
// bond-parallel kernels evaluate the exact reduced Hessian, eigen-clamped per
// bond when psd, and the particle kernel assembles it.
static bool rows_path(const bdem_ctx *ctx, bool hess) {
  return hess && ctx->opt.hessian == BDEM_HESS_GAUSS_NEWTON;
}
static void launch_evaluation(bdem_ctx *ctx, bool hess, bool psd, bool first, bool pot) {
  const DevPtrs &d = ctx->d;
  hipStream_t st = ctx->stream;
  const bool mixed = ctx->S.mixed, mid = ctx->P.midpoint != 0;
  if (rows_path(ctx, hess)) {
    if (first) {
      launch_bond_energy(d, false, mid, st);
      launch_particle_energy(d, ctx->P, pot, st);
    }
    prof_mark(ctx, 0, true);
    launch_rows_eval(d, ctx->P, mixed, mid, pot, st);
    prof_mark(ctx, 0, false);
  } else {
    prof_mark(ctx, 0, true);
    launch_bond_eval(d, mixed, psd, hess, mid, st);
    prof_mark(ctx, 0, false);
    launch_particle_eval(d, ctx->P, mixed, hess, pot, st);
  }
}

// one PCG iteration: update, SpMV with the three dots, per-scene scalars
static void launch_cg_iteration(bdem_ctx *ctx, bool profile_spmv) {
  const bool mixed = ctx->S.mixed;
  // block-Jacobi: the update forms (r, u) and (r, r) with the u it writes;
  // multigrid: the update writes the cycle's first step, and the cycle's last
  // kernel writes u = V(r) and forms them
  const bool amg = ctx->amg;
  // consecutive SpMVs walk the row blocks in opposite orders: block-Jacobi
  // has one per iteration (the next iteration takes the other order),
  // multigrid two (the cycle's r, the PCG's !r; every iteration starts with r)
  const bool rev = ctx->spmv_rev;
  if (!amg) ctx->spmv_rev = !rev;
  launch_cg_update(ctx->d, mixed, ctx->upd_variant, ctx->stream, !amg);
  if (amg)
    launch_amg_vcycle(ctx->d, ctx->amg_d, ctx->amg_hl.data(), ctx->S.n_scenes, mixed, ctx->spmv_variant, true,
                      rev, ctx->stream, cycle_marks(ctx, profile_spmv));
  if (profile_spmv) prof_mark(ctx, 1, true);
  launch_spmv(ctx->d, mixed, ctx->spmv_variant, ctx->stream, SPMV_DOTS_WU, amg ? !rev : rev);
  if (profile_spmv) prof_mark(ctx, 1, false);
  if (ctx->P.contact) launch_contact_spmv(ctx->d, ctx->P, ctx->stream);
  launch_cg_scalars(ctx->d, ctx->P, ctx->stream, true);
}

static void drop_cg_graphs(bdem_ctx *ctx) {
  for (int k = 0; k < 2; ++k) {
    if (ctx->cg_exec[k]) (void)hipGraphExecDestroy(ctx->cg_exec[k]);
    if (ctx->cg_graph[k]) (void)hipGraphDestroy(ctx->cg_graph[k]);
    ctx->cg_exec[k] = nullptr;
    ctx->cg_graph[k] = nullptr;
  }
}

static int build_cg_graphs(bdem_ctx *ctx, int chunk) {
  for (int slot = 0; slot < 2; ++slot) {
    HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) launch_cg_iteration(ctx, false);
    if (ctx->S.n_scenes > 1) launch_count_active(ctx->d, ctx->S.n_scenes, slot, ctx->stream);
    HIP_TRY(hipStreamEndCapture(ctx->stream, &ctx->cg_graph[slot]));
    HIP_TRY(hipGraphInstantiate(&ctx->cg_exec[slot], ctx->cg_graph[slot], nullptr, nullptr, 0));
  }
  return BDEM_OK;
}

// PCG for every scene whose cg_active flag is set.  Iterations are issued in
// chunks; after each chunk the active-scene count is copied to pinned host
// memory.  Pipelined polling: the host reads the count of chunk c-1 while
// chunk c is in flight, so the device never waits on the host.
static int run_pcg(bdem_ctx *ctx) {
  const bool mixed = ctx->S.mixed;
  hipStream_t st = ctx->stream;
  const size_t mark0 = ctx->ev_marks.size();
  // poll slots: 1 while PCG runs; with one scene the scalars kernel clears
  // both when it stops, with several the count kernel rewrites its slot
  ctx->h_counters[1] = 1;
  ctx->h_counters[5] = 1;
  if (ctx->in_scratch) {
    HIP_TRY(hipMemcpyAsync(ctx->d.counters, ctx->h_counters, 8 * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  launch_cg_init(ctx->d, mixed, st);
  const bool rev = ctx->spmv_rev;
  if (!ctx->amg) ctx->spmv_rev = !rev;
  if (ctx->amg)
    launch_amg_vcycle(ctx->d, ctx->amg_d, ctx->amg_hl.data(), ctx->S.n_scenes, mixed, ctx->spmv_variant, false, rev,
                      st, cycle_marks(ctx, ctx->profiling == 1));
  if (ctx->profiling == 1) prof_mark(ctx, 1, true);
  launch_spmv(ctx->d, mixed, ctx->spmv_variant, st, SPMV_DOTS_ALL, ctx->amg ? !rev : rev);
  if (ctx->profiling == 1) prof_mark(ctx, 1, false);
  if (ctx->P.contact) launch_contact_spmv(ctx->d, ctx->P, st);
  launch_cg_scalars(ctx->d, ctx->P, st, false);
  if (ctx->S.n_scenes > 1) launch_count_active(ctx->d, ctx->S.n_scenes, 0, st);
  const int chunk = std::max(1, ctx->opt.cg_chunk);
  const bool graph = ctx->opt.use_graph && st != nullptr && ctx->profiling != 1;
  int rc = BDEM_OK;
  // The first chunk is issued without waiting for the initial scalars: every
  // kernel of an iteration returns at once for a scene whose solve stopped,
  // and the first poll sees it.  (A handle in the static scratch reads its
  // counters synchronously, and capturing the chunk graphs waits as well.)
  if (ctx->in_scratch || (graph && !ctx->cg_exec[0])) {
    rc = read_counters(ctx);
    if (rc) return rc;
    if (ctx->h_counters[1] == 0) return BDEM_OK;
  }
  if (graph && !ctx->cg_exec[0]) {
    rc = build_cg_graphs(ctx, chunk);
    if (rc) return rc;
  }
  const int max_chunks = ctx->opt.max_cg / chunk + 3;
  int pending = -1;
  for (int c = 0; c < max_chunks; ++c) {
    const int slot = c & 1;
    if (graph) {
      HIP_TRY(hipGraphLaunch(ctx->cg_exec[slot], st));
    } else {
      for (int k = 0; k < chunk; ++k) {
        // profiling: the SpMV launches of every PROF_SPMV_EVERY-th iteration
        // are bracketed (events between launches lengthen the timed steps)
        const int it = c * chunk + k;
        ctx->prof_iter = it;
        launch_cg_iteration(ctx, ctx->profiling == 1 && it % PROF_SPMV_EVERY == 0);
      }
      ctx->prof_iter = -1;
      if (ctx->S.n_scenes > 1) launch_count_active(ctx->d, ctx->S.n_scenes, slot, st);
    }
    if (ctx->in_scratch) {   // no events: drain the stream and read this chunk's count
      rc = read_counters(ctx);
      if (rc) return rc;
      if (ctx->h_counters[4 * slot + 1] == 0) break;
      continue;
    }
    HIP_TRY(hipEventRecord(ctx->ev_slot[slot], st));
    if (pending >= 0) {
      HIP_TRY(hipEventSynchronize(ctx->ev_slot[pending]));
      if (ctx->h_counters[4 * pending + 1] == 0) break;
    }
    pending = slot;
  }
  // no wait for the chunk still in flight: what follows is issued behind it
  // on the same stream
  if (ctx->profiling == 1 && !graph) {
    HIP_TRY(hipStreamSynchronize(st));
    // SpMV launches issued after every scene had converged returned at once:
    // keep the timings of the initial product(s) and of iterations
    // 0 .. max(cg_it) - 1 of this solve
    std::vector<SceneCtl> after(ctx->S.n_scenes);
    HIP_TRY(hipMemcpy(after.data(), ctx->d.ctl, after.size() * sizeof(SceneCtl), hipMemcpyDeviceToHost));
    int real = 0;
    for (const auto &c : after) real = std::max(real, c.cg_it);
    std::vector<std::pair<int, size_t>> kept(ctx->ev_marks.begin(), ctx->ev_marks.begin() + mark0);
    std::vector<int> kept_it(ctx->ev_iter.begin(), ctx->ev_iter.begin() + mark0);
    for (size_t k = mark0; k < ctx->ev_marks.size(); ++k)
      if (ctx->ev_marks[k].first != 1 || ctx->ev_iter[k] < real) {
        kept.push_back(ctx->ev_marks[k]);
        kept_it.push_back(ctx->ev_iter[k]);
      }
    ctx->ev_marks.swap(kept);
    ctx->ev_iter.swap(kept_it);
  }
  return BDEM_OK;
}

static int run_line_search(bdem_ctx *ctx) {
  hipStream_t st = ctx->stream;
  for (int it = 0; it <= ctx->opt.max_ls + 2; ++it) {
    launch_ls_trial(ctx->d, ctx->P, st);
    launch_bond_energy(ctx->d, true, ctx->P.midpoint != 0, st);
    if (ctx->P.contact) launch_contact_trial_energy(ctx->d, ctx->P, st);
    launch_ls_decide(ctx->d, ctx->P, st);
    launch_ls_accept(ctx->d, st);
    launch_count_active(ctx->d, ctx->S.n_scenes, 0, st);
    int rc = read_counters(ctx);
    if (rc) return rc;
    if (ctx->h_counters[2] == 0) return BDEM_OK;
  }
  return BDEM_OK;
}

static double elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, a, b);
  return ms;
}

// one implicit step of every scene (Algorithm 3), dt per scene
static int step_impl(bdem_ctx *ctx, const double *dts, bdem_step_stats *stats, bool per_scene) {
  const int NS = ctx->S.n_scenes;
  for (int s = 0; s < NS; ++s)
    if (!(dts[s] > 0.0) || !std::isfinite(dts[s])) return fail(ctx, BDEM_E_INVALID, "dt must be > 0");
  hipStream_t st = ctx->stream;
  DevPtrs &d = ctx->d;
  const bool mixed = ctx->S.mixed;
  hipEvent_t ph[6];
  for (auto &e : ph) HIP_TRY(hipEventCreate(&e));
  struct EvGuard { hipEvent_t *e; ~EvGuard() { for (int k = 0; k < 6; ++k) (void)hipEventDestroy(e[k]); } } guard{ph};
  double t_eval = 0, t_cg = 0, t_ls = 0;
  HIP_TRY(hipEventRecord(ph[0], st));
  // reset the control blocks
  auto init_ctl = [&]() -> hipError_t {
    for (int s = 0; s < NS; ++s) {
      SceneCtl &c = ctx->h_ctl[s];
      std::memset(&c, 0, sizeof(c));
      c.dt = dts[s];
      c.inv_dt2 = 1.0 / (dts[s] * dts[s]);
      c.kc = ctx->scene_kc[s];
      c.kself = ctx->scene_kself[s];
      c.cmargin = ctx->scene_cmargin[s];
      c.ccell = ctx->scene_ccell[s];
      c.newton_active = 1;
    }
    hipError_t e = hipMemcpyAsync(d.ctl, ctx->h_ctl, NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(d.degenerate, 0, sizeof(int), st);
    return e;
  };
  HIP_TRY(init_ctl());
  launch_predict(d, true, st);
  {
    const int rc = contact_candidates(ctx);
    if (rc) return rc;
  }
  launch_step_target(d, ctx->P, st);
  bool restarted = false;
  for (int k = 0; k <= ctx->opt.max_newton + 1; ++k) {
    HIP_TRY(hipEventRecord(ph[1], st));
    const bool hess = !ctx->P.first_order;   // Algorithm 1 needs the gradient only
    launch_evaluation(ctx, hess, true, k == 0, false);
    // the multigrid hierarchy: every Newton iteration, or once per step
    if (hess && ctx->amg) {
      if (k == 0 || ctx->opt.amg_refresh == 0) launch_amg_setup(d, ctx->amg_d, ctx->amg_hl.data(), NS, mixed, st);
      launch_amg_couple(d, ctx->amg_d, mixed, st);   // H P of this iterate's Hessian
    }
    launch_newton_check(d, ctx->P, k == 0 ? 1 : 0, rows_path(ctx, hess), st);
    launch_count_active(d, NS, 0, st);
    int rc = read_counters(ctx);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ph[2], st));
    t_eval += elapsed(ph[1], ph[2]);
    if (ctx->h_counters[3] > 0) {
      if (k == 0 && !restarted) {
        // the prediction left the potential's domain: the affected scenes
        // start from x_n (always inside), evaluated as the first iterate
        restarted = true;
        launch_restart_from_state(d, st);
        HIP_TRY(init_ctl());
        k = -1;
        continue;
      }
      return fail(ctx, BDEM_E_DEGENERATE, "|q_i + q_j| < 1e-6 in a bond");
    }
    if (ctx->h_counters[0] == 0) break;
    if (ctx->P.first_order) {
      launch_steepest(d, st);
    } else {
      rc = run_pcg(ctx);
      if (rc) return rc;
    }
    launch_cg_slope(d, ctx->P, st);
    HIP_TRY(hipEventRecord(ph[3], st));
    rc = run_line_search(ctx);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(ph[4], st));
    HIP_TRY(hipEventSynchronize(ph[4]));
    t_cg += elapsed(ph[2], ph[3]);
    t_ls += elapsed(ph[3], ph[4]);
    if (ctx->trace) {
      HIP_TRY(hipMemcpy(ctx->h_ctl, d.ctl, sizeof(SceneCtl), hipMemcpyDeviceToHost));
      const SceneCtl &c = ctx->h_ctl[0];
      std::fprintf(stderr,
                   "[bdem trace] it %d |z| %.6e phi %.12e slope %.3e alpha %.3e ls %d cg %d "
                   "cg_tol %.3e |r| %.3e phi_trial %.12e move %.3e status %d (r,u) %.3e (w,u) %.3e\n",
                   c.newton_it, c.gnorm, c.phi, c.slope, c.alpha_ls, c.ls_it, c.cg_it, c.cg_tol,
                   std::sqrt(c.rr), c.phi_trial, c.last_move, c.status, c.rz_new, c.pAp);
    }
  }
  // outcome per scene
  HIP_TRY(hipMemcpyAsync(ctx->h_ctl, d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int s = 0; s < NS; ++s)
    if (ctx->h_ctl[s].status == ST_NONFINITE) return fail(ctx, BDEM_E_NONFINITE, "non-finite objective or gradient");
  HIP_TRY(hipEventRecord(ph[1], st));
  launch_finish_step(d, st);
  if (ctx->P.mu_s > 0.0 || ctx->P.mu_r > 0.0) launch_friction(d, ctx->P, st);
  int64_t broken = 0;
  if (ctx->opt.break_each_step && ctx->S.nb_pad > 0) {
    launch_bond_fracture(d, st);
    const int nt = ctx->S.nb_pad / TILE;
    std::vector<int> cnt(nt);
    HIP_TRY(hipMemcpyAsync(cnt.data(), d.part_cnt, nt * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int v : cnt) broken += v;
    if (per_scene && stats) {
      for (int s = 0; s < NS; ++s) {
        int64_t bs = 0;
        for (int t = ctx->scene_bbeg[s] / TILE; t < ctx->scene_bbeg[s + 1] / TILE; ++t) bs += cnt[t];
        stats[s].bonds_broken = bs;
      }
    }
  }
  HIP_TRY(hipEventRecord(ph[5], st));
  HIP_TRY(hipEventSynchronize(ph[5]));
  double kind_ms[2] = {0, 0};
  int kind_cnt[2] = {0, 0};
  prof_collect(ctx, kind_ms, kind_cnt);
  int ret = BDEM_OK;
  for (int s = 0; s < NS; ++s) {
    const SceneCtl &c = ctx->h_ctl[s];
    if (c.status == ST_NOT_CONVERGED) ret = std::max(ret, (int)BDEM_W_NOT_CONVERGED);
    if (c.status == ST_LS_FAILED) ret = std::max(ret, (int)BDEM_W_LS_FAILED);
  }
  if (stats) {
    auto fill = [&](bdem_step_stats &o, const SceneCtl &c) {
      o.newton_iters = c.newton_it;
      o.cg_iters = c.cg_total;
      o.ls_backtracks = c.ls_total;
      o.status = c.status;
      o.grad0 = c.gnorm0;
      o.grad_final = c.gnorm;
      o.phi = c.phi;
      o.t_ms[0] = 0;
      o.t_ms[1] = t_eval;
      o.t_ms[2] = t_cg;
      o.t_ms[3] = t_ls;
      o.t_ms[4] = elapsed(ph[1], ph[5]);
      o.t_ms[5] = elapsed(ph[0], ph[5]);
      o.t_ms[6] = kind_ms[0];
      o.t_ms[7] = kind_ms[1];
    };
    if (per_scene) {
      for (int s = 0; s < NS; ++s) fill(stats[s], ctx->h_ctl[s]);
    } else {
      bdem_step_stats &o = *stats;
      std::memset(&o, 0, sizeof(o));
      fill(o, ctx->h_ctl[0]);
      o.newton_iters = o.cg_iters = o.ls_backtracks = 0;
      o.grad0 = o.grad_final = o.phi = 0;
      for (int s = 0; s < NS; ++s) {
        const SceneCtl &c = ctx->h_ctl[s];
        o.newton_iters += c.newton_it;
        o.cg_iters += c.cg_total;
        o.ls_backtracks += c.ls_total;
        o.grad0 = std::max(o.grad0, c.gnorm0);
        o.grad_final = std::max(o.grad_final, c.gnorm);
        o.phi += c.phi;
        o.status = std::max(o.status, c.status);
      }
      o.bonds_broken = broken;
    }
  }
  ctx->prof_cnt[0] = kind_cnt[0];
  ctx->prof_cnt[1] = kind_cnt[1];
  return ret;
}

extern "C" int bdem_step(bdem_ctx *ctx, double dt, bdem_step_stats *stats) {
  if (!ctx) return BDEM_E_INVALID;
  std::vector<double> dts(ctx->S.n_scenes, dt);
  return step_impl(ctx, dts.data(), stats, false);
}

extern "C" int bdem_step_batched(bdem_ctx *ctx, const double *dt_per_scene, bdem_step_stats *stats) {
  if (!ctx || !dt_per_scene) return BDEM_E_INVALID;
  return step_impl(ctx, dt_per_scene, stats, true);
}

// ---------------------------------------------------------------------------
// state I/O
// ---------------------------------------------------------------------------

static int download4(bdem_ctx *ctx, const double4 *src, double *dst, int comps) {
  std::vector<double4> h(ctx->S.n_pad);
  HIP_TRY(hipMemcpyAsync(h.data(), src, h.size() * sizeof(double4), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < ctx->S.n; ++i) {
    const double4 v = h[ctx->p_int[i]];
    const double a[4] = {v.x, v.y, v.z, v.w};
    for (int c = 0; c < comps; ++c) dst[comps * i + c] = a[c];
  }
  return BDEM_OK;
}

static int upload4(bdem_ctx *ctx, double4 *dst, const double *src, int comps) {
  std::vector<double4> h(ctx->S.n_pad);
  HIP_TRY(hipMemcpyAsync(h.data(), dst, h.size() * sizeof(double4), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < ctx->S.n; ++i) {
    double a[4] = {0, 0, 0, 0};
    for (int c = 0; c < comps; ++c) a[c] = src[comps * i + c];
    h[ctx->p_int[i]] = make_double4(a[0], a[1], a[2], a[3]);
  }
  HIP_TRY(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(double4), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return BDEM_OK;
}

static bool unit_quats(const double *q, int n) {
  for (int i = 0; i < n; ++i) {
    const double s = std::sqrt(q[4 * i] * q[4 * i] + q[4 * i + 1] * q[4 * i + 1] + q[4 * i + 2] * q[4 * i + 2] +
                               q[4 * i + 3] * q[4 * i + 3]);
    if (!std::isfinite(s) || std::fabs(s - 1.0) > 1e-6) return false;
  }
  return true;
}
static bool finite(const double *a, size_t n) {
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(a[k])) return false;
  return true;
}

extern "C" int bdem_get_state(const bdem_ctx *cctx, double *pos, double *quat, double *vel,
                              double *qvel, uint8_t *alive) {
  bdem_ctx *ctx = const_cast<bdem_ctx *>(cctx);
  if (!ctx) return BDEM_E_INVALID;
  int rc;
  if (pos && (rc = download4(ctx, ctx->d.pn, pos, 3))) return rc;
  if (quat && (rc = download4(ctx, ctx->d.qn, quat, 4))) return rc;
  if (vel && (rc = download4(ctx, ctx->d.vn, vel, 3))) return rc;
  if (qvel && (rc = download4(ctx, ctx->d.wn, qvel, 4))) return rc;
  if (alive && ctx->S.nb > 0) {
    std::vector<uint8_t> h(ctx->S.nb_pad);
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->d.alive, h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < ctx->S.nb; ++k) alive[k] = h[ctx->b_int[k]];
  }
  return BDEM_OK;
}

extern "C" int bdem_set_state(bdem_ctx *ctx, const double *pos, const double *quat, const double *vel,
                              const double *qvel, const uint8_t *alive) {
  if (!ctx) return BDEM_E_INVALID;
  const int n = ctx->S.n;
  if (quat && !unit_quats(quat, n)) return fail(ctx, BDEM_E_INVALID, "non-unit quaternion");
  if ((pos && !finite(pos, 3 * (size_t)n)) || (vel && !finite(vel, 3 * (size_t)n)) ||
      (qvel && !finite(qvel, 4 * (size_t)n)))
    return fail(ctx, BDEM_E_NONFINITE, "non-finite state");
  int rc;
  if (pos && (rc = upload4(ctx, ctx->d.pn, pos, 3))) return rc;
  if (quat && (rc = upload4(ctx, ctx->d.qn, quat, 4))) return rc;
  if (vel && (rc = upload4(ctx, ctx->d.vn, vel, 3))) return rc;
  if (qvel && (rc = upload4(ctx, ctx->d.wn, qvel, 4))) return rc;
  if (alive && ctx->S.nb > 0) {
    std::vector<uint8_t> h(ctx->S.nb_pad);
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->d.alive, h.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    for (int64_t k = 0; k < ctx->S.nb; ++k) h[ctx->b_int[k]] = alive[k] ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(ctx->d.alive, h.data(), h.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
  }
  return BDEM_OK;
}

// ---------------------------------------------------------------------------
// objective / gradient / Hessian at a given state
// ---------------------------------------------------------------------------

template <typename T>
static void expand_blocks(const std::vector<T> &hd, const std::vector<T> &ho, bdem_ctx *ctx,
                          double *hdiag36, double *hoff36) {
  auto up = [](int r, int c) { return r <= c ? r * 6 - (r * (r - 1)) / 2 + (c - r) : c * 6 - (c * (c - 1)) / 2 + (r - c); };
  if (hdiag36)
    for (int i = 0; i < ctx->S.n; ++i) {
      const T *src = hd.data() + (size_t)ctx->p_int[i] * 21;
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) hdiag36[36 * (size_t)i + r * 6 + c] = double(src[up(r, c)]);
    }
  if (hoff36)
    for (int64_t k = 0; k < ctx->S.nb; ++k) {
      const T *src = ho.data() + (size_t)ctx->b_int[k] * 36;
      for (int e = 0; e < 36; ++e) hoff36[36 * (size_t)k + e] = double(src[e]);
    }
}

extern "C" int bdem_energy_grad_hess(bdem_ctx *ctx, double dt, int32_t what, const double *pos_eval,
                                     const double *quat_eval, double *energy, double *grad6,
                                     double *hdiag36, double *hoff36) {
  if (!ctx) return BDEM_E_INVALID;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, BDEM_E_INVALID, "dt must be > 0");
  const int n = ctx->S.n, NS = ctx->S.n_scenes, NP = ctx->S.n_pad;
  if (quat_eval && !unit_quats(quat_eval, n)) return fail(ctx, BDEM_E_INVALID, "non-unit quaternion");
  if (pos_eval && !finite(pos_eval, 3 * (size_t)n)) return fail(ctx, BDEM_E_NONFINITE, "non-finite state");
  hipStream_t st = ctx->stream;
  DevPtrs &d = ctx->d;
  const bool mixed = ctx->S.mixed, hess = (what & BDEM_EGH_H) != 0, psd = (what & BDEM_EGH_PSD) != 0;
  const bool pot = (what & BDEM_EGH_POTENTIAL_ONLY) != 0;
  for (int s = 0; s < NS; ++s) {
    SceneCtl &c = ctx->h_ctl[s];
    std::memset(&c, 0, sizeof(c));
    c.dt = dt;
    c.inv_dt2 = 1.0 / (dt * dt);
    c.kc = ctx->scene_kc[s];
    c.kself = ctx->scene_kself[s];
    c.cmargin = ctx->scene_cmargin[s];
    c.ccell = ctx->scene_ccell[s];
    c.newton_active = 1;
  }
  HIP_TRY(hipMemcpyAsync(d.ctl, ctx->h_ctl, NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(d.degenerate, 0, sizeof(int), st));
  launch_predict(d, false, st);
  int rc;
  if ((rc = contact_candidates(ctx))) return rc;
  launch_step_target(d, ctx->P, st);
  launch_copy_state_to_iterate(d, st);
  if (pos_eval && (rc = upload4(ctx, d.px, pos_eval, 3))) return rc;
  if (quat_eval && (rc = upload4(ctx, d.qx, quat_eval, 4))) return rc;
  const bool gn = (what & BDEM_EGH_GN) != 0;
  if (gn && !hess) return fail(ctx, BDEM_E_INVALID, "BDEM_EGH_GN needs BDEM_EGH_H");
  const bool rows = gn || (hess && psd && ctx->opt.hessian == BDEM_HESS_GAUSS_NEWTON && (what & BDEM_EGH_PCG_MATRIX));
  if (rows) {
    launch_bond_energy(d, false, ctx->P.midpoint != 0, st);
    launch_particle_energy(d, ctx->P, pot, st);
    launch_rows_eval(d, ctx->P, mixed, ctx->P.midpoint != 0, pot, st);
  } else {
    launch_bond_eval(d, mixed, psd, hess, ctx->P.midpoint != 0, st);
    launch_particle_eval(d, ctx->P, mixed, hess, pot, st);
  }
  launch_newton_check(d, ctx->P, 1, rows, st);
  launch_count_active(d, NS, 0, st);
  if ((rc = read_counters(ctx))) return rc;
  if (ctx->h_counters[3] > 0) return fail(ctx, BDEM_E_DEGENERATE, "|q_i + q_j| < 1e-6 in a bond");
  HIP_TRY(hipMemcpyAsync(ctx->h_ctl, d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost, st));
  std::vector<double> z;
  if (grad6) {
    z.resize((size_t)NP * 6);
    HIP_TRY(hipMemcpyAsync(z.data(), d.z, z.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (hess && (hdiag36 || hoff36)) {
    const size_t nbs = std::max(ctx->S.nb_pad, 1);
    if (mixed) {
      std::vector<float> hd((size_t)NP * 21), ho(nbs * 36);
      HIP_TRY(hipMemcpyAsync(hd.data(), d.hdiag, hd.size() * 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(ho.data(), d.hoff, ho.size() * 4, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      expand_blocks(hd, ho, ctx, hdiag36, hoff36);
    } else {
      std::vector<double> hd((size_t)NP * 21), ho(nbs * 36);
      HIP_TRY(hipMemcpyAsync(hd.data(), d.hdiag, hd.size() * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipMemcpyAsync(ho.data(), d.hoff, ho.size() * 8, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      expand_blocks(hd, ho, ctx, hdiag36, hoff36);
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (grad6)
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 6; ++c) grad6[6 * (size_t)i + c] = z[(size_t)ctx->p_int[i] * 6 + c];
  if (energy) {
    double e = 0.0;
    for (int s = 0; s < NS; ++s) e += ctx->h_ctl[s].phi;
    *energy = e;
  }
  for (int s = 0; s < NS; ++s)
    if (ctx->h_ctl[s].status == ST_NONFINITE) return fail(ctx, BDEM_E_NONFINITE, "non-finite objective");
  return BDEM_OK;
}

extern "C" int bdem_precond_apply(bdem_ctx *ctx, double dt, const double *pos_eval,
                                  const double *quat_eval, const double *in6, double *out6) {
  if (!ctx || !in6 || !out6) return BDEM_E_INVALID;
  const int n = ctx->S.n, NS = ctx->S.n_scenes, NP = ctx->S.n_pad;
  // the projected reduced Hessian at the evaluation state (as bdem_energy_grad_hess)
  int rc = bdem_energy_grad_hess(ctx, dt, BDEM_EGH_H | BDEM_EGH_PSD | BDEM_EGH_PCG_MATRIX, pos_eval,
                                 quat_eval, nullptr, nullptr, nullptr, nullptr);
  if (rc < 0) return rc;
  hipStream_t st = ctx->stream;
  DevPtrs &d = ctx->d;
  if (ctx->amg) {
    launch_amg_setup(d, ctx->amg_d, ctx->amg_hl.data(), NS, ctx->S.mixed, st);
    launch_amg_couple(d, ctx->amg_d, ctx->S.mixed, st);
  }
  // r = in (internal order), every scene active, then u = M^-1 r
  std::vector<double> r((size_t)NP * 6, 0.0), u((size_t)NP * 6);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 6; ++c) r[(size_t)ctx->p_int[i] * 6 + c] = in6[6 * (size_t)i + c];
  HIP_TRY(hipMemcpyAsync(d.cr, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ctx->h_ctl, d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int sc = 0; sc < NS; ++sc) ctx->h_ctl[sc].cg_active = 1;
  HIP_TRY(hipMemcpyAsync(d.ctl, ctx->h_ctl, NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
  if (ctx->amg) {
    launch_amg_vcycle(d, ctx->amg_d, ctx->amg_hl.data(), NS, ctx->S.mixed, ctx->spmv_variant, false, false, st);
  } else {
    // block-Jacobi: the PCG initialisation computes u = D^-1 r from r = -z
    HIP_TRY(hipMemcpyAsync(d.z, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice, st));
    launch_cg_init(d, ctx->S.mixed, st);
  }
  HIP_TRY(hipMemcpyAsync(u.data(), d.cs, u.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 6; ++c) out6[6 * (size_t)i + c] = u[(size_t)ctx->p_int[i] * 6 + c];
  if (!ctx->amg)   // k_cg_init took r = -z
    for (size_t k = 0; k < 6 * (size_t)n; ++k) out6[k] = -out6[k];
  return BDEM_OK;
}

extern "C" int bdem_hess_apply(bdem_ctx *ctx, double dt, const double *pos_eval,
                               const double *quat_eval, const double *in6, double *out6) {
  if (!ctx || !in6 || !out6) return BDEM_E_INVALID;
  const int n = ctx->S.n, NS = ctx->S.n_scenes, NP = ctx->S.n_pad;
  // the projected reduced Hessian at the evaluation state (as bdem_energy_grad_hess)
  int rc = bdem_energy_grad_hess(ctx, dt, BDEM_EGH_H | BDEM_EGH_PSD | BDEM_EGH_PCG_MATRIX, pos_eval,
                                 quat_eval, nullptr, nullptr, nullptr, nullptr);
  if (rc < 0) return rc;
  hipStream_t st = ctx->stream;
  DevPtrs &d = ctx->d;
  // u = in (internal order; padding rows zero), every scene active, then w = H u
  std::vector<double> u((size_t)NP * 6, 0.0), w((size_t)NP * 6);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 6; ++c) u[(size_t)ctx->p_int[i] * 6 + c] = in6[6 * (size_t)i + c];
  HIP_TRY(hipMemcpyAsync(d.cs, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(d.cr, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(ctx->h_ctl, d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int sc = 0; sc < NS; ++sc) ctx->h_ctl[sc].cg_active = 1;
  HIP_TRY(hipMemcpyAsync(d.ctl, ctx->h_ctl, NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
  launch_spmv(d, ctx->S.mixed, ctx->spmv_variant, st);
  if (ctx->P.contact) launch_contact_spmv(d, ctx->P, st);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(w.data(), d.cAp, w.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 6; ++c) out6[6 * (size_t)i + c] = w[(size_t)ctx->p_int[i] * 6 + c];
  return BDEM_OK;
}

extern "C" int bdem_break_bonds(bdem_ctx *ctx, int64_t *n_broken, uint8_t *alive_out) {
  if (!ctx) return BDEM_E_INVALID;
  hipStream_t st = ctx->stream;
  int64_t broken = 0;
  if (ctx->S.nb_pad > 0) {
    launch_bond_fracture(ctx->d, st);
    const int nt = ctx->S.nb_pad / TILE;
    std::vector<int> cnt(nt);
    HIP_TRY(hipMemcpyAsync(cnt.data(), ctx->d.part_cnt, nt * sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int v : cnt) broken += v;
  }
  if (n_broken) *n_broken = broken;
  if (alive_out) return bdem_get_state(ctx, nullptr, nullptr, nullptr, nullptr, alive_out);
  return BDEM_OK;
}

extern "C" int bdem_contact_pairs(const bdem_ctx *ctx, int64_t cap, int32_t *pairs, int64_t *count) {
  if (!ctx || cap < 0 || (cap > 0 && !pairs)) return BDEM_E_INVALID;
  std::vector<std::pair<int, int>> out;
  if (ctx->S.contact) {
    const int NP = ctx->S.n_pad;
    std::vector<int> nc(NP), cand((size_t)NP * CMAXC);
    if (hipMemcpy(nc.data(), ctx->d.ncand, NP * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(cand.data(), ctx->d.cand, cand.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      return BDEM_E_HIP;
    std::vector<int> user(NP, -1);
    for (int i = 0; i < ctx->S.n; ++i) user[ctx->p_int[i]] = i;
    for (int r = 0; r < NP; ++r)
      for (int k = 0; k < nc[r]; ++k) {
        const int a = user[r], b = user[cand[(size_t)r * CMAXC + k]];
        if (a >= 0 && b >= 0 && a < b) out.push_back({a, b});
      }
    std::sort(out.begin(), out.end());
  }
  if (count) *count = (int64_t)out.size();
  for (int64_t k = 0; k < cap && k < (int64_t)out.size(); ++k) {
    pairs[2 * k] = out[k].first;
    pairs[2 * k + 1] = out[k].second;
  }
  return BDEM_OK;
}

// ---------------------------------------------------------------------------
// launch-shape autotuning
// ---------------------------------------------------------------------------

static void fill_tuning(const bdem_ctx *ctx, bdem_tuning *t) {
  spmv_shape(ctx->spmv_variant, &t->spmv_threads, &t->spmv_trips);
  t->update_rows = update_rows(ctx->upd_variant);
  t->cg_chunk = ctx->opt.cg_chunk;
  t->use_graph = ctx->opt.use_graph;
  t->pad_ = 0;
  t->spmv_us = ctx->tune_us[0];
  t->update_us = ctx->tune_us[1];
  t->pcg_us_per_iter = ctx->tune_us[2];
}

extern "C" int bdem_get_tuning(const bdem_ctx *ctx, bdem_tuning *out) {
  if (!ctx || !out) return BDEM_E_INVALID;
  fill_tuning(ctx, out);
  return BDEM_OK;
}

extern "C" int bdem_set_tuning(bdem_ctx *ctx, const bdem_tuning *t) {
  if (!ctx || !t) return BDEM_E_INVALID;
  int sv = -1, uv = -1;
  for (int v = 0; v < spmv_variants(); ++v) {
    int nt, u;
    spmv_shape(v, &nt, &u);
    if (nt == t->spmv_threads && u == t->spmv_trips) sv = v;
  }
  for (int v = 0; v < update_variants(); ++v)
    if (update_rows(v) == t->update_rows) uv = v;
  if (sv < 0 || uv < 0 || t->cg_chunk < 1 || (t->use_graph != 0 && t->use_graph != 1))
    return fail(ctx, BDEM_E_INVALID, "no such launch shape");
  ctx->spmv_variant = sv;
  ctx->upd_variant = uv;
  ctx->opt.cg_chunk = t->cg_chunk;
  ctx->opt.use_graph = t->use_graph;
  drop_cg_graphs(ctx);
  return BDEM_OK;
}

// Times every candidate on this handle's own matrix and keeps the fastest:
// the Hessian is assembled at the prediction of a step of length dt_per_scene
// (as the first Newton iteration does), then each SpMV shape, each update
// tile and each PCG polling mode is timed with HIP events.  Every candidate
// computes the same bits, so the choice never changes a result.  The
// simulation state is not modified.
extern "C" int bdem_autotune(bdem_ctx *ctx, const double *dt_per_scene, bdem_tuning *out) {
  if (!ctx || !dt_per_scene) return BDEM_E_INVALID;
  const int NS = ctx->S.n_scenes;
  for (int s = 0; s < NS; ++s)
    if (!(dt_per_scene[s] > 0.0) || !std::isfinite(dt_per_scene[s])) return fail(ctx, BDEM_E_INVALID, "dt must be > 0");
  hipStream_t st = ctx->stream;
  DevPtrs &d = ctx->d;
  const bool mixed = ctx->S.mixed;
  const int prof = ctx->profiling;
  ctx->profiling = 0;
  struct Restore { bdem_ctx *c; int p; ~Restore() { c->profiling = p; } } restore{ctx, prof};
  for (int s = 0; s < NS; ++s) {
    SceneCtl &c = ctx->h_ctl[s];
    std::memset(&c, 0, sizeof(c));
    c.dt = dt_per_scene[s];
    c.inv_dt2 = 1.0 / (dt_per_scene[s] * dt_per_scene[s]);
    c.kc = ctx->scene_kc[s];
    c.kself = ctx->scene_kself[s];
    c.cmargin = ctx->scene_cmargin[s];
    c.ccell = ctx->scene_ccell[s];
    c.newton_active = 1;
  }
  HIP_TRY(hipMemcpyAsync(d.ctl, ctx->h_ctl, NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemsetAsync(d.degenerate, 0, sizeof(int), st));
  launch_predict(d, true, st);
  {
    const int rc = contact_candidates(ctx);
    if (rc) return rc;
  }
  launch_step_target(d, ctx->P, st);
  launch_evaluation(ctx, true, true, true, false);
  if (ctx->amg) {
    launch_amg_setup(d, ctx->amg_d, ctx->amg_hl.data(), NS, mixed, st);
    launch_amg_couple(d, ctx->amg_d, mixed, st);
  }
  launch_newton_check(d, ctx->P, 1, rows_path(ctx, true), st);
  launch_count_active(d, NS, 0, st);
  int rc = read_counters(ctx);
  if (rc) return rc;
  if (ctx->h_counters[3] > 0) return fail(ctx, BDEM_E_DEGENERATE, "|q_i + q_j| < 1e-6 in a bond");
  if (ctx->h_counters[0] == 0) {   // nothing to solve at this state: keep the current shapes
    if (out) fill_tuning(ctx, out);
    return BDEM_OK;
  }
  std::vector<SceneCtl> saved(NS), quiet(NS);
  HIP_TRY(hipMemcpyAsync(saved.data(), d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  quiet = saved;
  for (auto &c : quiet) { c.alpha = 0.0; c.beta = 0.0; }   // repeated updates leave x, r unchanged
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  struct EvGuard { hipEvent_t a, b; ~EvGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } eg{e0, e1};
  auto time_it = [&](auto &&launch, int reps) -> double {
    launch();
    launch();
    (void)hipEventRecord(e0, st);
    for (int k = 0; k < reps; ++k) launch();
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    return 1e3 * ms / reps;
  };
  HIP_TRY(hipMemcpyAsync(d.ctl, quiet.data(), NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
  launch_cg_init(d, mixed, st);
  // update tile and SpMV shape are timed as the pair the PCG loop runs: the
  // update's streams decide how much of the matrix the SpMV finds in cache.
  // Shapes differ by a few percent, so each pair keeps the better of two
  // passes over all pairs.
  const int nu = update_variants(), nsv = spmv_variants();
  std::vector<double> pair_us(nu * nsv, 1e300);
  for (int pass = 0; pass < 2; ++pass)
    for (int vu = 0; vu < nu; ++vu)
      for (int vs = 0; vs < nsv; ++vs) {
        const double us = time_it([&] {
          launch_cg_update(d, mixed, vu, st, !ctx->amg);
          launch_spmv(d, mixed, vs, st, SPMV_DOTS_WU);
        }, 20);
        pair_us[vu * nsv + vs] = std::min(pair_us[vu * nsv + vs], us);
      }
  double best = 1e300;
  for (int k = 0; k < nu * nsv; ++k)
    if (pair_us[k] < best) { best = pair_us[k]; ctx->upd_variant = k / nsv; ctx->spmv_variant = k % nsv; }
  ctx->tune_us[0] = time_it([&] { launch_spmv(d, mixed, ctx->spmv_variant, st, SPMV_DOTS_WU); }, 5);
  ctx->tune_us[1] = time_it([&] { launch_cg_update(d, mixed, ctx->upd_variant, st, !ctx->amg); }, 5);
  HIP_TRY(hipGetLastError());
  // PCG polling: each candidate runs the same solve from x = 0
  const int modes[][2] = {{1, 0}, {4, 0}, {4, 1}, {16, 1}};
  best = 1e300;
  const int chunk0 = ctx->opt.cg_chunk, graph0 = ctx->opt.use_graph;
  int bc = chunk0, bg = graph0;
  for (const auto &m : modes) {
    ctx->opt.cg_chunk = m[0];
    ctx->opt.use_graph = m[1];
    drop_cg_graphs(ctx);
    HIP_TRY(hipMemcpyAsync(d.ctl, saved.data(), NS * sizeof(SceneCtl), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(e0, st));
    rc = run_pcg(ctx);
    if (rc) return rc;
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    std::vector<SceneCtl> after(NS);
    HIP_TRY(hipMemcpy(after.data(), d.ctl, NS * sizeof(SceneCtl), hipMemcpyDeviceToHost));
    int iters = 1;
    for (const auto &c : after) iters = std::max(iters, c.cg_it);
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    const double us = 1e3 * ms / iters;
    if (us < best) { best = us; bc = m[0]; bg = m[1]; ctx->tune_us[2] = us; }
  }
  ctx->opt.cg_chunk = bc;
  ctx->opt.use_graph = bg;
  drop_cg_graphs(ctx);
  if (out) fill_tuning(ctx, out);
  return BDEM_OK;
}

extern "C" int bdem_set_profiling(bdem_ctx *ctx, int32_t enable) {
  if (!ctx) return BDEM_E_INVALID;
  if (enable < 0 || enable > 2) return fail(ctx, BDEM_E_INVALID, "profiling level must be 0, 1 or 2");
  ctx->profiling = enable;
  return BDEM_OK;
}

extern "C" int bdem_profile_counts(const bdem_ctx *ctx, int32_t *bond_launches, int32_t *spmv_launches) {
  if (!ctx) return BDEM_E_INVALID;
  if (bond_launches) *bond_launches = ctx->prof_cnt[0];
  if (spmv_launches) *spmv_launches = ctx->prof_cnt[1];
  return BDEM_OK;
}
