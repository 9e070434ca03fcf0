// Host-side symbolic construction of the aggregation multigrid hierarchy
// (see bdem_amg.hpp).
#include "bdem_amg.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

namespace bdem {

uint64_t amg_cell_key(int64_t x, int64_t y, int64_t z) {
  uint64_t c = 0;
  for (int bit = 20; bit >= 0; --bit)
    c = (c << 3) | ((uint64_t)((x >> bit) & 1) << 2) | ((uint64_t)((y >> bit) & 1) << 1) |
        (uint64_t)((z >> bit) & 1);
  return c;
}

namespace {

uint64_t morton3(int64_t x, int64_t y, int64_t z) { return amg_cell_key(x, y, z); }

// nodes of a level from keys (scene, cell) of the finer nodes: unique keys in
// (scene, Morton(cell)) order; parent of each finer node; children lists
struct Grouping {
  int n = 0;
  std::vector<int> parent, mbeg, mlist, scene;
  std::vector<int64_t> cell;   // 3 per node
};

Grouping group(const std::vector<int> &fscene, const std::vector<int64_t> &fcell,
               const std::vector<char> &real) {
  const int nf = (int)fscene.size();
  std::vector<int> idx;
  idx.reserve(nf);
  for (int i = 0; i < nf; ++i)
    if (real[i]) idx.push_back(i);
  auto key = [&](int i) {
    return std::make_pair(fscene[i], morton3(fcell[3 * i], fcell[3 * i + 1], fcell[3 * i + 2]));
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return key(a) < key(b); });
  Grouping g;
  g.parent.assign(nf, -1);
  for (size_t k = 0; k < idx.size(); ++k) {
    const int i = idx[k];
    if (k == 0 || key(idx[k - 1]) != key(i)) {
      g.scene.push_back(fscene[i]);
      g.cell.insert(g.cell.end(), {fcell[3 * i], fcell[3 * i + 1], fcell[3 * i + 2]});
      g.n++;
    }
    g.parent[i] = g.n - 1;
  }
  g.mbeg.assign(g.n + 1, 0);
  for (int i = 0; i < nf; ++i)
    if (g.parent[i] >= 0) g.mbeg[g.parent[i] + 1]++;
  for (int a = 0; a < g.n; ++a) g.mbeg[a + 1] += g.mbeg[a];
  g.mlist.assign(g.mbeg[g.n], 0);
  std::vector<int> fill(g.mbeg.begin(), g.mbeg.end() - 1);
  for (int i = 0; i < nf; ++i)   // ascending finer index within each node
    if (g.parent[i] >= 0) g.mlist[fill[g.parent[i]]++] = i;
  return g;
}

// coarse pattern from (row, col, src) triples: CSR sorted by (row, col),
// contributions sorted by src
void pattern(int n, std::vector<std::array<int64_t, 3>> &t, AmgHostLevel &L) {
  std::sort(t.begin(), t.end());
  L.row_ptr.assign(n + 1, 0);
  L.col.clear();
  L.slot_row.clear();
  L.gptr.assign(1, 0);
  L.gsrc.clear();
  L.dslot.assign(n, -1);
  for (size_t k = 0; k < t.size(); ++k) {
    const bool fresh = k == 0 || t[k][0] != t[k - 1][0] || t[k][1] != t[k - 1][1];
    if (fresh) {
      if (k > 0) L.gptr.push_back((int)L.gsrc.size());
      const int r = (int)t[k][0], c = (int)t[k][1];
      if (r == c) L.dslot[r] = (int)L.col.size();
      L.col.push_back(c);
      L.slot_row.push_back(r);
      L.row_ptr[r + 1]++;
    }
    L.gsrc.push_back((int)t[k][2]);
  }
  L.gptr.push_back((int)L.gsrc.size());
  for (int r = 0; r < n; ++r) L.row_ptr[r + 1] += L.row_ptr[r];
}

}  // namespace

void amg_build(int n_pad, int n_scenes, const std::vector<double> &pos4,
               const std::vector<uint8_t> &flags, const std::vector<int> &psid,
               const std::vector<int> &scene_pbeg, const std::vector<int> &row_ptr,
               const std::vector<int> &col, const std::vector<double> &lo3,
               const std::vector<double> &h0, AmgHost &H) {
  (void)scene_pbeg;
  H = AmgHost();
  H.lv.resize(1);
  // fine rows: cells of side h0 from the scene's box corner
  std::vector<int64_t> fcell(3 * (size_t)n_pad, 0);
  std::vector<char> real(n_pad, 0);
  std::vector<int> fscene(psid.begin(), psid.end());
  std::vector<int> factive(n_pad, 0);
  for (int r = 0; r < n_pad; ++r) {
    if (flags[r] == 255) continue;
    real[r] = 1;
    factive[r] = flags[r] == 0;
    const int s = psid[r];
    for (int k = 0; k < 3; ++k)
      fcell[3 * r + k] = (int64_t)std::floor((pos4[4 * (size_t)r + k] - lo3[3 * s + k]) / h0[s]);
  }
  H.slot_row0.assign(std::max<size_t>(col.size(), 1), 0);
  for (int r = 0; r < n_pad; ++r)
    for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) H.slot_row0[k] = r;
  // level 1
  Grouping g = group(fscene, fcell, real);
  H.parent0 = g.parent;
  // fine coupling H P: the distinct aggregates of each row's diagonal and
  // off-diagonal columns that are unknowns (P is zero elsewhere), ascending;
  // the off-diagonal sources of an entry in slot order, and per row the
  // entry its diagonal block adds to first (-1: none)
  H.hp_ptr.assign(n_pad + 1, 0);
  H.hp_gptr.assign(1, 0);
  H.hp_self.assign(n_pad, -1);
  {
    std::vector<std::pair<int, int>> src;   // (aggregate, slot; -1: the diagonal)
    for (int r = 0; r < n_pad; ++r) {
      src.clear();
      if (g.parent[r] >= 0 && factive[r]) src.push_back({g.parent[r], -1});
      for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k)
        if (g.parent[col[k]] >= 0 && factive[col[k]]) src.push_back({g.parent[col[k]], k});
      std::stable_sort(src.begin(), src.end(),
                       [](const std::pair<int, int> &x, const std::pair<int, int> &y) { return x.first < y.first; });
      for (size_t k = 0; k < src.size(); ++k) {
        const bool fresh = k == 0 || src[k].first != src[k - 1].first;
        if (fresh && k > 0) H.hp_gptr.push_back((int)H.hp_gsrc.size());
        if (fresh) H.hp_agg.push_back(src[k].first);
        if (src[k].second < 0) H.hp_self[r] = (int)H.hp_agg.size() - 1;
        else H.hp_gsrc.push_back(src[k].second);
      }
      if (!src.empty()) H.hp_gptr.push_back((int)H.hp_gsrc.size());
      H.hp_ptr[r + 1] = (int)H.hp_agg.size();
    }
  }
  int level = 0;
  std::vector<int> prev_scene = fscene, prev_active = factive;
  std::vector<int64_t> prev_cell = fcell;
  std::vector<char> prev_real = real;
  while (true) {
    ++level;
    AmgHostLevel L;
    L.n = g.n;
    L.mbeg = g.mbeg;
    L.mlist = g.mlist;
    L.scene = g.scene;
    L.active.assign(g.n, 0);
    for (size_t i = 0; i < prev_active.size(); ++i)
      if (g.parent[i] >= 0 && prev_active[i]) L.active[g.parent[i]] = 1;
    std::vector<std::array<int64_t, 3>> t;
    if (level == 1) {
      for (int r = 0; r < n_pad; ++r) {
        if (!real[r]) continue;
        const int a = g.parent[r];
        t.push_back({a, a, -1 - (int64_t)r});
        for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) t.push_back({a, g.parent[col[k]], k});
      }
    } else {
      const AmgHostLevel &F = H.lv[level - 1];
      for (int s = 0; s < (int)F.col.size(); ++s)
        t.push_back({g.parent[F.slot_row[s]], g.parent[F.col[s]], s});
    }
    pattern(g.n, t, L);
    H.lv.push_back(std::move(L));
    // stop once every scene has at most AMG_COARSE_MAX nodes
    std::vector<int> per(n_scenes, 0);
    for (int a = 0; a < g.n; ++a) per[g.scene[a]]++;
    const int most = *std::max_element(per.begin(), per.end());
    if (most <= AMG_COARSE_MAX || level == 15) break;
    // next level: cells of twice the side
    std::vector<int64_t> ccell(g.cell.size());
    for (size_t k = 0; k < g.cell.size(); ++k) ccell[k] = g.cell[k] >> 1;
    std::vector<char> creal(g.n, 1);
    Grouping nx = group(g.scene, ccell, creal);
    H.lv[level].parent = nx.parent;
    prev_active = H.lv[level].active;
    g = std::move(nx);
  }
  H.L = level;
  H.lv[level].parent.assign(H.lv[level].n, -1);
  // coarsest: node range and dense block per scene
  const AmgHostLevel &C = H.lv[level];
  H.cbeg.assign(n_scenes + 1, 0);
  for (int a = 0; a < C.n; ++a) H.cbeg[C.scene[a] + 1]++;
  for (int s = 0; s < n_scenes; ++s) H.cbeg[s + 1] += H.cbeg[s];
  // the tail: the first level at which every scene has at most
  // AMG_DENSE_MAX nodes (so are all coarser ones)
  H.Lt = H.L;
  auto most = [&](int l) {
    std::vector<int> nodes(n_scenes, 0);
    for (int a = 0; a < H.lv[l].n; ++a) nodes[H.lv[l].scene[a]]++;
    return *std::max_element(nodes.begin(), nodes.end());
  };
  while (H.Lt > 1 && most(H.Lt - 1) <= AMG_DENSE_MAX) --H.Lt;
  H.tbeg.assign((size_t)(H.L - H.Lt + 1) * (n_scenes + 1), 0);
  H.tmax.assign(H.L + 1, 0);
  for (int l = H.Lt; l <= H.L; ++l) {
    int *tb = H.tbeg.data() + (size_t)(l - H.Lt) * (n_scenes + 1);
    for (int a = 0; a < H.lv[l].n; ++a) tb[H.lv[l].scene[a] + 1]++;
    for (int s = 0; s < n_scenes; ++s) tb[s + 1] += tb[s];
    H.tmax[l] = most(l);
  }
  H.noff.assign(n_scenes + 1, 0);
  for (int s = 0; s < n_scenes; ++s) {
    const int64_t m = 6 * (int64_t)(H.tbeg[s + 1] - H.tbeg[s]);
    H.noff[s + 1] = H.noff[s] + m * m;
  }
  H.coff.assign(n_scenes, 0);
  int64_t off = 0;
  for (int s = 0; s < n_scenes; ++s) {
    H.coff[s] = off;
    const int64_t m = 6 * (int64_t)(H.cbeg[s + 1] - H.cbeg[s]);
    off += m * m;
  }
  H.cdense = std::max<int64_t>(off, 1);
}

}  // namespace bdem
