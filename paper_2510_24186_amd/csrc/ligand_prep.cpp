// Host-side ligand preparation: atom typing, rigid fragments, torsion tree,
// intra-ligand pair list and the depth-first packing used by the kernels.
//
// The DOFs are translation, rotation and one torsion per rotatable bond
// (Methods, "Conformation sampling"; N_tor in E_screen).  The tree rules
// (root of smallest height, breadth-first torsion order, >= 4-bond pairs in
// different fragments) are stated in include/dock.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <set>

#include "dock_internal.h"

namespace dock {

namespace {

// Type radii (Angstrom) and flags; order C_H C_P N_P N_D N_A O_A O_DA Cl_H.
const double kRadius[kTypes] = {1.9, 1.9, 1.8, 1.8, 1.8, 1.7, 1.7, 1.8};
const bool kHydrophobic[kTypes] = {true, false, false, false, false, false, false, true};
const bool kDonor[kTypes] = {false, false, false, true, false, false, true, false};
const bool kAcceptor[kTypes] = {false, false, false, false, true, true, true, false};

enum { T_C_H, T_C_P, T_N_P, T_N_D, T_N_A, T_O_A, T_O_DA, T_CL_H };

std::vector<int> bfs_levels(const std::vector<std::vector<int>>& adj, int src) {
  std::vector<int> d(adj.size(), -1);
  std::deque<int> q{src};
  d[src] = 0;
  while (!q.empty()) {
    int u = q.front();
    q.pop_front();
    for (int v : adj[u])
      if (d[v] < 0) {
        d[v] = d[u] + 1;
        q.push_back(v);
      }
  }
  return d;
}

}  // namespace

void type_pair_table(int preset, TypePair table[kTypes * kTypes]) {
  for (int a = 0; a < kTypes; ++a)
    for (int b = 0; b < kTypes; ++b) {
      TypePair& tp = table[a * kTypes + b];
      bool hb = (kDonor[a] && kAcceptor[b]) || (kAcceptor[a] && kDonor[b]);
      bool hyd = kHydrophobic[a] && kHydrophobic[b];
      tp.rsum64 = kRadius[a] + kRadius[b];
      tp.dclash64 = (preset == DOCK_PRESET_TRIDS && hb) ? 2.6 : tp.rsum64;
      tp.rsum = float(tp.rsum64);
      tp.dclash = float(tp.dclash64);
      tp.dclash2 = tp.dclash * tp.dclash;
      tp.flags = (hb ? 1u : 0u) | (hyd ? 2u : 0u);
    }
}

void preset_weights(int preset, float* w, int* K) {
  if (preset == DOCK_PRESET_TRIDS) {
    const float v[3] = {0.2f, 10.0f, 0.6f};
    std::memcpy(w, v, sizeof v);
    *K = 3;
  } else {
    const float v[5] = {-0.0356f, -0.00516f, 0.840f, -0.0351f, -0.587f};
    std::memcpy(w, v, sizeof v);
    *K = 5;
  }
}

int prepare_ligand(int n, const uint8_t* element, const uint8_t* n_h, const float* xyz,
                   int n_bonds, const int32_t* bonds, const uint8_t* rotatable,
                   const float* box_min, const float* box_max, LigandHost& L, std::string& err) {
  if (n < 1) {
    err = "ligand has no atoms";
    return DOCK_E_TOPOLOGY;
  }
  if (n > kMaxAtoms) {
    err = "ligand has " + std::to_string(n) + " atoms > " + std::to_string(kMaxAtoms);
    return DOCK_E_LIMIT;
  }
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(xyz[i])) {
      err = "non-finite ligand coordinate";
      return DOCK_E_TOPOLOGY;
    }
  for (int i = 0; i < n; ++i)
    if (element[i] > 3) {
      err = "unknown element code " + std::to_string(element[i]);
      return DOCK_E_ARG;
    }
  std::vector<std::vector<int>> adj(n), rigid(n);
  std::set<std::pair<int, int>> seen;
  int n_rot = 0;
  for (int b = 0; b < n_bonds; ++b) {
    int i = bonds[2 * b], j = bonds[2 * b + 1];
    if (i < 0 || j < 0 || i >= n || j >= n || i == j) {
      err = "bad bond (" + std::to_string(i) + ", " + std::to_string(j) + ")";
      return DOCK_E_TOPOLOGY;
    }
    auto key = std::make_pair(std::min(i, j), std::max(i, j));
    if (!seen.insert(key).second) {
      err = "duplicate bond";
      return DOCK_E_TOPOLOGY;
    }
    adj[i].push_back(j);
    adj[j].push_back(i);
    if (rotatable[b]) {
      ++n_rot;
    } else {
      rigid[i].push_back(j);
      rigid[j].push_back(i);
    }
  }
  {
    auto d = bfs_levels(adj, 0);
    for (int v : d)
      if (v < 0) {
        err = "disconnected ligand";
        return DOCK_E_TOPOLOGY;
      }
  }
  if (n_rot > kMaxTors) {
    err = "too many rotatable bonds (" + std::to_string(n_rot) + ")";
    return DOCK_E_LIMIT;
  }
  L = LigandHost();
  L.n_atoms = n;
  L.x0.assign(xyz, xyz + 3 * n);

  // typing
  L.type.resize(n);
  for (int a = 0; a < n; ++a) {
    int e = element[a];
    int t;
    if (e == 0) {
      bool polar = false;
      for (int b : adj[a]) polar |= (element[b] == 1 || element[b] == 2);
      t = polar ? T_C_P : T_C_H;
    } else if (e == 1) {
      t = n_h[a] >= 1 ? T_N_D : (adj[a].size() <= 2 ? T_N_A : T_N_P);
    } else if (e == 2) {
      t = n_h[a] >= 1 ? T_O_DA : T_O_A;
    } else {
      t = T_CL_H;
    }
    L.type[a] = uint8_t(t);
  }

  // rigid fragments, ids in order of their lowest atom
  L.atom_frag.assign(n, -1);
  int F = 0;
  for (int a = 0; a < n; ++a) {
    if (L.atom_frag[a] >= 0) continue;
    auto d = bfs_levels(rigid, a);
    for (int b = 0; b < n; ++b)
      if (d[b] >= 0) L.atom_frag[b] = F;
    ++F;
  }
  L.n_frags = F;
  // fragment tree
  std::vector<std::vector<int>> fadj(F);
  std::set<std::pair<int, int>> fseen;
  std::vector<std::vector<std::pair<int, int>>> fbond(F);  // (neighbour frag, atom in this frag)
  for (int b = 0; b < n_bonds; ++b) {
    if (!rotatable[b]) continue;
    int i = bonds[2 * b], j = bonds[2 * b + 1];
    int fi = L.atom_frag[i], fj = L.atom_frag[j];
    auto key = std::make_pair(std::min(fi, fj), std::max(fi, fj));
    if (fi == fj || !fseen.insert(key).second) {
      err = "rotatable bond inside a ring";
      return DOCK_E_TOPOLOGY;
    }
    fadj[fi].push_back(fj);
    fadj[fj].push_back(fi);
    fbond[fi].push_back({fj, i});
    fbond[fj].push_back({fi, j});
  }
  if (int(fseen.size()) != F - 1) {
    err = "fragment graph is not a tree";
    return DOCK_E_TOPOLOGY;
  }
  for (auto& v : fadj) std::sort(v.begin(), v.end());
  int best = 1 << 30, root = 0;
  for (int f = 0; f < F; ++f) {
    auto d = bfs_levels(fadj, f);
    int h = *std::max_element(d.begin(), d.end());
    if (h < best) {
      best = h;
      root = f;
    }
  }
  L.root = root;
  L.height = best;
  // breadth-first order from the root, children by id
  L.frag_parent.assign(F, -1);
  std::vector<char> vis(F, 0);
  std::deque<int> q{root};
  vis[root] = 1;
  L.bfs.push_back(root);
  while (!q.empty()) {
    int u = q.front();
    q.pop_front();
    for (int v : fadj[u])
      if (!vis[v]) {
        vis[v] = 1;
        L.frag_parent[v] = u;
        L.bfs.push_back(v);
        q.push_back(v);
      }
  }
  auto atom_toward = [&](int f, int other) {
    for (auto& pr : fbond[f])
      if (pr.first == other) return pr.second;
    return -1;
  };
  for (size_t k = 1; k < L.bfs.size(); ++k) {
    int f = L.bfs[k], p = L.frag_parent[f];
    L.tors_frag.push_back(f);
    L.tors_a.push_back(atom_toward(p, f));
    L.tors_b.push_back(atom_toward(f, p));
  }
  L.n_tors = int(L.tors_frag.size());

  // intra-ligand pairs
  for (int i = 0; i < n; ++i) {
    auto d = bfs_levels(adj, i);
    for (int j = i + 1; j < n; ++j)
      if (L.atom_frag[i] != L.atom_frag[j] && d[j] >= 4) {
        L.pair_i.push_back(i);
        L.pair_j.push_back(j);
      }
  }

  // centroid of the root fragment (FP64) and the translation box
  int cnt = 0;
  for (int a = 0; a < n; ++a)
    if (L.atom_frag[a] == root) {
      for (int c = 0; c < 3; ++c) L.c0[c] += double(xyz[3 * a + c]);
      ++cnt;
    }
  for (int c = 0; c < 3; ++c) L.c0[c] /= cnt;
  for (int c = 0; c < 3; ++c) {
    float lo = xyz[c], hi = xyz[c];
    for (int a = 1; a < n; ++a) {
      lo = std::min(lo, xyz[3 * a + c]);
      hi = std::max(hi, xyz[3 * a + c]);
    }
    L.box_min[c] = box_min ? box_min[c] : lo;
    L.box_max[c] = box_max ? box_max[c] : hi;
    if (!(L.box_min[c] <= L.box_max[c]) || !std::isfinite(L.box_min[c]) ||
        !std::isfinite(L.box_max[c])) {
      err = "invalid translation box";
      return DOCK_E_ARG;
    }
  }

  // depth-first pre-order of fragments (children by id) -> atom packing
  std::vector<std::vector<int>> kids(F);
  for (int f : L.bfs)
    if (L.frag_parent[f] >= 0) kids[L.frag_parent[f]].push_back(f);
  for (auto& v : kids) std::sort(v.begin(), v.end());
  std::vector<int> stack{root};
  while (!stack.empty()) {
    int f = stack.back();
    stack.pop_back();
    L.dfs_frag.push_back(f);
    for (auto it = kids[f].rbegin(); it != kids[f].rend(); ++it) stack.push_back(*it);
  }
  L.frag_new.assign(F, -1);
  for (int i = 0; i < F; ++i) L.frag_new[L.dfs_frag[i]] = i;
  L.atom_new.assign(n, -1);
  for (int f : L.dfs_frag)
    for (int a = 0; a < n; ++a)
      if (L.atom_frag[a] == f) {
        L.atom_new[a] = int(L.dfs_atom.size());
        L.dfs_atom.push_back(a);
      }
  return DOCK_OK;
}

}  // namespace dock

namespace dock {

namespace {

// Assigns every pair to one of k passes of at most `width` pairs, with at
// most `cap` pairs per atom and pass.  Pairs of busy atoms go first, each to
// the pass where its two atoms have the fewest pairs so far (then the
// emptiest pass).  A pair that fits nowhere takes the place of a pair that
// blocks it in some pass, which moves to a pass with room for it.  Returns
// false when that also fails (the caller then tries k + 1).
bool assign_passes(int n_atoms, const std::vector<int>& pi, const std::vector<int>& pj, int width, int cap,
                   int k, const std::vector<int>& order, std::vector<int>& pass_of) {
  const size_t P = pi.size();
  std::vector<int> load(size_t(n_atoms) * k, 0), size(k, 0);
  std::vector<std::vector<int>> members(k);
  pass_of.assign(P, -1);
  auto L = [&](int a, int p) -> int& { return load[size_t(a) * k + p]; };
  auto fits = [&](int e, int p) { return size[p] < width && L(pi[e], p) < cap && L(pj[e], p) < cap; };
  auto place = [&](int e, int p) {
    pass_of[e] = p;
    ++L(pi[e], p);
    ++L(pj[e], p);
    ++size[p];
    members[p].push_back(e);
  };
  auto unplace = [&](int e) {
    const int p = pass_of[e];
    pass_of[e] = -1;
    --L(pi[e], p);
    --L(pj[e], p);
    --size[p];
    members[p].erase(std::find(members[p].begin(), members[p].end(), e));
  };
  for (int e : order) {
    const int a = pi[e], b = pj[e];
    int best = -1;
    long best_score = 0;
    for (int p = 0; p < k; ++p) {
      if (!fits(e, p)) continue;
      const long score = long(L(a, p) + L(b, p)) * (width + 1) + size[p];
      if (best < 0 || score < best_score) {
        best = p;
        best_score = score;
      }
    }
    if (best >= 0) {
      place(e, best);
      continue;
    }
    bool done = false;
    for (int p = 0; p < k && !done; ++p) {
      const bool full = size[p] >= width, a_full = L(a, p) >= cap, b_full = L(b, p) >= cap;
      if (a_full && b_full) continue;
      const int blocker = a_full ? a : (b_full ? b : -1);
      const std::vector<int> cand = members[p];
      for (int f : cand) {
        if (blocker >= 0 && pi[f] != blocker && pj[f] != blocker) continue;
        if (blocker < 0 && !full) continue;
        int q = 0;
        while (q < k && (q == p || !fits(f, q))) ++q;
        if (q == k) continue;
        unplace(f);
        place(f, q);
        place(e, p);
        done = true;
        break;
      }
    }
    if (!done) return false;
  }
  return true;
}

// The plan with the fewest passes that the assignment finds for one cap,
// starting from the lower bound max(P / width, max degree / cap).
PassPlan plan_for_cap(int n_atoms, const std::vector<int>& pi, const std::vector<int>& pj, int width, int cap,
                      const std::vector<int>& order, int max_deg) {
  const int P = int(pi.size());
  int k = std::max((P + width - 1) / width, (max_deg + cap - 1) / cap);
  std::vector<int> pass_of;
  // k = P always succeeds (every pair can have a pass of its own)
  while (!assign_passes(n_atoms, pi, pj, width, cap, k, order, pass_of)) ++k;
  PassPlan plan;
  plan.n_pass = k;
  plan.cap = cap;
  plan.slot_i.assign(size_t(k) * width, -1);
  plan.slot_j.assign(size_t(k) * width, -1);
  std::vector<int> fill(k, 0);
  for (int e = 0; e < P; ++e) {
    const int p = pass_of[e];
    const size_t slot = size_t(p) * width + fill[p]++;
    plan.slot_i[slot] = pi[e];
    plan.slot_j[slot] = pj[e];
  }
  return plan;
}

}  // namespace

PassPlan schedule_passes(int n_atoms, const std::vector<int>& pi, const std::vector<int>& pj, int width,
                         int apl) {
  PassPlan plan;
  const size_t P = pi.size();
  if (P == 0) return plan;
  std::vector<int> deg(n_atoms, 0);
  for (size_t p = 0; p < P; ++p) {
    ++deg[pi[p]];
    ++deg[pj[p]];
  }
  const int max_deg = *std::max_element(deg.begin(), deg.end());
  // pairs of busy atoms first (larger endpoint degree, then the smaller one)
  std::vector<int> order(P);
  for (size_t p = 0; p < P; ++p) order[p] = int(p);
  const auto key = [&](int e) {
    const int hi = std::max(deg[pi[e]], deg[pj[e]]), lo = std::min(deg[pi[e]], deg[pj[e]]);
    return long(hi) * (n_atoms + 1) + lo;
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) > key(b); });
  // Each atom's gather reads `cap` entries per pass: 4 or 8 with one atom
  // per lane, 2 or 4 with two (the lane's 16 reads of 8 + 8 would not fit its
  // registers).  Cost of a plan ~ passes x (pair work, about 12 gathered
  // entries' worth, + entries read per lane); the cheapest cap is kept.  A
  // larger cap only pays when the busiest atom, not the slot count, sets the
  // number of passes.
  const int min_pass = (int(P) + width - 1) / width;
  const auto cost = [&](const PassPlan& q) { return q.n_pass * (12 + apl * q.cap); };
  bool have = false;
  for (int cap = apl == 1 ? 4 : 2; cap <= (apl == 1 ? kMaxPull : 4); cap *= 2) {
    if (have && (max_deg + cap / 2 - 1) / (cap / 2) <= min_pass) break;  // the previous cap already met P / width
    PassPlan q = plan_for_cap(n_atoms, pi, pj, width, cap, order, max_deg);
    if (!have || cost(q) < cost(plan)) plan = std::move(q);
    have = true;
  }
  plan.n_pull = apl * width;
  // Orientation: within a pass every atom is the first endpoint of at most
  // half its pairs rounded up, and the second endpoint of at most as many
  // (trails between odd-degree atoms, then closed trails, each pair pointing
  // along its trail).  With at most `cap` pairs per atom, neither list
  // exceeds cap / 2.
  const int half = plan.cap / 2;
  std::vector<std::vector<std::pair<int, int>>> adj(n_atoms);  // (other atom, slot)
  std::vector<char> used(width);
  std::vector<int> next_edge(n_atoms);
  for (int ps = 0; ps < plan.n_pass; ++ps) {
    const size_t base = size_t(ps) * width;
    for (auto& v : adj) v.clear();
    for (int sl = 0; sl < width; ++sl) {
      const int a = plan.slot_i[base + sl], b = plan.slot_j[base + sl];
      if (a < 0) continue;
      adj[a].push_back({b, sl});
      adj[b].push_back({a, sl});
    }
    std::fill(used.begin(), used.end(), 0);
    std::fill(next_edge.begin(), next_edge.end(), 0);
    auto walk = [&](int v) {
      for (;;) {
        while (next_edge[v] < int(adj[v].size()) && used[adj[v][next_edge[v]].second]) ++next_edge[v];
        if (next_edge[v] == int(adj[v].size())) return;
        const auto [w, sl] = adj[v][next_edge[v]];
        used[sl] = 1;
        plan.slot_i[base + sl] = v;  // the pair points from v to w
        plan.slot_j[base + sl] = w;
        v = w;
      }
    };
    for (int v = 0; v < n_atoms; ++v)
      if (adj[v].size() % 2) walk(v);
    for (int v = 0; v < n_atoms; ++v) walk(v);
  }
  // pull lists: per pass and atom, byte k < cap / 2 names a slot where the
  // atom is the first endpoint (+f), byte cap / 2 + k one where it is the
  // second (-f); unused bytes name the zero entry `width`
  const uint64_t none = uint64_t(width) * 0x0101010101010101ull;
  plan.pulls.assign(size_t(plan.n_pass) * plan.n_pull, none);
  std::vector<int> n_plus(n_atoms), n_minus(n_atoms);
  for (int ps = 0; ps < plan.n_pass; ++ps) {
    std::fill(n_plus.begin(), n_plus.end(), 0);
    std::fill(n_minus.begin(), n_minus.end(), 0);
    for (int sl = 0; sl < width; ++sl) {
      const int a = plan.slot_i[size_t(ps) * width + sl], b = plan.slot_j[size_t(ps) * width + sl];
      if (a < 0) continue;
      uint64_t& la = plan.pulls[size_t(ps) * plan.n_pull + a];
      uint64_t& lb = plan.pulls[size_t(ps) * plan.n_pull + b];
      const int ka = 8 * n_plus[a]++, kb = 8 * (half + n_minus[b]++);
      la = (la & ~(0xffull << ka)) | (uint64_t(sl) << ka);
      lb = (lb & ~(0xffull << kb)) | (uint64_t(sl) << kb);
    }
  }
  return plan;
}

}  // namespace dock

namespace dock {

int build_mdn_geometry(int n, const float* xyz, const int32_t* residue, MdnGeometry& g, std::string& err) {
  g = MdnGeometry();
  if (n <= 0) return DOCK_OK;
  int n_res = 0;
  for (int a = 0; a < n; ++a) {
    if (residue[a] < 0) {
      err = "negative residue index";
      return DOCK_E_ARG;
    }
    n_res = std::max(n_res, residue[a] + 1);
  }
  std::vector<int> count(n_res, 0);
  for (int a = 0; a < n; ++a) ++count[residue[a]];
  for (int i = 0; i < n_res; ++i)
    if (count[i] == 0) {
      err = "residue indices must cover 0 .. n_res - 1";
      return DOCK_E_ARG;
    }
  g.n_res = n_res;
  // atoms grouped by residue, in increasing atom index within a residue
  g.res_range.resize(n_res);
  int off = 0;
  for (int i = 0; i < n_res; ++i) {
    g.res_range[i] = make_int2(off, off + count[i]);
    off += count[i];
  }
  std::vector<int> fill(n_res, 0);
  g.res_xyz.resize(n);
  for (int a = 0; a < n; ++a) {
    const int i = residue[a];
    g.res_xyz[g.res_range[i].x + fill[i]++] = make_float4(xyz[3 * a], xyz[3 * a + 1], xyz[3 * a + 2], 0.f);
  }
  // lattice over the receptor box grown by the cutoff and one cell
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) {
    lo[c] = hi[c] = xyz[c];
    for (int a = 1; a < n; ++a) {
      lo[c] = std::min(lo[c], double(xyz[3 * a + c]));
      hi[c] = std::max(hi[c], double(xyz[3 * a + c]));
    }
    lo[c] -= kMdnCutoff + kMdnCell;
    hi[c] += kMdnCutoff + kMdnCell;
    g.origin[c] = float(lo[c]);
    g.dims[c] = int(std::ceil((hi[c] - double(g.origin[c])) / kMdnCell));
  }
  const long long ncell = (long long)g.dims[0] * g.dims[1] * g.dims[2];
  if (ncell > (1ll << 26)) {
    err = "receptor too large for the E_MDN lattice";
    return DOCK_E_LIMIT;
  }
  // residue i is listed in every cell whose box comes within the cutoff
  // (plus 1e-3 A for rounding of the query's cell index) of one of its atoms
  const double reach = kMdnCutoff + 1e-3;
  std::vector<int> stamp(ncell, -1);
  std::vector<std::vector<int>> lists(ncell);
  for (int i = 0; i < n_res; ++i) {
    for (int k = g.res_range[i].x; k < g.res_range[i].y; ++k) {
      const float4 r = g.res_xyz[k];
      const double p[3] = {r.x, r.y, r.z};
      int c0[3], c1[3];
      for (int c = 0; c < 3; ++c) {
        c0[c] = std::max(0, int(std::floor((p[c] - reach - g.origin[c]) / kMdnCell)));
        c1[c] = std::min(g.dims[c] - 1, int(std::floor((p[c] + reach - g.origin[c]) / kMdnCell)));
      }
      for (int z = c0[2]; z <= c1[2]; ++z)
        for (int y = c0[1]; y <= c1[1]; ++y)
          for (int x = c0[0]; x <= c1[0]; ++x) {
            const long long cell = ((long long)z * g.dims[1] + y) * g.dims[0] + x;
            if (stamp[cell] == i) continue;
            const int idx[3] = {x, y, z};
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
              const double b0 = g.origin[c] + double(idx[c]) * kMdnCell, b1 = b0 + kMdnCell;
              const double dd = p[c] < b0 ? b0 - p[c] : (p[c] > b1 ? p[c] - b1 : 0.0);
              d2 += dd * dd;
            }
            if (d2 < reach * reach) {
              stamp[cell] = i;
              lists[cell].push_back(i);
            }
          }
    }
  }
  g.cell_start.resize(ncell + 1);
  g.cell_start[0] = 0;
  for (long long c = 0; c < ncell; ++c) g.cell_start[c + 1] = g.cell_start[c] + int(lists[c].size());
  g.cell_res.reserve(g.cell_start[ncell]);
  for (long long c = 0; c < ncell; ++c) g.cell_res.insert(g.cell_res.end(), lists[c].begin(), lists[c].end());
  return DOCK_OK;
}

}  // namespace dock
