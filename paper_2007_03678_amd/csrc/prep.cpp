// Host-side ligand preparation: validation, torsion tree, internal atom
// order and intramolecular pair list.
//
// Readings of the method (the paper's genotype is translation, orientation
// and the torsions of the ligand's rotatable bonds, Sec. 1.1):
//   * bonds form a tree; rigid fragments are the pieces left when the
//     rotatable bonds are cut;
//   * the root is the atom nearest the reference centroid (lowest index on
//     ties); each torsion's root-side atom is a, its leaf-side atom b, and it
//     moves the atoms whose path to the root passes through b;
//   * intramolecular pairs: atoms in different fragments at bond distance
//     >= 4 (1-2, 1-3, 1-4 excluded).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "ad_internal.h"

namespace ad {

namespace {

int fail(std::string *err, const char *msg) {
  if (err) *err = msg;
  return AD_E_INVALID;
}

struct UnionFind {
  std::vector<int> p;
  explicit UnionFind(int n) : p(n) {
    for (int i = 0; i < n; ++i) p[i] = i;
  }
  int find(int x) {
    while (p[x] != x) x = p[x] = p[p[x]];
    return x;
  }
  bool unite(int a, int b) {
    a = find(a);
    b = find(b);
    if (a == b) return false;
    p[a] = b;
    return true;
  }
};

}  // namespace

int prepare_ligand(const ad_ligand &L, const ad_forcefield &ff, const int *type_to_map, PreparedLigand *out,
                   std::string *err) {
  const int n = L.n_atoms;
  if (n < 1 || n > kMaxAtoms) return fail(err, "atom count must be 1..128");
  if (L.n_bonds != n - 1) return fail(err, "a tree of n atoms needs n-1 bonds");
  if (!L.type_id || !L.charge || !L.xyz) return fail(err, "missing atom arrays");
  if (n > 1 && (!L.bonds || !L.rotatable)) return fail(err, "missing bond arrays");
  for (int i = 0; i < n; ++i) {
    if (L.type_id[i] < 0 || L.type_id[i] >= ff.n_types) return fail(err, "atom type out of range");
    if (!std::isfinite(L.charge[i]) || !std::isfinite(L.xyz[3 * i]) || !std::isfinite(L.xyz[3 * i + 1]) ||
        !std::isfinite(L.xyz[3 * i + 2]))
      return fail(err, "non-finite atom data");
  }
  // adjacency with bond ids
  std::vector<std::vector<std::pair<int, int>>> adj(n);
  UnionFind all(n), rigid(n);
  int n_tor = 0;
  for (int b = 0; b < L.n_bonds; ++b) {
    int u = L.bonds[2 * b], v = L.bonds[2 * b + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) return fail(err, "bond index out of range");
    if (!all.unite(u, v)) return fail(err, "bonds contain a cycle or a duplicate");
    adj[u].push_back({v, b});
    adj[v].push_back({u, b});
    if (L.rotatable[b]) ++n_tor;
    else rigid.unite(u, v);
  }
  if (n_tor > kMaxTor) return fail(err, "more than 32 rotatable bonds");
  for (int b = 0; b < L.n_bonds; ++b)
    if (L.rotatable[b] && (adj[L.bonds[2 * b]].size() < 2 || adj[L.bonds[2 * b + 1]].size() < 2))
      return fail(err, "a rotatable bond ends in a terminal atom");
  if (type_to_map) {
    for (int i = 0; i < n; ++i)
      if (type_to_map[L.type_id[i]] < 0) {
        if (err) *err = "an atom type has no grid map";
        return AD_E_NOMAP;
      }
  }
  if (!out) return AD_OK;

  // centroid and root atom
  double c[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) c[d] += L.xyz[3 * i + d];
  for (int d = 0; d < 3; ++d) c[d] /= n;
  int root = 0;
  double best = INFINITY;
  for (int i = 0; i < n; ++i) {
    double r2 = 0;
    for (int d = 0; d < 3; ++d) r2 += (L.xyz[3 * i + d] - c[d]) * (L.xyz[3 * i + d] - c[d]);
    if (r2 < best) {
      best = r2;
      root = i;
    }
  }

  // depth-first preorder from the root (children by ascending input index);
  // owner torsion and subtree size per atom
  std::vector<int> order, pos(n, -1), parent(n, -1), pbond(n, -1), owner(n, -1), depth(n, 0);
  std::vector<int> tor_of_bond(L.n_bonds, -1);
  {
    int k = 0;
    for (int b = 0; b < L.n_bonds; ++b)
      if (L.rotatable[b]) tor_of_bond[b] = k++;
  }
  std::vector<int> stack = {root};
  while (!stack.empty()) {
    int u = stack.back();
    stack.pop_back();
    pos[u] = (int)order.size();
    order.push_back(u);
    std::vector<std::pair<int, int>> kids;
    for (auto &e : adj[u])
      if (e.first != parent[u]) kids.push_back(e);
    std::sort(kids.begin(), kids.end());
    for (int s = (int)kids.size() - 1; s >= 0; --s) {
      int v = kids[s].first, b = kids[s].second;
      parent[v] = u;
      pbond[v] = b;
      depth[v] = depth[u] + 1;
      owner[v] = tor_of_bond[b] >= 0 ? tor_of_bond[b] : owner[u];
      stack.push_back(v);
    }
  }
  std::vector<int> subtree(n, 1);
  for (int s = n - 1; s > 0; --s) subtree[parent[order[s]]] += subtree[order[s]];

  PreparedLigand &P = *out;
  P = PreparedLigand();
  P.n_atoms = n;
  P.n_tor = n_tor;
  P.perm = order;
  {
    std::vector<int> seen(n, 0);
    int nf = 0;
    for (int i = 0; i < n; ++i) {
      int r = rigid.find(i);
      if (!seen[r]) {
        seen[r] = 1;
        ++nf;
      }
    }
    P.n_frag = nf;
  }
  P.geo.resize(n);
  P.info.resize(n);
  for (int s = 0; s < n; ++s) {
    int i = order[s];
    for (int d = 0; d < 3; ++d) P.geo[s].y[d] = (double)L.xyz[3 * i + d] - c[d];
    P.geo[s].pad = 0;
    P.info[s].map = type_to_map ? type_to_map[L.type_id[i]] : 0;
    P.info[s].q = L.charge[i];
    P.info[s].owner = owner[i];
    P.info[s].type = (int16_t)L.type_id[i];
    P.info[s].slot = -1;
  }
  // torsions in input order
  P.tors.resize(n_tor);
  for (int b = 0; b < L.n_bonds; ++b) {
    int k = tor_of_bond[b];
    if (k < 0) continue;
    int u = L.bonds[2 * b], v = L.bonds[2 * b + 1];
    int bb = parent[v] == u ? v : u;   // leaf side: the child in the rooted tree
    int aa = bb == v ? u : v;
    TorRec &t = P.tors[k];
    double len2 = 0;
    for (int d = 0; d < 3; ++d) {
      t.o[d] = (double)L.xyz[3 * aa + d] - c[d];
      double dd = (double)L.xyz[3 * bb + d] - (double)L.xyz[3 * aa + d];
      t.u[d] = dd;
      len2 += dd * dd;
    }
    double len = std::sqrt(len2);
    for (int d = 0; d < 3; ++d) t.u[d] /= len;
    t.inv_len = 1.0 / len;
    t.parent = owner[aa];
    t.s = pos[bb];
    t.e = pos[bb] + subtree[bb];
    t.a = pos[aa];
    t.b = pos[bb];
    t.depth = 0;
  }
  // prefix-sum slots: the last atom takes slot 0, every other atom where a
  // moving set ends (e - 1) or starts after (s - 1) one slot in atom order
  {
    std::vector<int> need;
    for (int k = 0; k < n_tor; ++k) {
      if (P.tors[k].e - 1 != n - 1) need.push_back(P.tors[k].e - 1);
      if (P.tors[k].s > 0) need.push_back(P.tors[k].s - 1);
    }
    std::sort(need.begin(), need.end());
    need.erase(std::unique(need.begin(), need.end()), need.end());
    P.info[n - 1].slot = 0;
    for (size_t q = 0; q < need.size(); ++q) P.info[need[q]].slot = (int16_t)(q + 1);
    for (int k = 0; k < n_tor; ++k) {
      P.tors[k].e_slot = P.info[P.tors[k].e - 1].slot;
      P.tors[k].s_slot = P.tors[k].s > 0 ? P.info[P.tors[k].s - 1].slot : -1;
    }
  }
  // nesting depth: torsions on the path root -> b, this one included
  for (int k = 0; k < n_tor; ++k) {
    int d = 1;
    for (int q = P.tors[k].parent; q >= 0; q = P.tors[q].parent) ++d;
    P.tors[k].depth = d;
    P.max_depth = std::max(P.max_depth, d);
  }
  // torsions moving each atom, summed over atoms
  for (int i = 0; i < n; ++i)
    for (int q = owner[i]; q >= 0; q = P.tors[q].parent) ++P.depth_sum;
  // bond distances by breadth-first search from every atom (n <= 128)
  std::vector<std::vector<int>> dist(n, std::vector<int>(n, -1));
  for (int s0 = 0; s0 < n; ++s0) {
    std::vector<int> q = {s0};
    dist[s0][s0] = 0;
    for (size_t h = 0; h < q.size(); ++h)
      for (auto &e : adj[q[h]])
        if (dist[s0][e.first] < 0) {
          dist[s0][e.first] = dist[s0][q[h]] + 1;
          q.push_back(e.first);
        }
  }
  // pair list in "rotation" order over internal indices (i, i+k mod n), so
  // that consecutive pairs touch distinct atoms
  const double w_el_ke = ff.w_el * ff.coulomb;
  for (int k = 1; k <= n / 2; ++k) {
    for (int si = 0; si < n; ++si) {
      int sj = (si + k) % n;
      if (2 * k == n && sj < si) continue;   // each pair once when n is even
      int i = order[si], j = order[sj];
      if (rigid.find(i) == rigid.find(j) || dist[i][j] < 4) continue;
      int ti = L.type_id[i], tj = L.type_id[j];
      double qi = L.charge[i], qj = L.charge[j];
      double Si = ff.solpar[ti] + ff.qasp * std::fabs(qi), Sj = ff.solpar[tj] + ff.qasp * std::fabs(qj);
      PairRec r;
      r.ijt = (uint32_t)si | ((uint32_t)sj << 8) | ((uint32_t)(ti * ff.n_types + tj) << 16);
      r.qq = (float)(w_el_ke * qi * qj);
      r.dsv = (float)(ff.w_sol * (Si * ff.vol[tj] + Sj * ff.vol[ti]));
      r.pad = 0;
      P.pairs.push_back(r);
    }
  }
  return AD_OK;
}

void build_lj_table(const ad_forcefield &ff, std::vector<LJRec> *out) {
  const int T = ff.n_types;
  out->assign((size_t)T * T, LJRec{0, 0, 0, 0});
  for (int i = 0; i < T; ++i)
    for (int j = 0; j < T; ++j) {
      int acc = -1;
      if (ff.hbrole[i] == 1 && ff.hbrole[j] == 2) acc = j;
      if (ff.hbrole[i] == 2 && ff.hbrole[j] == 1) acc = i;
      LJRec r;
      if (acc >= 0) {
        double R = ff.Rhb[acc], e = ff.epshb[acc];
        double R10 = std::pow(R, 10.0);
        r.A = (float)(ff.w_hb * 5.0 * e * R10 * R * R);
        r.B = (float)(ff.w_hb * 6.0 * e * R10);
        r.r0 = (float)R;
        r.hb = 1.0f;
      } else {
        double R = 0.5 * (ff.Rii[i] + ff.Rii[j]), e = std::sqrt(ff.epsii[i] * ff.epsii[j]);
        double R6 = std::pow(R, 6.0);
        r.A = (float)(ff.w_vdw * e * R6 * R6);
        r.B = (float)(ff.w_vdw * 2.0 * e * R6);
        r.r0 = (float)R;
        r.hb = 0.0f;
      }
      (*out)[(size_t)i * T + j] = r;
    }
}

FFConst make_ffconst(const ad_forcefield &ff) {
  const double log2e = 1.4426950408889634;
  FFConst c;
  double B = ff.diel_eps0 - ff.diel_A;
  c.diel_A = (float)ff.diel_A;
  c.diel_B = (float)B;
  c.diel_k = (float)ff.diel_k;
  c.diel_lB_log2e = (float)(ff.diel_lambda * B * log2e);
  c.ds_log2e = (float)(log2e / (2.0 * ff.sigma * ff.sigma));
  c.inv_s2 = (float)(1.0 / (ff.sigma * ff.sigma));
  c.diel_c1 = (float)(ff.diel_k * B * ff.diel_lambda * B);
  c.half_smooth = (float)(0.5 * ff.smooth);
  c.r_floor2 = (float)(ff.r_floor * ff.r_floor);
  c.w_tor = (float)ff.w_tor;
  c.n_types = ff.n_types;
  c.k_out = ff.k_out;
  return c;
}

}  // namespace ad

namespace ad {

uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Pre-screen inputs of one ligand in the internal atom order: 32 features
// per atom (one-hot type, q, |q|, one-hot degree 0..3 / >=4, rotatable bonds
// at the atom / 2, constant 1), rounded to BF16, and up to kMaxDeg neighbour
// indices per atom (0xff = none).  Returns false if an atom has more
// neighbours than that.
bool featurize(const ad_ligand &L, const std::vector<int> &perm, std::vector<uint16_t> *X,
               std::vector<uint8_t> *nbr) {
  const int n = L.n_atoms;
  std::vector<int> pos(n);
  for (int s = 0; s < n; ++s) pos[perm[s]] = s;
  std::vector<int> deg(n, 0), rot(n, 0);
  nbr->assign((size_t)n * kMaxDeg, 0xff);
  for (int b = 0; b < L.n_bonds; ++b) {
    const int u = L.bonds[2 * b], v = L.bonds[2 * b + 1];
    if (deg[u] >= kMaxDeg || deg[v] >= kMaxDeg) return false;
    (*nbr)[(size_t)pos[u] * kMaxDeg + deg[u]] = (uint8_t)pos[v];
    (*nbr)[(size_t)pos[v] * kMaxDeg + deg[v]] = (uint8_t)pos[u];
    ++deg[u];
    ++deg[v];
    if (L.rotatable[b]) {
      ++rot[u];
      ++rot[v];
    }
  }
  X->assign((size_t)n * kFeat, 0);
  for (int s = 0; s < n; ++s) {
    const int i = perm[s];
    uint16_t *x = &(*X)[(size_t)s * kFeat];
    x[L.type_id[i]] = f32_to_bf16(1.0f);
    x[16] = f32_to_bf16(L.charge[i]);
    x[17] = f32_to_bf16(std::fabs(L.charge[i]));
    x[18 + std::min(deg[i], 4)] = f32_to_bf16(1.0f);
    x[23] = f32_to_bf16(0.5f * rot[i]);
    x[31] = f32_to_bf16(1.0f);
  }
  return true;
}

}  // namespace ad
