/*
 * FP64 CPU oracle for the docking hot path -- TEST INFRASTRUCTURE ONLY.
 * Loaded by the tests, the smoke check and the benchmark's CPU-baseline leg;
 * never by the GPU product path, with which it shares no code.
 *
 * The paper (AutoDock-GPU on Summit) names the method -- the AutoDock4
 * scoring function with van der Waals, hydrogen-bond, electrostatic and
 * desolvation terms and the Lamarckian GA with local search (Sec. 1), the
 * ADADELTA local search, nrun runs and the evaluation cap nev (Sec. 1.1),
 * and AutoGrid4 affinity / electrostatic / desolvation maps (Sec. 2.3) -- but
 * prints no formula.  Each function states the reading it implements.  All
 * arithmetic is double precision; map node values are stored as float
 * because the method stores FP32 maps.
 */
#include "oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ===================================================================== */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,     */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).                */
/* ===================================================================== */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; round++) {
    if (round > 0) {
      k0 += 0x9E3779B9u; /* Weyl key schedule */
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Word w of a named stream.  Counter layout (a reading; the paper names no
 * generator): key = seed split in two words; counter = (ligand, run,
 * generation, individual<<16 | stream<<10 | w/4); the word is lane w%4. */
enum { ST_INIT = 0, ST_SELECT = 1, ST_CROSS = 2, ST_MUTATE = 3, ST_LSPICK = 4 };

static uint32_t orc_word(uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen,
                         uint32_t indiv, uint32_t stream, uint32_t w) {
  uint32_t ctr[4] = {lig, run, gen, (indiv << 16) | (stream << 10) | (w >> 2)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[w & 3];
}
/* uniform in [0,1) with 24 random bits (exact in float and double) */
static double orc_unif(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }
/* integer in [0,n) by the multiply-high rule */
static uint32_t orc_randint(uint32_t x, uint32_t n) { return (uint32_t)(((uint64_t)x * n) >> 32); }

uint32_t orc_stream_word(uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen,
                         uint32_t indiv, uint32_t stream, uint32_t w) {
  return orc_word(seed, lig, run, gen, indiv, stream, w);
}

/* ===================================================================== */
/* Pair potentials (Sec. 1: van der Waals, hydrogen bond, electrostatic   */
/* and desolvation terms of the AutoDock4 function).                      */
/* ===================================================================== */

/* Parameters of the repulsion/dispersion term of a type pair.  Reading:
 * donor-acceptor pairs use a 12-10 well C/r^12 - D/r^10 of the acceptor's
 * depth eps_hb at R_hb (C = 5 eps R^12, D = 6 eps R^10); all other pairs a
 * 12-6 well A/r^12 - B/r^6 (A = eps R^12, B = 2 eps R^6) with R the mean of
 * the two radii and eps the geometric mean of the two depths.  The term
 * weight (w_hb or w_vdw) is folded in. */
static void orc_lj_params(const orc_ff *ff, int ti, int tj, double *A, double *B, int *m, double *r0) {
  int acc = -1;
  if (ff->hbrole[ti] == 1 && ff->hbrole[tj] == 2) acc = tj;
  if (ff->hbrole[ti] == 2 && ff->hbrole[tj] == 1) acc = ti;
  if (acc >= 0) {
    double R = ff->Rhb[acc], e = ff->epshb[acc];
    double R2 = R * R, R10 = R2 * R2 * R2 * R2 * R2;
    *A = ff->w_hb * 5.0 * e * R10 * R2;
    *B = ff->w_hb * 6.0 * e * R10;
    *m = 10;
    *r0 = R;
  } else {
    double R = 0.5 * (ff->Rii[ti] + ff->Rii[tj]);
    double e = sqrt(ff->epsii[ti] * ff->epsii[tj]);
    double R2 = R * R, R6 = R2 * R2 * R2;
    *A = ff->w_vdw * e * R6 * R6;
    *B = ff->w_vdw * 2.0 * e * R6;
    *m = 6;
    *r0 = R;
  }
}

/* Smoothed 12-6 / 12-10 term.  Reading of AutoDock's smoothing: within
 * +-smooth/2 of the well minimum r0 the energy is the minimum itself; outside
 * the band the curve is shifted by smooth/2 towards r0.  Distances below
 * r_floor are raised to r_floor. */
double orc_lj(const orc_ff *ff, int ti, int tj, double r, double *dEdr) {
  double A, B, r0;
  int m;
  orc_lj_params(ff, ti, tj, &A, &B, &m, &r0);
  double slope = 1.0;
  if (r < ff->r_floor) { r = ff->r_floor; slope = 0.0; }
  double half = 0.5 * ff->smooth, rr;
  if (r > r0 + half) rr = r - half;
  else if (r < r0 - half) rr = r + half;
  else { rr = r0; slope = 0.0; }
  double i1 = 1.0 / rr, i2 = i1 * i1, i6 = i2 * i2 * i2, i12 = i6 * i6;
  double im = (m == 10) ? i6 * i2 * i2 : i6;
  double E = A * i12 - B * im;
  if (dEdr) *dEdr = slope * (-12.0 * A * i12 + m * B * im) * i1;
  return E;
}

/* Distance-dependent dielectric of Mehler and Solmajer as used by
 * AutoDock4: eps(r) = A + B / (1 + k exp(-lambda B r)), B = eps0 - A. */
double orc_diel(const orc_ff *ff, double r, double *deps) {
  double A = ff->diel_A, B = ff->diel_eps0 - ff->diel_A;
  double lB = ff->diel_lambda * B;
  double e = exp(-lB * r);
  double den = 1.0 + ff->diel_k * e;
  if (deps) *deps = B * ff->diel_k * lB * e / (den * den);
  return A + B / den;
}

/* Screened Coulomb term w_el * k_e * qi qj / (eps(r) r). */
double orc_elec(const orc_ff *ff, double qi, double qj, double r, double *dEdr) {
  double slope = 1.0;
  if (r < ff->r_floor) { r = ff->r_floor; slope = 0.0; }
  double de, eps = orc_diel(ff, r, &de);
  double K = ff->w_el * ff->coulomb * qi * qj;
  double E = K / (eps * r);
  if (dEdr) *dEdr = -slope * K * (eps + r * de) / ((eps * r) * (eps * r));
  return E;
}

/* Desolvation term w_sol (S_i V_j + S_j V_i) exp(-r^2 / (2 sigma^2)) with
 * atomic solvation S = solpar + qasp |q|. */
double orc_desolv(const orc_ff *ff, int ti, double qi, int tj, double qj, double r, double *dEdr) {
  double slope = 1.0;
  if (r < ff->r_floor) { r = ff->r_floor; slope = 0.0; }
  double Si = ff->solpar[ti] + ff->qasp * fabs(qi);
  double Sj = ff->solpar[tj] + ff->qasp * fabs(qj);
  double s2 = ff->sigma * ff->sigma;
  double E = ff->w_sol * (Si * ff->vol[tj] + Sj * ff->vol[ti]) * exp(-r * r / (2.0 * s2));
  if (dEdr) *dEdr = -slope * E * r / s2;
  return E;
}

/* Full intramolecular pair energy: all three terms, no cutoff. */
double orc_pair(const orc_ff *ff, int ti, double qi, int tj, double qj, double r, double *dEdr) {
  double d1 = 0, d2 = 0, d3 = 0;
  double E = orc_lj(ff, ti, tj, r, &d1) + orc_elec(ff, qi, qj, r, &d2) + orc_desolv(ff, ti, qi, tj, qj, r, &d3);
  if (dEdr) *dEdr = d1 + d2 + d3;
  return E;
}

/* ===================================================================== */
/* Grid maps (Sec. 2.3: per-atom-type affinity, electrostatic and         */
/* desolvation maps; Sec. 2.2.3: all maps resident, one per ligand type). */
/* ===================================================================== */

static size_t orc_nodes(const orc_grid *g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }

/* All map values at node (i,j,k) by direct summation over the receptor.
 * Affinity map of ligand type t: sum over atoms within the cutoff of the
 * 12-6/12-10 term plus the type-dependent half of desolvation,
 * w_sol (solpar_t V_a + S_a V_t) g(r); capped at +cap.  Electrostatic map:
 * w_el k_e q_a / (eps(r) r) over all atoms (no cutoff).  Desolvation map:
 * w_sol qasp V_a g(r) within the cutoff.  A ligand atom of type t and
 * charge q then scores map_t + q map_e + |q| map_d, which is exactly its
 * pair sum with the receptor. */
void orc_node_values(const orc_grid *g, int i, int j, int k, double *out) {
  const orc_ff *ff = &g->ff;
  double p[3] = {g->origin[0] + g->h * i, g->origin[1] + g->h * j, g->origin[2] + g->h * k};
  int M = g->n_maps;
  for (int m = 0; m < M + 2; m++) out[m] = 0.0;
  double s2 = ff->sigma * ff->sigma;
  for (int a = 0; a < g->n_rec; a++) {
    double dx = p[0] - g->rec_xyz[3 * a], dy = p[1] - g->rec_xyz[3 * a + 1], dz = p[2] - g->rec_xyz[3 * a + 2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    int ta = g->rec_type[a];
    double qa = g->rec_q[a];
    out[M] += orc_elec(ff, 1.0, qa, r, NULL);
    if (r < ff->cutoff) {
      double rf = r < ff->r_floor ? ff->r_floor : r;
      double gds = exp(-rf * rf / (2.0 * s2));
      double Sa = ff->solpar[ta] + ff->qasp * fabs(qa);
      out[M + 1] += ff->w_sol * ff->qasp * ff->vol[ta] * gds;
      for (int m = 0; m < M; m++) {
        int t = g->map_type[m];
        out[m] += orc_lj(ff, t, ta, r, NULL) + ff->w_sol * (ff->solpar[t] * ff->vol[ta] + Sa * ff->vol[t]) * gds;
      }
    }
  }
  for (int m = 0; m < M; m++)
    if (out[m] > ff->cap) out[m] = ff->cap;
}

static void orc_store_node(orc_grid *g, size_t node, const double *v) {
  size_t nn = orc_nodes(g);
  for (int m = 0; m < g->n_maps + 2; m++) g->vals[m * nn + node] = (float)v[m];
}

/* Make sure node (i,j,k) holds its values (lazy grids compute on demand). */
static void orc_ensure(orc_grid *g, int i, int j, int k) {
  if (!g->have) return;
  size_t node = ((size_t)k * g->n[1] + j) * g->n[0] + i;
  if (g->have[node]) return;
#pragma omp critical(orc_lazy)
  {
    if (!g->have[node]) {
      double v[ORC_MAXT + 2];
      orc_node_values(g, i, j, k, v);
      orc_store_node(g, node, v);
      g->have[node] = 1;
    }
  }
}

orc_grid *orc_grid_create(const orc_ff *ff, const int n[3], double h, const double origin[3],
                          int n_maps, const int *map_types, const float *vals) {
  if (n[0] < 2 || n[1] < 2 || n[2] < 2 || !(h > 0) || n_maps < 0 || n_maps > ORC_MAXT) return NULL;
  orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
  g->ff = *ff;
  for (int d = 0; d < 3; d++) { g->n[d] = n[d]; g->origin[d] = origin[d]; }
  g->h = h;
  g->n_maps = n_maps;
  for (int t = 0; t < ORC_MAXT; t++) g->type_to_map[t] = -1;
  for (int m = 0; m < n_maps; m++) {
    g->map_type[m] = map_types[m];
    if (map_types[m] >= 0 && map_types[m] < ORC_MAXT) g->type_to_map[map_types[m]] = m;
  }
  size_t total = orc_nodes(g) * (size_t)(n_maps + 2);
  g->vals = (float *)calloc(total, sizeof(float));
  if (vals) memcpy(g->vals, vals, total * sizeof(float));
  return g;
}

/* Attach a receptor.  lazy=0 computes every node now (OpenMP over z);
 * lazy=1 computes nodes when first touched. */
void orc_grid_set_receptor(orc_grid *g, int n_rec, const float *xyz, const int *types, const float *q, int lazy) {
  free(g->rec_xyz); free(g->rec_type); free(g->rec_q); free(g->have);
  g->have = NULL;
  g->n_rec = n_rec;
  g->rec_xyz = (double *)malloc(sizeof(double) * 3 * (n_rec > 0 ? n_rec : 1));
  g->rec_type = (int *)malloc(sizeof(int) * (n_rec > 0 ? n_rec : 1));
  g->rec_q = (double *)malloc(sizeof(double) * (n_rec > 0 ? n_rec : 1));
  for (int a = 0; a < n_rec; a++) {
    for (int d = 0; d < 3; d++) g->rec_xyz[3 * a + d] = xyz[3 * a + d];
    g->rec_type[a] = types[a];
    g->rec_q[a] = q[a];
  }
  if (lazy) {
    g->have = (unsigned char *)calloc(orc_nodes(g), 1);
    return;
  }
#pragma omp parallel for schedule(dynamic)
  for (int k = 0; k < g->n[2]; k++) {
    double v[ORC_MAXT + 2];
    for (int j = 0; j < g->n[1]; j++)
      for (int i = 0; i < g->n[0]; i++) {
        orc_node_values(g, i, j, k, v);
        orc_store_node(g, ((size_t)k * g->n[1] + j) * g->n[0] + i, v);
      }
  }
}

/* Copy out the values of node (i,j,k), computing them if the grid is lazy. */
void orc_grid_node(orc_grid *g, int i, int j, int k, float *out) {
  orc_ensure(g, i, j, k);
  size_t nn = orc_nodes(g), node = ((size_t)k * g->n[1] + j) * g->n[0] + i;
  for (int m = 0; m < g->n_maps + 2; m++) out[m] = g->vals[m * nn + node];
}

float *orc_grid_values(orc_grid *g) { return g->vals; }

void orc_grid_free(orc_grid *g) {
  if (!g) return;
  free(g->vals); free(g->have); free(g->rec_xyz); free(g->rec_type); free(g->rec_q);
  free(g);
}

/* Inter-molecular energy of one ligand atom (reading of map use: trilinear
 * interpolation of map_t + q map_e + |q| map_d; a coordinate outside the
 * grid is clamped to the nearest face and a restraint k_out |x - x_c|^2 to
 * the clamped point x_c is added).  Adds dE/dx to grad. */
static double orc_atom_inter(orc_grid *g, int type, double q, const double x[3], double grad[3]) {
  int m = g->type_to_map[type];
  size_t nn = orc_nodes(g);
  double uc[3], f[3];
  int i0[3], clamped[3];
  for (int d = 0; d < 3; d++) {
    double u = (x[d] - g->origin[d]) / g->h, top = g->n[d] - 1;
    clamped[d] = (u < 0.0 || u > top);
    uc[d] = u < 0.0 ? 0.0 : (u > top ? top : u);
    i0[d] = (int)floor(uc[d]);
    if (i0[d] > g->n[d] - 2) i0[d] = g->n[d] - 2;
    f[d] = uc[d] - i0[d];
  }
  double v[2][2][2];
  for (int c = 0; c < 8; c++) {
    int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
    int ii = i0[0] + dx, jj = i0[1] + dy, kk = i0[2] + dz;
    orc_ensure(g, ii, jj, kk);
    size_t node = ((size_t)kk * g->n[1] + jj) * g->n[0] + ii;
    v[dz][dy][dx] = (double)g->vals[m * nn + node] + q * (double)g->vals[g->n_maps * nn + node] +
                    fabs(q) * (double)g->vals[(g->n_maps + 1) * nn + node];
  }
  double E = 0, dEdu[3] = {0, 0, 0};
  for (int dz = 0; dz < 2; dz++)
    for (int dy = 0; dy < 2; dy++)
      for (int dx = 0; dx < 2; dx++) {
        double wx = dx ? f[0] : 1 - f[0], wy = dy ? f[1] : 1 - f[1], wz = dz ? f[2] : 1 - f[2];
        double val = v[dz][dy][dx];
        E += wx * wy * wz * val;
        dEdu[0] += (dx ? 1 : -1) * wy * wz * val;
        dEdu[1] += (dy ? 1 : -1) * wx * wz * val;
        dEdu[2] += (dz ? 1 : -1) * wx * wy * val;
      }
  for (int d = 0; d < 3; d++) {
    if (!clamped[d]) {
      grad[d] += dEdu[d] / g->h;
    } else {
      double dd = x[d] - (g->origin[d] + g->h * uc[d]);
      E += g->ff.k_out * dd * dd;
      grad[d] += 2.0 * g->ff.k_out * dd;
    }
  }
  return E;
}

/* ===================================================================== */
/* Ligand preparation: torsion tree (Sec. 1.1: the genotype's torsions     */
/* are the ligand's rotatable bonds).                                     */
/* ===================================================================== */

static int orc_fail(orc_ligand *L, int code, const char *msg) {
  snprintf(L->msg, sizeof(L->msg), "%s", msg);
  return code;
}

/* Validate and prepare a ligand.  Readings: the bonds form a tree; rigid
 * fragments are the components left after cutting the rotatable bonds; the
 * root fragment holds the atom nearest the reference centroid (lowest index
 * on ties); torsion k (the k-th rotatable bond in input order) has its
 * root-side atom a_k and leaf-side atom b_k, and S_k is the set of atoms on
 * the leaf side; intramolecular pairs are atom pairs in different fragments at
 * bond-path distance >= 4 (1-2, 1-3, 1-4 excluded). */
int orc_ligand_prepare(orc_ligand *L, const orc_ff *ff, int n, int n_bonds, const int *bonds,
                       const unsigned char *rotatable, const int *types, const float *charges,
                       const float *xyz) {
  memset(L, 0, sizeof(*L));
  if (n < 1 || n > ORC_MAXA) return orc_fail(L, ORC_E_INVALID, "atom count out of range");
  if (n_bonds != n - 1) return orc_fail(L, ORC_E_INVALID, "a tree needs n-1 bonds");
  L->n = n;
  static const int NONE = -1;
  int deg[ORC_MAXA] = {0};
  int adj[ORC_MAXA][ORC_MAXA];
  int nadj[ORC_MAXA] = {0};
  int adj_rot[ORC_MAXA][ORC_MAXA];
  for (int i = 0; i < n; i++) {
    if (types[i] < 0 || types[i] >= ff->n_types) return orc_fail(L, ORC_E_INVALID, "atom type out of range");
    if (!isfinite(charges[i]) || !isfinite(xyz[3 * i]) || !isfinite(xyz[3 * i + 1]) || !isfinite(xyz[3 * i + 2]))
      return orc_fail(L, ORC_E_INVALID, "non-finite atom data");
    L->type[i] = types[i];
    L->q[i] = charges[i];
    for (int d = 0; d < 3; d++) L->y[i][d] = xyz[3 * i + d];
  }
  int n_tor = 0;
  for (int b = 0; b < n_bonds; b++) {
    int u = bonds[2 * b], v = bonds[2 * b + 1];
    if (u < 0 || v < 0 || u >= n || v >= n || u == v) return orc_fail(L, ORC_E_INVALID, "bad bond index");
    for (int e = 0; e < nadj[u]; e++)
      if (adj[u][e] == v) return orc_fail(L, ORC_E_INVALID, "duplicate bond");
    adj[u][nadj[u]] = v; adj_rot[u][nadj[u]++] = rotatable[b] ? 1 : 0;
    adj[v][nadj[v]] = u; adj_rot[v][nadj[v]++] = rotatable[b] ? 1 : 0;
    deg[u]++; deg[v]++;
    if (rotatable[b]) n_tor++;
  }
  if (n_tor > ORC_MAXTOR) return orc_fail(L, ORC_E_INVALID, "too many torsions");
  for (int b = 0; b < n_bonds; b++)
    if (rotatable[b] && (deg[bonds[2 * b]] < 2 || deg[bonds[2 * b + 1]] < 2))
      return orc_fail(L, ORC_E_INVALID, "rotatable bond ends in a terminal atom");
  /* connectivity and path distances by breadth-first search from each atom */
  int (*dist)[ORC_MAXA] = L->dist;
  for (int s = 0; s < n; s++) {
    int queue[ORC_MAXA], head = 0, tail = 0;
    for (int i = 0; i < n; i++) dist[s][i] = NONE;
    dist[s][s] = 0;
    queue[tail++] = s;
    while (head < tail) {
      int u = queue[head++];
      for (int e = 0; e < nadj[u]; e++) {
        int v = adj[u][e];
        if (dist[s][v] == NONE) { dist[s][v] = dist[s][u] + 1; queue[tail++] = v; }
      }
    }
    if (tail != n) return orc_fail(L, ORC_E_INVALID, "bonds do not connect all atoms");
  }
  /* rigid fragments: components over non-rotatable bonds */
  for (int i = 0; i < n; i++) L->frag[i] = NONE;
  L->n_frag = 0;
  for (int s = 0; s < n; s++) {
    if (L->frag[s] != NONE) continue;
    int stack[ORC_MAXA], top = 0;
    stack[top++] = s;
    L->frag[s] = L->n_frag;
    while (top) {
      int u = stack[--top];
      for (int e = 0; e < nadj[u]; e++)
        if (!adj_rot[u][e] && L->frag[adj[u][e]] == NONE) {
          L->frag[adj[u][e]] = L->n_frag;
          stack[top++] = adj[u][e];
        }
    }
    L->n_frag++;
  }
  /* rotation centre and root atom */
  for (int d = 0; d < 3; d++) {
    double s = 0;
    for (int i = 0; i < n; i++) s += L->y[i][d];
    L->center[d] = s / n;
  }
  int root = 0;
  double best = 1e300;
  for (int i = 0; i < n; i++) {
    double dx = L->y[i][0] - L->center[0], dy = L->y[i][1] - L->center[1], dz = L->y[i][2] - L->center[2];
    double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < best) { best = r2; root = i; }
  }
  L->root_atom = root;
  /* rotatable bonds on each atom's path from the root */
  int rotcount[ORC_MAXA];
  {
    int queue[ORC_MAXA], head = 0, tail = 0, seen[ORC_MAXA] = {0};
    queue[tail++] = root; seen[root] = 1; rotcount[root] = 0;
    while (head < tail) {
      int u = queue[head++];
      for (int e = 0; e < nadj[u]; e++) {
        int v = adj[u][e];
        if (!seen[v]) { seen[v] = 1; rotcount[v] = rotcount[u] + adj_rot[u][e]; queue[tail++] = v; }
      }
    }
  }
  /* torsions in input order */
  int k = 0;
  for (int b = 0; b < n_bonds; b++) {
    if (!rotatable[b]) continue;
    int u = bonds[2 * b], v = bonds[2 * b + 1];
    int a = dist[root][u] < dist[root][v] ? u : v;
    int bb = (a == u) ? v : u;
    L->tor_a[k] = a;
    L->tor_b[k] = bb;
    L->tor_depth[k] = rotcount[bb];
    /* S_k: atoms whose path to the root passes through b_k */
    for (int i = 0; i < n; i++) L->moves[k][i] = (dist[root][i] == dist[root][bb] + dist[bb][i]) ? 1 : 0;
    k++;
  }
  L->n_tor = n_tor;
  /* deepest first (stable on ties) */
  for (int i = 0; i < n_tor; i++) L->leaf_first[i] = i;
  for (int i = 1; i < n_tor; i++) {
    int x = L->leaf_first[i], j = i - 1;
    while (j >= 0 && L->tor_depth[L->leaf_first[j]] < L->tor_depth[x]) { L->leaf_first[j + 1] = L->leaf_first[j]; j--; }
    L->leaf_first[j + 1] = x;
  }
  /* intramolecular pairs */
  L->n_pairs = 0;
  for (int i = 0; i < n; i++)
    for (int j = i + 1; j < n; j++)
      if (L->frag[i] != L->frag[j] && dist[i][j] >= 4) {
        L->pair_i[L->n_pairs] = i;
        L->pair_j[L->n_pairs] = j;
        L->n_pairs++;
      }
  return ORC_OK;
}

orc_ligand *orc_ligand_new(void) { return (orc_ligand *)calloc(1, sizeof(orc_ligand)); }
void orc_ligand_free(orc_ligand *L) { free(L); }
const char *orc_ligand_msg(const orc_ligand *L) { return L->msg; }
int orc_ligand_info(const orc_ligand *L, int *out /* n, n_tor, n_pairs, n_frag, root_atom */) {
  out[0] = L->n; out[1] = L->n_tor; out[2] = L->n_pairs; out[3] = L->n_frag; out[4] = L->root_atom;
  return 0;
}
void orc_ligand_pairs(const orc_ligand *L, int *pi, int *pj) {
  for (int p = 0; p < L->n_pairs; p++) { pi[p] = L->pair_i[p]; pj[p] = L->pair_j[p]; }
}
void orc_ligand_torsion(const orc_ligand *L, int k, int *a, int *b, int *depth, unsigned char *moves) {
  *a = L->tor_a[k]; *b = L->tor_b[k]; *depth = L->tor_depth[k];
  for (int i = 0; i < L->n; i++) moves[i] = L->moves[k][i];
}

/* ===================================================================== */
/* Pose from genotype.                                                   */
/* ===================================================================== */

/* Rotate point p about the axis through o with unit direction u by angle
 * th (right-handed; Rodrigues' formula). */
static void orc_rotate_about(double p[3], const double o[3], const double u[3], double th) {
  double v[3] = {p[0] - o[0], p[1] - o[1], p[2] - o[2]};
  double c = cos(th), s = sin(th);
  double dot = u[0] * v[0] + u[1] * v[1] + u[2] * v[2];
  double cr[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
  for (int d = 0; d < 3; d++) p[d] = o[d] + v[d] * c + cr[d] * s + u[d] * dot * (1 - c);
}

/* Rotation matrix of the unit quaternion (w,x,y,z). */
static void orc_quat_matrix(const double q[4], double R[3][3]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z);     R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z);     R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y);     R[2][1] = 2 * (y * z + w * x);     R[2][2] = 1 - 2 * (x * x + y * y);
}

/* Pose (reading of the genotype of Sec. 1.1, translation + orientation +
 * torsions): starting from the reference conformation, each torsion k turns
 * the atoms of S_k by theta_k about the axis a_k -> b_k, deepest torsion
 * first, each step using the current positions of a_k and b_k; then
 * x = R(q/|q|) (y - c) + t with c the reference centroid.  order=1 applies
 * the torsions root first instead (same pose; used as a cross-check). */
void orc_pose(const orc_ligand *L, const double *geno, int order, double *xyz) {
  double y[ORC_MAXA][3];
  memcpy(y, L->y, sizeof(double) * 3 * L->n);
  for (int s = 0; s < L->n_tor; s++) {
    int k = order == 0 ? L->leaf_first[s] : L->leaf_first[L->n_tor - 1 - s];
    double o[3] = {y[L->tor_a[k]][0], y[L->tor_a[k]][1], y[L->tor_a[k]][2]};
    double u[3] = {y[L->tor_b[k]][0] - o[0], y[L->tor_b[k]][1] - o[1], y[L->tor_b[k]][2] - o[2]};
    double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (int d = 0; d < 3; d++) u[d] /= nu;
    for (int i = 0; i < L->n; i++)
      if (L->moves[k][i]) orc_rotate_about(y[i], o, u, geno[7 + k]);
  }
  double qn = sqrt(geno[3] * geno[3] + geno[4] * geno[4] + geno[5] * geno[5] + geno[6] * geno[6]);
  double q[4] = {geno[3] / qn, geno[4] / qn, geno[5] / qn, geno[6] / qn};
  double R[3][3];
  orc_quat_matrix(q, R);
  for (int i = 0; i < L->n; i++) {
    double v[3] = {y[i][0] - L->center[0], y[i][1] - L->center[1], y[i][2] - L->center[2]};
    for (int d = 0; d < 3; d++) xyz[3 * i + d] = R[d][0] * v[0] + R[d][1] * v[1] + R[d][2] * v[2] + geno[d];
  }
}

/* ===================================================================== */
/* Energy and analytic gradient.                                         */
/* ===================================================================== */

/* E = sum_i inter_i + sum_pairs pair(r_ij).  Gradient layout (stride 40):
 * [0..2] dE/dt, [3..5] dE/domega for a world-frame rotation vector omega
 * applied as q <- exp(omega/2) (x) q, [6] = 0, [7+k] dE/dtheta_k.  With
 * g_i = dE/dx_i: dE/dt = sum g_i; dE/domega = sum (x_i - t) x g_i;
 * dE/dtheta_k = u_k . sum_{i in S_k} (x_i - x_{a_k}) x g_i, u_k the unit
 * axis a_k -> b_k in the posed ligand.  terms = {inter (with restraint),
 * intra, score = inter + w_tor * T}.  A non-finite genotype gives NaN. */
int orc_score(const orc_ligand *L, orc_grid *g, const double *geno, double *E_out, double *grad,
              double *terms, double *xyz_out) {
  int n = L->n;
  for (int i = 0; i < 7 + L->n_tor; i++)
    if (!isfinite(geno[i])) {
      *E_out = NAN;
      if (grad) for (int j = 0; j < ORC_STRIDE; j++) grad[j] = NAN;
      if (terms) terms[0] = terms[1] = terms[2] = NAN;
      return ORC_OK;
    }
  for (int i = 0; i < n; i++)
    if (g->type_to_map[L->type[i]] < 0) return ORC_E_NOMAP;
  double x[ORC_MAXA * 3], gi[ORC_MAXA][3];
  orc_pose(L, geno, 0, x);
  if (xyz_out) memcpy(xyz_out, x, sizeof(double) * 3 * n);
  double Einter = 0, Eintra = 0;
  for (int i = 0; i < n; i++) {
    gi[i][0] = gi[i][1] = gi[i][2] = 0;
    Einter += orc_atom_inter(g, L->type[i], L->q[i], &x[3 * i], gi[i]);
  }
  for (int p = 0; p < L->n_pairs; p++) {
    int i = L->pair_i[p], j = L->pair_j[p];
    double d[3] = {x[3 * i] - x[3 * j], x[3 * i + 1] - x[3 * j + 1], x[3 * i + 2] - x[3 * j + 2]};
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dEdr;
    Eintra += orc_pair(&g->ff, L->type[i], L->q[i], L->type[j], L->q[j], r, &dEdr);
    if (r > 0)
      for (int c = 0; c < 3; c++) {
        gi[i][c] += dEdr * d[c] / r;
        gi[j][c] -= dEdr * d[c] / r;
      }
  }
  *E_out = Einter + Eintra;
  if (terms) { terms[0] = Einter; terms[1] = Eintra; terms[2] = Einter + g->ff.w_tor * L->n_tor; }
  if (!grad) return ORC_OK;
  for (int j = 0; j < ORC_STRIDE; j++) grad[j] = 0;
  for (int i = 0; i < n; i++) {
    double r[3] = {x[3 * i] - geno[0], x[3 * i + 1] - geno[1], x[3 * i + 2] - geno[2]};
    for (int c = 0; c < 3; c++) grad[c] += gi[i][c];
    grad[3] += r[1] * gi[i][2] - r[2] * gi[i][1];
    grad[4] += r[2] * gi[i][0] - r[0] * gi[i][2];
    grad[5] += r[0] * gi[i][1] - r[1] * gi[i][0];
  }
  for (int k = 0; k < L->n_tor; k++) {
    const double *xa = &x[3 * L->tor_a[k]], *xb = &x[3 * L->tor_b[k]];
    double u[3] = {xb[0] - xa[0], xb[1] - xa[1], xb[2] - xa[2]};
    double nu = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double tq[3] = {0, 0, 0};
    for (int i = 0; i < n; i++) {
      if (!L->moves[k][i]) continue;
      double r[3] = {x[3 * i] - xa[0], x[3 * i + 1] - xa[1], x[3 * i + 2] - xa[2]};
      tq[0] += r[1] * gi[i][2] - r[2] * gi[i][1];
      tq[1] += r[2] * gi[i][0] - r[0] * gi[i][2];
      tq[2] += r[0] * gi[i][1] - r[1] * gi[i][0];
    }
    grad[7 + k] = (u[0] * tq[0] + u[1] * tq[1] + u[2] * tq[2]) / nu;
  }
  return ORC_OK;
}

/* Many poses (float genotypes, stride 40), optionally in parallel.  Lazy
 * grids are computed on demand under a lock. */
int orc_score_batch(orc_ligand **ligs, const int *lig_idx, int n_poses, orc_grid *g, const float *genos,
                    double *E, double *grads, double *terms, int n_threads) {
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 4) reduction(| : err)
  for (int p = 0; p < n_poses; p++) {
    double geno[ORC_STRIDE];
    for (int j = 0; j < ORC_STRIDE; j++) geno[j] = genos[(size_t)p * ORC_STRIDE + j];
    err |= -orc_score(ligs[lig_idx[p]], g, geno, &E[p], grads ? &grads[(size_t)p * ORC_STRIDE] : NULL,
                      terms ? &terms[(size_t)p * 3] : NULL, NULL);
  }
  return err ? ORC_E_NOMAP : ORC_OK;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ===================================================================== */
/* Lamarckian GA with ADADELTA local search (Sec. 1: LGA whose locally    */
/* improved poses enter crossover; Sec. 1.1: ADADELTA, nrun, nev).        */
/* Hyper-parameters are not given by the paper; the readings below are    */
/* the documented defaults of this implementation.                        */
/* ===================================================================== */

static void orc_qmul(const double a[4], const double b[4], double out[4]) {
  out[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  out[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  out[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  out[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}
static void orc_qnormalize(double q[4]) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; i++) q[i] /= n;
}
/* q <- exp(omega/2) (x) q, renormalised */
static void orc_apply_rotvec(double q[4], const double w[3]) {
  double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  double s = th > 1e-300 ? sin(0.5 * th) / th : 0.5;
  double r[4] = {cos(0.5 * th), s * w[0], s * w[1], s * w[2]}, out[4];
  orc_qmul(r, q, out);
  orc_qnormalize(out);
  memcpy(q, out, sizeof(out));
}
static double orc_wrap(double th) { return th - 2.0 * PI * floor((th + PI) / (2.0 * PI)); }

void orc_genotype_rotate(double *geno, const double w[3]) { orc_apply_rotvec(&geno[3], w); }

/* Initial individual (reading): t uniform over the grid box, q uniform on
 * the rotation group by Shoemake's subgroup algorithm, each theta uniform in
 * [-pi, pi).  Draws: words 0-2 translation, 3-5 orientation, 6+k torsions. */
void orc_init_individual(const orc_ligand *L, const orc_grid *g, uint64_t seed, uint32_t lig, uint32_t run,
                         uint32_t indiv, double *geno) {
  for (int j = 0; j < ORC_STRIDE; j++) geno[j] = 0;
  for (int d = 0; d < 3; d++)
    geno[d] = g->origin[d] + orc_unif(orc_word(seed, lig, run, 0, indiv, ST_INIT, d)) * g->h * (g->n[d] - 1);
  double u1 = orc_unif(orc_word(seed, lig, run, 0, indiv, ST_INIT, 3));
  double u2 = orc_unif(orc_word(seed, lig, run, 0, indiv, ST_INIT, 4));
  double u3 = orc_unif(orc_word(seed, lig, run, 0, indiv, ST_INIT, 5));
  double a = sqrt(1 - u1), b = sqrt(u1);
  geno[3] = a * sin(2 * PI * u2);
  geno[4] = a * cos(2 * PI * u2);
  geno[5] = b * sin(2 * PI * u3);
  geno[6] = b * cos(2 * PI * u3);
  for (int k = 0; k < L->n_tor; k++)
    geno[7 + k] = -PI + 2 * PI * orc_unif(orc_word(seed, lig, run, 0, indiv, ST_INIT, 6 + k));
}

/* Index of the lowest energy (lowest index on ties). */
static int orc_argmin(const double *E, int n) {
  int b = 0;
  for (int i = 1; i < n; i++)
    if (E[i] < E[b]) b = i;
  return b;
}

/* Binary tournament: two uniform candidates; the better (lower energy,
 * lower index on ties) wins with probability tour_p. */
static int orc_tournament(const double *E, int pop, double tour_p, uint32_t w0, uint32_t w1, uint32_t w2) {
  int a = (int)orc_randint(w0, (uint32_t)pop), b = (int)orc_randint(w1, (uint32_t)pop);
  int better = (E[a] < E[b] || (E[a] == E[b] && a < b)) ? a : b;
  int worse = better == a ? b : a;
  return orc_unif(w2) < tour_p ? better : worse;
}

/* One GA generation: individual 0 is the previous best (energy carried
 * over); every other child is built from two tournament winners A and B by
 * two-point crossover over gene blocks {t, q, theta_0, ..., theta_{T-1}}
 * (with probability cx_rate; blocks lo..hi inclusive come from B, lo/hi the
 * sorted draws), then mutated slot by slot with probability mut_rate:
 * translation axes by U(-mut_t, mut_t), the orientation by a rotation of
 * U(-mut_rot, mut_rot) about a uniform axis, torsions by
 * U(-mut_theta, mut_theta) (wrapped to [-pi, pi)).  Children are left
 * unevaluated (new_E = NaN) except the elite. */
void orc_ga_offspring(const orc_ligand *L, const orc_dock_params *p, uint64_t seed, uint32_t lig, uint32_t run,
                      uint32_t gen, int pop, const double *old_geno, const double *old_E, double *new_geno,
                      double *new_E) {
  int best = orc_argmin(old_E, pop);
  memcpy(&new_geno[0], &old_geno[(size_t)best * ORC_STRIDE], sizeof(double) * ORC_STRIDE);
  new_E[0] = old_E[best];
  int T = L->n_tor, nb = 2 + T;
  for (int i = 1; i < pop; i++) {
    uint32_t s[6];
    for (int w = 0; w < 6; w++) s[w] = orc_word(seed, lig, run, gen, i, ST_SELECT, w);
    int A = orc_tournament(old_E, pop, p->tour_p, s[0], s[1], s[2]);
    int B = orc_tournament(old_E, pop, p->tour_p, s[3], s[4], s[5]);
    double *c = &new_geno[(size_t)i * ORC_STRIDE];
    memcpy(c, &old_geno[(size_t)A * ORC_STRIDE], sizeof(double) * ORC_STRIDE);
    if (orc_unif(orc_word(seed, lig, run, gen, i, ST_CROSS, 0)) < p->cx_rate) {
      int c1 = (int)orc_randint(orc_word(seed, lig, run, gen, i, ST_CROSS, 1), (uint32_t)nb);
      int c2 = (int)orc_randint(orc_word(seed, lig, run, gen, i, ST_CROSS, 2), (uint32_t)nb);
      int lo = c1 < c2 ? c1 : c2, hi = c1 < c2 ? c2 : c1;
      const double *b = &old_geno[(size_t)B * ORC_STRIDE];
      for (int blk = lo; blk <= hi; blk++) {
        if (blk == 0) { c[0] = b[0]; c[1] = b[1]; c[2] = b[2]; }
        else if (blk == 1) { c[3] = b[3]; c[4] = b[4]; c[5] = b[5]; c[6] = b[6]; }
        else c[7 + blk - 2] = b[7 + blk - 2];
      }
    }
    /* mutation: slot s uses Philox block s = words 4s..4s+3 */
    int nslots = 4 + T;
    for (int slot = 0; slot < nslots; slot++) {
      uint32_t w0 = orc_word(seed, lig, run, gen, i, ST_MUTATE, 4 * slot);
      if (!(orc_unif(w0) < p->mut_rate)) continue;
      double a1 = orc_unif(orc_word(seed, lig, run, gen, i, ST_MUTATE, 4 * slot + 1));
      if (slot < 3) {
        c[slot] += (2 * a1 - 1) * p->mut_t;
      } else if (slot == 3) {
        double a2 = orc_unif(orc_word(seed, lig, run, gen, i, ST_MUTATE, 4 * slot + 2));
        double a3 = orc_unif(orc_word(seed, lig, run, gen, i, ST_MUTATE, 4 * slot + 3));
        double z = 2 * a1 - 1, phi = 2 * PI * a2, rho = sqrt(1 - z * z);
        double ang = (2 * a3 - 1) * p->mut_rot;
        double w[3] = {ang * rho * cos(phi), ang * rho * sin(phi), ang * z};
        orc_apply_rotvec(&c[3], w);
      } else {
        int k = slot - 4;
        c[7 + k] = orc_wrap(c[7 + k] + (2 * a1 - 1) * p->mut_theta);
      }
    }
    new_E[i] = NAN;
  }
}

/* Individuals that receive local search this generation: n_ls distinct
 * indices from 1..pop-1 by a partial Fisher-Yates shuffle (word s draws the
 * swap partner of position s). */
void orc_ls_pick(uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen, int pop, int n_ls, int *picked) {
  int idx[ORC_MAXPOP];
  int m = pop - 1;
  for (int i = 0; i < m; i++) idx[i] = i + 1;
  for (int s = 0; s < n_ls; s++) {
    int r = s + (int)orc_randint(orc_word(seed, lig, run, gen, 0, ST_LSPICK, s), (uint32_t)(m - s));
    int tmp = idx[s]; idx[s] = idx[r]; idx[r] = tmp;
    picked[s] = idx[s];
  }
}

/* ADADELTA local search (Sec. 1.1; Zeiler 2012) over the degrees of freedom
 * (t, omega, theta): per component E[g^2] <- rho E[g^2] + (1-rho) g^2,
 * dx = -sqrt(E[dx^2] + eps) / sqrt(E[g^2] + eps) * g,
 * E[dx^2] <- rho E[dx^2] + (1-rho) dx^2; t += dx_t,
 * q <- exp(dx_omega/2) (x) q, theta += dx_theta (wrapped).  Each of the
 * `iters` iterations evaluates energy and gradient once; the best evaluated
 * genotype is returned (Lamarckian write-back happens in the caller). */
int orc_adadelta(const orc_ligand *L, orc_grid *g, const orc_dock_params *p, const double *geno_in, int iters,
                 double *best_geno, double *best_E) {
  double x[ORC_STRIDE], grad[ORC_STRIDE];
  memcpy(x, geno_in, sizeof(x));
  int nd = 6 + L->n_tor;
  double Eg2[6 + ORC_MAXTOR] = {0}, Edx2[6 + ORC_MAXTOR] = {0};
  *best_E = INFINITY;
  memcpy(best_geno, x, sizeof(x));
  for (int it = 0; it < iters; it++) {
    double E;
    int rc = orc_score(L, g, x, &E, grad, NULL, NULL);
    if (rc) return rc;
    if (E < *best_E) { *best_E = E; memcpy(best_geno, x, sizeof(x)); }
    double dx[6 + ORC_MAXTOR];
    for (int d = 0; d < nd; d++) {
      double gd = grad[d < 6 ? d : d + 1];
      Eg2[d] = p->rho * Eg2[d] + (1 - p->rho) * gd * gd;
      dx[d] = -sqrt(Edx2[d] + p->eps) / sqrt(Eg2[d] + p->eps) * gd;
      Edx2[d] = p->rho * Edx2[d] + (1 - p->rho) * dx[d] * dx[d];
    }
    for (int c = 0; c < 3; c++) x[c] += dx[c];
    orc_apply_rotvec(&x[3], &dx[3]);
    for (int k = 0; k < L->n_tor; k++) x[7 + k] = orc_wrap(x[7 + k] + dx[6 + k]);
  }
  return ORC_OK;
}

/* Solis-Wets random local search (Solis and Wets 1981; the energy-only
 * local search of the LGA, Sec. 1.1), reading: a deviate
 * d_k ~ N(0, (rho s_k)^2) per degree of freedom (s = sw_sigma_t for
 * translation, sw_sigma_ang for the rotation vector and the torsions); the
 * candidate x + b + d is tried first and, if it is not better, x - b - d.
 * On success at x + b + d the bias becomes 0.2 b + 0.4 d, on success at
 * x - b - d it becomes b - 0.4 d, and when both fail it is halved.  After
 * sw_max_succ consecutive successes rho doubles, after sw_max_fail
 * consecutive failures it halves.  The search stops when `max_ev`
 * evaluations are used or rho drops below sw_rho_lb; only improvements are
 * accepted, so the final point is the best one.  E_in is the energy of
 * geno_in (evaluated here, counting one evaluation, if it is NaN).
 * Random numbers: Philox with key (seed lo, seed hi ^ 0x9E3779B9) and
 * counter (ligand, run, generation << 16 | individual, iteration << 8 |
 * block); degree of freedom k uses block k/2 and the Box-Muller pair of its
 * words 0 and 1, u1 = ((w0 >> 8) + 1) 2^-24, u2 = (w1 >> 8) 2^-24, taking
 * the cosine branch for even k and the sine branch for odd k. */
static double orc_sw_normal(uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen, uint32_t indiv, uint32_t it,
                            int k) {
  uint32_t ctr[4] = {lig, run, (gen << 16) | indiv, (it << 8) | (uint32_t)(k >> 1)};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x9E3779B9u};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  double u1 = (double)((w[0] >> 8) + 1) * (1.0 / 16777216.0);
  double u2 = (double)(w[1] >> 8) * (1.0 / 16777216.0);
  double r = sqrt(-2.0 * log(u1));
  return (k & 1) ? r * sin(2 * PI * u2) : r * cos(2 * PI * u2);
}

double orc_sw_deviate(uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen, uint32_t indiv, uint32_t it, int k) {
  return orc_sw_normal(seed, lig, run, gen, indiv, it, k);
}

/* x <- x + sgn (b + d) over the degrees of freedom (t, omega, theta) */
static void orc_sw_move(const orc_ligand *L, double *x, const double *b, const double *d, double sgn) {
  double w[3];
  for (int c = 0; c < 3; c++) x[c] += sgn * (b[c] + d[c]);
  for (int c = 0; c < 3; c++) w[c] = sgn * (b[3 + c] + d[3 + c]);
  orc_apply_rotvec(&x[3], w);
  for (int k = 0; k < L->n_tor; k++) x[7 + k] = orc_wrap(x[7 + k] + sgn * (b[6 + k] + d[6 + k]));
}

int orc_solis_wets(const orc_ligand *L, orc_grid *g, const orc_dock_params *p, const double *geno_in, double E_in,
                   int max_ev, uint64_t seed, uint32_t lig, uint32_t run, uint32_t gen, uint32_t indiv,
                   double *best_geno, double *best_E, int *evals_used) {
  double x[ORC_STRIDE], xt[ORC_STRIDE];
  memcpy(x, geno_in, sizeof(x));
  int nd = 6 + L->n_tor, ev = 0, rc = ORC_OK;
  double Ex = E_in;
  if (isnan(Ex) && max_ev > 0) {
    rc = orc_score(L, g, x, &Ex, NULL, NULL, NULL);
    ev++;
  }
  double b[6 + ORC_MAXTOR] = {0}, d[6 + ORC_MAXTOR];
  double rho = p->sw_rho;
  int succ = 0, fail = 0;
  for (uint32_t it = 0; !rc && ev < max_ev && rho >= p->sw_rho_lb; it++) {
    for (int k = 0; k < nd; k++)
      d[k] = rho * (k < 3 ? p->sw_sigma_t : p->sw_sigma_ang) * orc_sw_normal(seed, lig, run, gen, indiv, it, k);
    double Et;
    memcpy(xt, x, sizeof(x));
    orc_sw_move(L, xt, b, d, 1.0);
    rc |= orc_score(L, g, xt, &Et, NULL, NULL, NULL);
    ev++;
    int ok = 0;
    if (Et < Ex) {
      memcpy(x, xt, sizeof(x));
      Ex = Et;
      for (int k = 0; k < nd; k++) b[k] = 0.2 * b[k] + 0.4 * d[k];
      ok = 1;
    } else if (ev < max_ev) {
      memcpy(xt, x, sizeof(x));
      orc_sw_move(L, xt, b, d, -1.0);
      rc |= orc_score(L, g, xt, &Et, NULL, NULL, NULL);
      ev++;
      if (Et < Ex) {
        memcpy(x, xt, sizeof(x));
        Ex = Et;
        for (int k = 0; k < nd; k++) b[k] = b[k] - 0.4 * d[k];
        ok = 1;
      }
    }
    if (ok) {
      succ++;
      fail = 0;
    } else {
      for (int k = 0; k < nd; k++) b[k] *= 0.5;
      fail++;
      succ = 0;
    }
    if (succ >= p->sw_max_succ) {
      rho *= 2.0;
      succ = 0;
    } else if (fail >= p->sw_max_fail) {
      rho *= 0.5;
      fail = 0;
    }
  }
  memcpy(best_geno, x, sizeof(x));
  *best_E = Ex;
  *evals_used = ev;
  return rc;
}

int orc_n_ls(const orc_dock_params *p) {
  int n = (int)floor(p->ls_rate * p->pop + 0.5);
  if (n > p->pop - 1) n = p->pop - 1;
  if (n < 0) n = 0;
  return n;
}

/* One run: generation 0 evaluates `pop` random individuals; each later
 * generation does the GA step (pop-1 evaluations) and then local search on
 * n_ls picked individuals (ls_iters evaluations each), as long as the
 * generation count stays <= max_gens and the evaluation count <= max_evals.
 * Returns the best individual of the final population. */
int orc_dock_run(const orc_ligand *L, orc_grid *g, const orc_dock_params *p, uint64_t seed, uint32_t lig,
                 uint32_t run, double *best_geno, double *best_E, int64_t *evals_out, int *gens_out) {
  int pop = p->pop;
  if (pop < 1 || pop > ORC_MAXPOP) return ORC_E_INVALID;
  double *G0 = (double *)malloc(sizeof(double) * ORC_STRIDE * pop);
  double *G1 = (double *)malloc(sizeof(double) * ORC_STRIDE * pop);
  double *E0 = (double *)malloc(sizeof(double) * pop), *E1 = (double *)malloc(sizeof(double) * pop);
  int rc = ORC_OK;
  int64_t evals = 0;
  for (int i = 0; i < pop; i++) {
    orc_init_individual(L, g, seed, lig, run, (uint32_t)i, &G0[(size_t)i * ORC_STRIDE]);
    rc |= orc_score(L, g, &G0[(size_t)i * ORC_STRIDE], &E0[i], NULL, NULL, NULL);
  }
  evals += pop;
  int n_ls = orc_n_ls(p);
  /* the most a generation can cost: ADADELTA uses exactly ls_iters
   * evaluations per local search, Solis-Wets at most ls_iters */
  int64_t per_gen_max = (pop - 1) + (int64_t)n_ls * p->ls_iters;
  int gen = 1;
  int picked[ORC_MAXPOP];
  /* autostop (reading): the best energy of the population after every
   * generation (generation 0 included); a run stops once 10 of them are
   * recorded and their standard deviation (over the last 10, divided by
   * 10) is below stop_std */
  double hist[10];
  int nh = 0;
  hist[nh++ % 10] = E0[orc_argmin(E0, pop)];
  for (;;) {
    if (rc || gen > p->max_gens || evals + per_gen_max > p->max_evals) break;
    if (p->autostop && nh >= 10) {
      double m = 0, v = 0;
      for (int k = 0; k < 10; k++) m += hist[k];
      m /= 10;
      for (int k = 0; k < 10; k++) v += (hist[k] - m) * (hist[k] - m);
      if (sqrt(v / 10) < p->stop_std) break;
    }
    orc_ga_offspring(L, p, seed, lig, run, (uint32_t)gen, pop, G0, E0, G1, E1);
    for (int i = 1; i < pop; i++) rc |= orc_score(L, g, &G1[(size_t)i * ORC_STRIDE], &E1[i], NULL, NULL, NULL);
    evals += pop - 1;
    orc_ls_pick(seed, lig, run, (uint32_t)gen, pop, n_ls, picked);
    for (int s = 0; s < n_ls; s++) {
      int i = picked[s];
      double bg[ORC_STRIDE], bE;
      if (p->ls_method == 1) {
        int used = 0;
        rc |= orc_solis_wets(L, g, p, &G1[(size_t)i * ORC_STRIDE], E1[i], p->ls_iters, seed, lig, run,
                             (uint32_t)gen, (uint32_t)i, bg, &bE, &used);
        evals += used;
      } else {
        rc |= orc_adadelta(L, g, p, &G1[(size_t)i * ORC_STRIDE], p->ls_iters, bg, &bE);
        evals += p->ls_iters;
      }
      memcpy(&G1[(size_t)i * ORC_STRIDE], bg, sizeof(bg));
      E1[i] = bE;
    }
    double *t = G0; G0 = G1; G1 = t;
    t = E0; E0 = E1; E1 = t;
    hist[nh++ % 10] = E0[orc_argmin(E0, pop)];
    gen++;
  }
  int b = orc_argmin(E0, pop);
  memcpy(best_geno, &G0[(size_t)b * ORC_STRIDE], sizeof(double) * ORC_STRIDE);
  *best_E = E0[b];
  *evals_out = evals;
  *gens_out = gen - 1;
  free(G0); free(G1); free(E0); free(E1);
  return rc;
}

/* nrun independent runs of one ligand (Sec. 1.1), in parallel over runs. */
int orc_dock(const orc_ligand *L, orc_grid *g, const orc_dock_params *p, uint64_t seed, uint32_t lig,
             double *run_geno, double *run_E, int64_t *run_evals, int *run_gens, int n_threads) {
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int r = 0; r < p->nrun; r++)
    err |= -orc_dock_run(L, g, p, seed, lig, (uint32_t)r, &run_geno[(size_t)r * ORC_STRIDE], &run_E[r],
                         &run_evals[r], &run_gens[r]);
  return err ? ORC_E_NOMAP : ORC_OK;
}
