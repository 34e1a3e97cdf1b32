/* Fast seeded generator of synthetic ligands (inputs only: no scoring or
 * search arithmetic).  Same recipe as synth.ligand -- a random typed tree
 * grown together with a clash-free 3-D conformation -- with its own random
 * stream (xoshiro256** seeded by splitmix64), so large sets (10^4 - 10^5
 * ligands) are generated in about a second.
 *
 *   types: per-type caps on bond count; HD atoms are leaves on N or OA (a C
 *          leaf replaces an HD that finds no host); heavy types drawn from
 *          the given frequencies;
 *   geometry: bond length U(1.0, 1.55) A, bond angle 109.5 +- 5 degrees to
 *          the parent's parent with a random dihedral; pairs two bonds apart
 *          >= 1.2 A, pairs three or more bonds apart >= min_nonlocal;
 *   torsions: min(n_torsions, eligible) bonds drawn without replacement from
 *          the bonds whose atoms both have degree >= 2;
 *   charges: N(0, 0.2) shifted to sum zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LG_TYPES 8
#define LG_MAX 256
enum { T_C = 0, T_A = 1, T_N = 2, T_NA = 3, T_OA = 4, T_S = 5, T_SA = 6, T_HD = 7 };
static const int kMaxValence[LG_TYPES] = {4, 3, 3, 3, 2, 2, 2, 1};

typedef struct {
  uint64_t s[4];
} rng_t;

static uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static uint64_t next_u64(rng_t *r) {
  uint64_t *s = r->s;
  const uint64_t out = rotl(s[1] * 5, 7) * 9;
  const uint64_t t = s[1] << 17;
  s[2] ^= s[0];
  s[3] ^= s[1];
  s[1] ^= s[2];
  s[0] ^= s[3];
  s[2] ^= t;
  s[3] = rotl(s[3], 45);
  return out;
}

static double unif(rng_t *r) { return (double)(next_u64(r) >> 11) * 0x1.0p-53; }
static double unif_ab(rng_t *r, double a, double b) { return a + (b - a) * unif(r); }
static int randint(rng_t *r, int n) { return (int)(unif(r) * n); }
static double normal(rng_t *r) {
  double u1 = unif(r), u2 = unif(r);
  if (u1 < 1e-300) u1 = 1e-300;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

static void unit3(double *v) {
  const double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= n;
  v[1] /= n;
  v[2] /= n;
}
static void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

typedef struct {
  int n;
  double x[LG_MAX][3];
  int parent[LG_MAX], deg[LG_MAX], type[LG_MAX];
  unsigned char pathd[LG_MAX][LG_MAX];
} grow_t;

/* one placement attempt series for a new atom bonded to p */
static int place(rng_t *r, grow_t *g, int p, double blen, double min_nl, int tries, double *out) {
  const int gp = g->parent[p];
  for (int t = 0; t < tries; ++t) {
    double d[3];
    if (gp < 0) {
      d[0] = normal(r);
      d[1] = normal(r);
      d[2] = normal(r);
      unit3(d);
    } else {
      const double ang = (109.5 + unif_ab(r, -5.0, 5.0)) * M_PI / 180.0;
      double b[3] = {g->x[gp][0] - g->x[p][0], g->x[gp][1] - g->x[p][1], g->x[gp][2] - g->x[p][2]};
      unit3(b);
      double rv[3] = {normal(r), normal(r), normal(r)}, h[3], bh[3];
      cross3(b, rv, h);
      unit3(h);
      cross3(b, h, bh);
      const double phi = unif_ab(r, -M_PI, M_PI);
      for (int k = 0; k < 3; ++k) {
        const double perp = h[k] * cos(phi) + bh[k] * sin(phi);
        d[k] = b[k] * cos(ang) + perp * sin(ang);
      }
    }
    double c[3] = {g->x[p][0] + blen * d[0], g->x[p][1] + blen * d[1], g->x[p][2] + blen * d[2]};
    int ok = 1;
    for (int j = 0; j < g->n && ok; ++j) {
      const int dj = g->pathd[p][j] + 1;
      const double dx = c[0] - g->x[j][0], dy = c[1] - g->x[j][1], dz = c[2] - g->x[j][2];
      const double rr = dx * dx + dy * dy + dz * dz;
      if ((dj >= 3 && rr < min_nl * min_nl) || (dj == 2 && rr < 1.44)) ok = 0;
    }
    if (ok) {
      memcpy(out, c, sizeof(c));
      return 1;
    }
  }
  return 0;
}

static int draw_type(rng_t *r, const double *cum, int n) {
  const double u = unif(r) * cum[n - 1];
  for (int k = 0; k < n; ++k)
    if (u < cum[k]) return k;
  return n - 1;
}

static int grow(rng_t *r, int n, int n_tor, const double *freqs, double min_nl, grow_t *g, int *types, float *q,
                float *xyz, int *bonds, unsigned char *rot) {
  int n_hd = 0;
  if (n >= 3)
    for (int i = 0; i < n; ++i) n_hd += unif(r) < freqs[T_HD];
  const int n_heavy = n - n_hd;
  double cum[LG_TYPES];
  double acc = 0.0;
  for (int k = 0; k < LG_TYPES; ++k) {
    acc += k == T_HD ? 0.0 : freqs[k];
    cum[k] = acc;
  }
  int kinds[LG_MAX];
  for (int i = 0; i < n; ++i) kinds[i] = i < n_heavy ? draw_type(r, cum, LG_TYPES) : T_HD;
  g->n = 1;
  g->x[0][0] = g->x[0][1] = g->x[0][2] = 0.0;
  g->parent[0] = -1;
  g->deg[0] = 0;
  g->type[0] = kinds[0];
  g->pathd[0][0] = 0;
  int hosts[LG_MAX];
  for (int i = 1; i < n; ++i) {
    int want = kinds[i], nh = 0;
    if (want == T_HD) {
      for (int j = 0; j < g->n; ++j)
        if ((g->type[j] == T_N || g->type[j] == T_OA) && g->deg[j] < kMaxValence[g->type[j]]) hosts[nh++] = j;
      if (!nh) want = T_C;
    }
    if (want != T_HD) {
      nh = 0;
      for (int j = 0; j < g->n; ++j)
        if (g->deg[j] < kMaxValence[g->type[j]]) hosts[nh++] = j;
    }
    for (int k = nh - 1; k > 0; --k) {   /* random host order */
      const int m = randint(r, k + 1), t = hosts[k];
      hosts[k] = hosts[m];
      hosts[m] = t;
    }
    int placed = 0, p = -1;
    double pos[3];
    for (int k = 0; k < nh && !placed; ++k) {
      p = hosts[k];
      placed = place(r, g, p, unif_ab(r, 1.0, 1.55), min_nl, 24, pos);
    }
    if (!placed) return 0;
    const int a = g->n;
    memcpy(g->x[a], pos, sizeof(pos));
    g->parent[a] = p;
    g->deg[a] = 1;
    g->deg[p] += 1;
    g->type[a] = want;
    for (int j = 0; j < a; ++j) {
      const int d = g->pathd[p][j] + 1;
      g->pathd[j][a] = g->pathd[a][j] = (unsigned char)(d > 255 ? 255 : d);
    }
    g->pathd[a][a] = 0;
    g->n = a + 1;
  }
  /* bonds, torsions */
  int elig[LG_MAX], ne = 0;
  for (int i = 1; i < n; ++i) {
    bonds[2 * (i - 1)] = g->parent[i];
    bonds[2 * (i - 1) + 1] = i;
    rot[i - 1] = 0;
    if (g->deg[g->parent[i]] >= 2 && g->deg[i] >= 2) elig[ne++] = i - 1;
  }
  const int t = n_tor < ne ? n_tor : ne;
  for (int k = 0; k < t; ++k) {   /* partial Fisher-Yates */
    const int m = k + randint(r, ne - k), s = elig[k];
    elig[k] = elig[m];
    elig[m] = s;
    rot[elig[k]] = 1;
  }
  double qs[LG_MAX], qm = 0.0, c[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i) {
    qs[i] = 0.2 * normal(r);
    qm += qs[i];
    for (int k = 0; k < 3; ++k) c[k] += g->x[i][k];
  }
  qm /= n;
  for (int i = 0; i < n; ++i) {
    types[i] = g->type[i];
    q[i] = (float)(qs[i] - qm);
    for (int k = 0; k < 3; ++k) xyz[3 * i + k] = (float)(g->x[i][k] - c[k] / n);
  }
  return 1;
}

/* One ligand of n atoms (1..256).  freqs[8]: type frequencies by type id
 * (C, A, N, NA, OA, S, SA, HD).  Outputs: types[n], q[n], xyz[3n],
 * bonds[2(n-1)], rot[n-1].  Returns the torsion count, or -1 if no
 * conformation was found in 100 attempts. */
int lg_ligand(uint64_t seed, int n, int n_tor, const double *freqs, double min_nonlocal, int *types, float *q,
              float *xyz, int *bonds, unsigned char *rot) {
  if (n < 1 || n > LG_MAX) return -1;
  rng_t r;
  uint64_t sm = seed;
  for (int k = 0; k < 4; ++k) r.s[k] = splitmix64(&sm);
  grow_t *g = (grow_t *)malloc(sizeof(grow_t));
  if (!g) return -1;
  int ok = 0;
  for (int attempt = 0; attempt < 100 && !ok; ++attempt)
    ok = grow(&r, n, n_tor, freqs, min_nonlocal, g, types, q, xyz, bonds, rot);
  free(g);
  if (!ok) return -1;
  int t = 0;
  for (int i = 0; i + 1 < n; ++i) t += rot[i];
  return t;
}

/* A set of ligands: sizes n[i], torsion requests t[i], seeds seed0 + i,
 * written back to back (atom offsets are the prefix sums of n).  Returns 0,
 * or -(i+1) for the first ligand that failed. */
int lg_ligand_set(uint64_t seed0, int count, const int *n, const int *t, const double *freqs, double min_nonlocal,
                  int *types, float *q, float *xyz, int *bonds, unsigned char *rot) {
  /* offsets first (serial), then the ligands in parallel */
  long *ao = (long *)malloc(sizeof(long) * (count + 1));
  long *bo = (long *)malloc(sizeof(long) * (count + 1));
  if (!ao || !bo) {
    free(ao);
    free(bo);
    return -1;
  }
  ao[0] = bo[0] = 0;
  for (int i = 0; i < count; ++i) {
    ao[i + 1] = ao[i] + n[i];
    bo[i + 1] = bo[i] + (n[i] > 0 ? n[i] - 1 : 0);
  }
  int first_bad = count;
#pragma omp parallel for schedule(dynamic, 16) reduction(min : first_bad)
  for (int i = 0; i < count; ++i) {
    const int r = lg_ligand(seed0 + (uint64_t)i, n[i], t[i], freqs, min_nonlocal, types + ao[i], q + ao[i],
                            xyz + 3 * ao[i], bonds + 2 * bo[i], rot + bo[i]);
    if (r < 0 && i < first_bad) first_bad = i;
  }
  free(ao);
  free(bo);
  return first_bad < count ? -(first_bad + 1) : 0;
}
