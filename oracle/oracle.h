/*
 * FP64 CPU oracle for the docking hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The GPU product path never links, loads or calls it,
 * and it shares no code, header or table with that path.
 *
 * What it computes (the paper names the method, AutoDock4's scoring function
 * and the Lamarckian GA with Solis-Wets / ADADELTA local search, Sec. 1 and
 * Sec. 1.1, but prints no formula; every formula here is the stated reading
 * of the AutoDock4 functional form):
 *   - pair potentials (smoothed 12-6 vdW, 12-10 H-bond, distance-dependent
 *     dielectric electrostatics, desolvation),
 *   - receptor grid maps by direct receptor-atom sums (Sec. 2.3: AutoGrid4
 *     affinity, electrostatic and desolvation maps), stored as FP32,
 *   - ligand torsion-tree preparation, pose from genotype, energy (trilinear
 *     map interpolation + intramolecular pairs) and its analytic gradient,
 *   - Philox4x32-10 random numbers, the Lamarckian GA and ADADELTA local
 *     search (Sec. 1: LGA with local search written back; Sec. 1.1: nrun
 *     independent runs, evaluation cap nev, ADADELTA).
 * Everything is double precision except the stored map values (float).
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#define ORC_MAXT 16      /* force-field types */
#define ORC_MAXA 128     /* atoms per ligand */
#define ORC_MAXTOR 32    /* torsions per ligand */
#define ORC_MAXPAIRS (ORC_MAXA * (ORC_MAXA - 1) / 2)
#define ORC_MAXPOP 4096   /* individuals per run */
#define ORC_STRIDE 40    /* genotype / gradient stride: t(3) q(4) theta(32) pad */

typedef struct {
  int n_types;
  double Rii[ORC_MAXT], epsii[ORC_MAXT], vol[ORC_MAXT], solpar[ORC_MAXT];
  double Rhb[ORC_MAXT], epshb[ORC_MAXT];
  int hbrole[ORC_MAXT]; /* 0 none, 1 donor, 2 acceptor */
  double w_vdw, w_hb, w_el, w_sol, w_tor;
  double coulomb, diel_A, diel_eps0, diel_lambda, diel_k;
  double sigma, qasp, smooth, cutoff, cap, r_floor, k_out;
} orc_ff;

typedef struct {
  int n[3];            /* nx, ny, nz (points per axis) */
  double h;            /* spacing (A) */
  double origin[3];    /* position of node (0,0,0) */
  int n_maps;          /* affinity maps; map n_maps = elec, n_maps+1 = desolv */
  int map_type[ORC_MAXT];
  int type_to_map[ORC_MAXT];
  float *vals;         /* [n_maps+2][nz][ny][nx] */
  unsigned char *have; /* lazy grids: per node, 1 once all maps are computed */
  int n_rec;           /* receptor kept for lazy grids */
  double *rec_xyz;
  int *rec_type;
  double *rec_q;
  orc_ff ff;
} orc_grid;

typedef struct {
  int n, n_tor, n_pairs;
  int type[ORC_MAXA];
  double q[ORC_MAXA];
  double y[ORC_MAXA][3];          /* reference coordinates */
  int frag[ORC_MAXA], n_frag;
  int root_atom;
  double center[3];               /* rotation centre: reference centroid */
  int tor_a[ORC_MAXTOR], tor_b[ORC_MAXTOR];  /* root side, leaf side */
  int tor_depth[ORC_MAXTOR];
  unsigned char moves[ORC_MAXTOR][ORC_MAXA]; /* S_k membership */
  int leaf_first[ORC_MAXTOR];     /* torsions, deepest first */
  int pair_i[ORC_MAXPAIRS], pair_j[ORC_MAXPAIRS];
  int dist[ORC_MAXA][ORC_MAXA];   /* bond-path distances */
  char msg[160];
} orc_ligand;

typedef struct {
  int nrun, pop, max_gens;
  int64_t max_evals;
  double ls_rate;
  int ls_iters;
  double cx_rate, mut_rate, tour_p;
  double rho, eps;                /* ADADELTA */
  double mut_t, mut_theta, mut_rot;
  int ls_method;                  /* 0 ADADELTA, 1 Solis-Wets */
  int autostop;                   /* 1: stop a run when its best energy has settled */
  double sw_rho, sw_rho_lb;       /* Solis-Wets step size: initial, lower bound */
  int sw_max_succ, sw_max_fail;   /* consecutive successes / failures that expand / contract */
  double sw_sigma_t, sw_sigma_ang;/* deviate scale per unit step: translation (A), angles (rad) */
  double stop_std;                /* autostop threshold (kcal/mol) over the last 10 generations */
} orc_dock_params;

/* error codes (mirrors the meaning, not the code, of the product's) */
#define ORC_OK 0
#define ORC_E_INVALID -1
#define ORC_E_NOMAP -2

#endif
