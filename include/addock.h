/*
 * addock -- MI355X-native docking hot path behind a C ABI.
 *
 * The library evaluates the AutoDock4-form scoring function with its
 * analytic gradient on the GPU and drives the Lamarckian GA with ADADELTA
 * local search built on it.  Its calls follow the paper's statement of the
 * screening problem (Sec. 2.2 of "GPU-Accelerated Drug Discovery with Docking
 * on the Summit Supercomputer"): many ligands are docked against one
 * receptor whose grid maps are sent to the GPU once and stay resident
 * (Sec. 2.2.1, Sec. 2.2.3); each ligand uses the maps of its own atom types
 * (Sec. 2.2.3); each ligand gets nrun independent LGA runs, each with its own
 * final pose and an evaluation cap nev, and the screen keeps the best run
 * (Sec. 1.1).
 *
 * Conventions for every call:
 *   - Return AD_OK (0) or a negative AD_E_* code; the message of the last
 *     failure on a context is available from ad_last_error().
 *   - Inputs are read during the call and never retained; outputs go to
 *     caller buffers.  With ptrs_on_device != 0, genotype / energy / gradient
 *     pointers are device pointers of the context's device and the call is
 *     asynchronous on the context's stream; otherwise they are host pointers,
 *     the library stages them and the call returns when the results are in
 *     the caller's buffers.
 *   - Calls on one context are serialised on its stream (the analogue of the
 *     paper's one-at-a-time GPU section, Sec. 2.2.2).  A context must not be
 *     used from two threads at once.
 *   - Coordinates are in Angstrom, energies in kcal/mol, angles in radians.
 *   - All numerical work runs in the library's HIP kernels.
 */
#ifndef ADDOCK_H
#define ADDOCK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AD_OK 0
#define AD_E_INVALID -1     /* malformed argument (sizes, topology, values) */
#define AD_E_NOMAP -2       /* a ligand atom type has no resident map */
#define AD_E_OOM -3         /* device or host allocation failed */
#define AD_E_DEVICE -4      /* no usable GPU / bad device index */
#define AD_E_STATE -5       /* call order (e.g. scoring before a grid is loaded) */
#define AD_E_UNSUPPORTED -6 /* option not implemented */
#define AD_E_HIP -7         /* HIP runtime error */

#define AD_MAX_TYPES 16
#define AD_MAX_ATOMS 128
#define AD_MAX_TORSIONS 32
#define AD_GENO_STRIDE 40   /* genotype / gradient floats per pose */
#define AD_MAX_POP 4096

typedef struct ad_ctx ad_ctx;
typedef struct ad_batch ad_batch;

/* Force-field table (AutoDock4 functional form, Sec. 1).  Per type: radius
 * R_ii and well depth eps_ii of the 12-6 term, atomic volume V, solvation
 * parameter solpar, H-bond role (0 none, 1 donor, 2 acceptor) and, for
 * acceptors, the 12-10 H-bond radius R_hb and depth eps_hb.  Scalars: term
 * weights, Coulomb constant, Mehler-Solmajer dielectric (A, eps0, lambda,
 * k), desolvation sigma and charge factor qasp, smoothing band width,
 * map cutoff, affinity-map cap, distance floor and out-of-grid restraint
 * constant.  Copied by ad_create. */
typedef struct {
  int n_types;
  double Rii[AD_MAX_TYPES], epsii[AD_MAX_TYPES], vol[AD_MAX_TYPES], solpar[AD_MAX_TYPES];
  double Rhb[AD_MAX_TYPES], epshb[AD_MAX_TYPES];
  int hbrole[AD_MAX_TYPES];
  double w_vdw, w_hb, w_el, w_sol, w_tor;
  double coulomb, diel_A, diel_eps0, diel_lambda, diel_k;
  double sigma, qasp, smooth, cutoff, cap, r_floor, k_out;
} ad_forcefield;

/* Grid geometry: nx*ny*nz points (each >= 2), node (i,j,k) at
 * origin + spacing*(i,j,k).  map_types[m] is the force-field type of
 * affinity map m (n_maps of them, distinct, each < n_types). */
typedef struct {
  int nx, ny, nz;
  double spacing;
  double origin[3];
  int n_maps;
  const int *map_types;
} ad_grid_desc;

/* One ligand: n_atoms (1..128) atoms with force-field type ids, partial
 * charges and reference coordinates ([n_atoms][3]); n_bonds = n_atoms-1
 * bonds ([n_bonds][2] atom indices) forming a tree; rotatable[b] != 0 marks
 * bond b as a torsion.  Torsion k of the genotype is the k-th rotatable bond
 * in bond order. */
typedef struct {
  int n_atoms, n_bonds;
  const int *type_id;
  const float *charge;
  const float *xyz;
  const int *bonds;
  const unsigned char *rotatable;
} ad_ligand;

/* ---- context ----------------------------------------------------------
 * ad_create: binds a context to GPU `device`, copies the force field and
 * creates (hip_stream == NULL) or borrows (e.g. PyTorch's current stream)
 * the stream all work is queued on.  No GPU -> AD_E_DEVICE; malformed force
 * field -> AD_E_INVALID.  Device memory is owned by the context and freed by
 * ad_destroy (which first waits for the stream).  Batches (ad_load_ligands)
 * and pre-screens (ad_prescreen_create) belong to their context, in any
 * teardown order: ad_destroy releases the device memory of those still alive
 * and detaches them, after which ad_free_batch / ad_prescreen_destroy only
 * delete the handle and every other call with them returns AD_E_INVALID. */
int ad_create(ad_ctx **out, int device, const ad_forcefield *ff, void *hip_stream);
void ad_destroy(ad_ctx *ctx);
const char *ad_last_error(const ad_ctx *ctx);
int ad_set_stream(ad_ctx *ctx, void *hip_stream);
/* Waits for all work queued on the context's stream. */
int ad_synchronize(ad_ctx *ctx);

/* ---- receptor grids (Sec. 2.2.1, 2.2.3, 2.3) ----------------------------
 * ad_load_grids: maps are FP32 [n_maps+2][nz][ny][nx], x fastest: the
 * n_maps affinity maps in map_types order, then the electrostatic map, then
 * the desolvation map.  A ligand atom of type t and charge q scores
 * map_t + q*map_elec + |q|*map_desolv, interpolated trilinearly; outside the
 * box the coordinate is clamped to the nearest face and
 * k_out*|x - x_clamped|^2 is added.  The library copies the maps (host or
 * device source) and keeps them resident until the next load or destroy.
 * Errors: AD_E_INVALID (dims < 2, spacing <= 0, bad map types, non-finite
 * values, nx*ny >= 2^24, n_maps*nz >= 2^24 or n_maps*nx*ny*nz >= 2^32: the
 * kernels index map records in 32 bits with 24-bit products), AD_E_OOM. */
int ad_load_grids(ad_ctx *ctx, const ad_grid_desc *g, const float *maps, int ptrs_on_device);
/* ad_grid_check: the host-only validation of ad_load_grids (geometry, map
 * types against a force field with n_types types, index limits); no context
 * or GPU needed.  Returns AD_OK or AD_E_INVALID with a message in msg (if
 * msg_len > 0). */
int ad_grid_check(const ad_grid_desc *g, int n_types, char *msg, int msg_len);

/* ad_build_grids: computes the maps on the GPU from receptor atoms (host
 * arrays: xyz [n_rec][3], type ids, charges) by direct sums in the same
 * AutoDock4 form -- affinity map of type t: 12-6/12-10 plus the
 * type-dependent desolvation half within `cutoff`, capped at `cap`;
 * electrostatic map without cutoff; desolvation map qasp-part within
 * `cutoff` -- and makes them resident as ad_load_grids would.  If maps_out
 * is non-NULL the maps are also copied to that host buffer (layout as
 * above).  Errors as ad_load_grids. */
int ad_build_grids(ad_ctx *ctx, const ad_grid_desc *g, int n_rec, const float *rec_xyz, const int *rec_type,
                   const float *rec_charge, float *maps_out);

/* ---- ligands -------------------------------------------------------------
 * ad_ligand_check: host-only validation of one ligand against a force
 * field with n_types types (no context or GPU needed).  Returns AD_OK or
 * AD_E_INVALID with a message in msg (if msg_len > 0). */
int ad_ligand_check(const ad_ligand *lig, int n_types, char *msg, int msg_len);

/* ad_load_ligands: validates every ligand (a tree; every rotatable bond
 * between two non-terminal atoms; <= 128 atoms, <= 32 torsions; finite
 * data), prepares its torsion tree and intramolecular pair list (atoms in
 * different rigid fragments at bond distance >= 4) and uploads the batch.
 * Needs loaded grids (AD_E_STATE otherwise); AD_E_NOMAP if an atom type has
 * no map.  The batch belongs to the caller until ad_free_batch, and stays
 * valid across grid reloads that keep the map types. */
int ad_load_ligands(ad_ctx *ctx, int n, const ad_ligand *ligs, ad_batch **out);
/* ad_load_ligands_packed: as ad_load_ligands for n ligands stored back to
 * back (host arrays): ligand i has n_atoms[i] atoms and n_bonds[i] bonds;
 * its atoms start at the sum of the earlier n_atoms in type_id, charge and
 * xyz (3 floats per atom), its bonds at the sum of the earlier n_bonds in
 * bonds (2 ints per bond) and rotatable.  Serves large synthetic sets
 * without one host structure per ligand (Sec. 2.2.1: many ligands per run). */
int ad_load_ligands_packed(ad_ctx *ctx, int n, const int *n_atoms, const int *n_bonds, const int *type_id,
                           const float *charge, const float *xyz, const int *bonds, const unsigned char *rotatable,
                           ad_batch **out);
void ad_free_batch(ad_batch *b);
/* Per-ligand sizes: atoms, torsions, intramolecular pairs, rigid fragments,
 * and depth_sum = sum over atoms of the number of torsions that move the
 * atom (each output pointer may be NULL). */
int ad_batch_info(const ad_batch *b, int lig, int *n_atoms, int *n_torsions, int *n_pairs, int *n_fragments,
                  int *depth_sum);

/* ---- scoring: the hot path ----------------------------------------------
 * ad_score_poses: for pose p, ligand lig_idx[p] of the batch and genotype
 * genotypes[p*40 + ...] = [t(3) | q(4: w,x,y,z) | theta(T)] (q need not be
 * unit; it is normalised first; slots past 7+T are ignored):
 *   pose: each torsion turns its leaf-side atoms by theta_k about its bond
 *   (root side -> leaf side, right-handed), deepest torsion first; then
 *   x = R(q)(y - c) + t, c the reference centroid.
 *   energy[p] = inter (maps + restraint) + intramolecular pair energy.
 *   grad (optional, [n][40]) = [dE/dt(3) | dE/domega(3) | 0 | dE/dtheta(T) |
 *   0...], omega a world-frame rotation vector applied as
 *   q <- exp(omega/2) q.
 *   terms (optional, [n][3]) = {inter, intra, score = inter + w_tor*T}.
 * Pure and deterministic.  A non-finite genotype gives NaN outputs (not an
 * error).  Errors: AD_E_INVALID (bad lig_idx, n < 0), AD_E_STATE.
 * One 64-lane work-group per pose, sized by the batch's largest ligand (up
 * to 64 or up to 128 atoms), so a batch of small ligands alone scores
 * faster than the same ligands in a batch that also holds large ones. */
int ad_score_poses(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, const float *genotypes,
                   float *energy, float *grad, float *terms, int ptrs_on_device);

/* Evaluation shapes: the kernel variant that evaluates a pose.  Every shape
 * computes the same function within the stated tolerance; they differ in
 * the order of the FP64 sums (the last bits) and in speed.
 *   AD_SHAPE_AUTO     the batch's default: AD_SHAPE_WAVE64 when every ligand
 *                     of the batch has at most 64 atoms, else AD_SHAPE_WAVE128
 *   AD_SHAPE_WAVE64   one 64-lane wavefront per pose, one atom per lane
 *                     (ligands of at most 64 atoms)
 *   AD_SHAPE_WAVE128  one wavefront per pose, two atoms per lane (<= 128)
 *   AD_SHAPE_PACKED   two poses per wavefront, one per 32-lane half (ligands
 *                     of at most 32 atoms and 25 torsions) -- the evaluation
 *                     the docking search uses for the local search of small
 *                     ligands; poses 2w and 2w+1 share wavefront w and must
 *                     name the same ligand.
 * ad_score_poses_shape / ad_local_search_shape: ad_score_poses /
 * ad_local_search evaluated with the given shape.  A pose whose ligand does
 * not fit the shape (or, packed, whose partner names another ligand) is
 * AD_E_INVALID with host indices and gives NaN with device indices; an
 * unknown shape is AD_E_INVALID. */
#define AD_SHAPE_AUTO 0
#define AD_SHAPE_WAVE64 1
#define AD_SHAPE_WAVE128 2
#define AD_SHAPE_PACKED 3
int ad_score_poses_shape(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, const float *genotypes,
                         float *energy, float *grad, float *terms, int ptrs_on_device, int shape);

/* ad_score_poses_noalloc: for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Computes exactly what ad_score_poses
 * computes with host buffers (ptrs_on_device = 0; same kernels, bitwise the
 * same results) but stages indices, genotypes and results through a static
 * device block of AD_NOALLOC_MAX_POSES poses (1.33 MiB) that every GPU the
 * library runs on holds until the process ends, so the call allocates
 * nothing.  lig_idx, genotypes, energy, grad (optional, [n][40]) and terms
 * (optional, [n][3]) are host pointers; the call returns when the results
 * are in them.  Every section of the block is written before it is read, so
 * nothing carries over from an earlier call.  All calls on one GPU share its
 * block: calls that overlap on one GPU (two contexts, two threads) race and
 * must be serialised by the caller.  Kernel timing does not cover this call.
 * Errors: as ad_score_poses; n > AD_NOALLOC_MAX_POSES -> AD_E_INVALID. */
#define AD_NOALLOC_MAX_POSES 4096
int ad_score_poses_noalloc(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, const float *genotypes,
                           float *energy, float *grad, float *terms);

/* ---- docking: Lamarckian GA + ADADELTA (Sec. 1, Sec. 1.1) ----------------
 * Per ligand, nrun independent runs.  Generation 0 evaluates pop random
 * individuals (t uniform in the grid box, uniform random orientation,
 * torsions uniform in [-pi, pi)); every later generation keeps the best
 * individual, fills the rest by binary tournaments (win probability tour_p),
 * two-point crossover over gene blocks (cx_rate) and per-slot mutation
 * (mut_rate; +-mut_t A, +-mut_rot rad about a random axis, +-mut_theta rad),
 * evaluates the pop-1 children, then runs ADADELTA (rho, eps) for ls_iters
 * evaluations on round(ls_rate*pop) distinct non-elite individuals and
 * writes the best pose each finds back into the population.  A run stops
 * before a generation that would pass max_evals evaluations or max_gens
 * generations.  Random numbers: Philox4x32-10 keyed by seed, counter
 * (ligand id, run, generation, individual/stream/word) -- a ligand's
 * result depends only on (seed, its id, params). */
typedef struct {
  int nrun, pop, max_gens;
  int64_t max_evals;
  double ls_rate;
  int ls_iters;
  double cx_rate, mut_rate, tour_p;
  double rho, eps;
  double mut_t, mut_theta, mut_rot;
  int ls_method;   /* 0 = ADADELTA (gradient), 1 = Solis-Wets (energy only); others AD_E_UNSUPPORTED */
  int autostop;    /* 1: a run stops once its best energy has settled (below) */
  /* Solis-Wets (Sec. 1.1; Solis and Wets 1981): per degree of freedom a
   * deviate d ~ N(0, (rho s)^2), s = sw_sigma_t (A) for translation and
   * sw_sigma_ang (rad) for the rotation vector and torsions; x + b + d is
   * tried, then x - b - d; the bias b becomes 0.2 b + 0.4 d, b - 0.4 d or
   * b / 2 (both failed); rho doubles after sw_max_succ consecutive
   * successes and halves after sw_max_fail consecutive failures; a search
   * stops after ls_iters evaluations or when rho < sw_rho_lb.  Each
   * evaluation counts towards max_evals. */
  double sw_rho, sw_rho_lb;     /* 1.0, 0.01 */
  int sw_max_succ, sw_max_fail; /* 4, 4 */
  double sw_sigma_t, sw_sigma_ang; /* 1.0 A, 0.2 rad */
  /* autostop (Sec. 1.1): after every generation the run records the best
   * energy of its population; it stops once ten are recorded and their
   * standard deviation (over the last ten) is below stop_std (kcal/mol). */
  double stop_std;              /* 0.15 */
} ad_dock_params;

typedef struct {
  float best_energy;                  /* lowest search energy over runs */
  float best_score;                   /* inter + w_tor*T at that pose */
  float best_genotype[AD_GENO_STRIDE];
  int best_run;
  int generations;                    /* generations of the best run */
  int64_t evals;                      /* evaluations over all runs */
} ad_dock_result;

/* ad_dock_batch: docks every ligand of the batch.  lig_ids (optional, [n])
 * gives each ligand's id for the random streams (default: batch index).
 * out: [n_lig] results (host).  run_energy / run_genotype (optional, host):
 * [n_lig][nrun] best energy and [n_lig][nrun][40] genotype of every run.
 * Synchronous.  Errors: AD_E_INVALID (params), AD_E_UNSUPPORTED, AD_E_OOM,
 * AD_E_STATE. */
int ad_dock_batch(ad_ctx *ctx, const ad_batch *b, const ad_dock_params *p, uint64_t seed, const uint32_t *lig_ids,
                  ad_dock_result *out, float *run_energy, float *run_genotype);

/* ad_dock_select: docks the n ligands lig_idx[0..n) (batch indices, host)
 * of batch b exactly as ad_dock_batch docks them (a ligand's random streams
 * are keyed by its batch index, so its result does not depend on which
 * other ligands are docked with it).  out: [n] results, run_energy [n][nrun]
 * and run_genotype [n][nrun][40] (optional), host.  Serves a screened
 * campaign: dock only the ligands a pre-screen ranks best (Sec. 2.2: many
 * ligands against one receptor).  Errors as ad_dock_batch. */
int ad_dock_select(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, const ad_dock_params *p, uint64_t seed,
                   ad_dock_result *out, float *run_energy, float *run_genotype);

/* ad_local_search: ADADELTA on n given poses (genotypes in/out, [n][40]):
 * `iters` evaluations each; on return genotypes hold the best evaluated
 * pose and energy its energy (Lamarckian write-back).  Uses p->rho, p->eps. */
int ad_local_search(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, float *genotypes, float *energy,
                    const ad_dock_params *p, int iters, int ptrs_on_device);
int ad_local_search_shape(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, float *genotypes,
                          float *energy, const ad_dock_params *p, int iters, int ptrs_on_device, int shape);

/* ad_solis_wets: Solis-Wets local search (parameters sw_* of p) on n given
 * poses (host arrays: lig_idx [n], genotypes [n][40] in/out, energy [n]
 * out, evals_used [n] out, optional).  The start pose is evaluated first
 * (one evaluation), then at most max_evals - 1 more; on return genotypes
 * hold the best pose found.  Random streams: ligand id = lig_idx[i],
 * run 0, generation 0, individual i (n <= 65536). */
int ad_solis_wets(ad_ctx *ctx, const ad_batch *b, int n, const int *lig_idx, float *genotypes, float *energy,
                  int *evals_used, const ad_dock_params *p, int max_evals, uint64_t seed);

/* Diagnostics: the initial population genotypes of generation 0 for
 * (ligand, run), [pop][40] host, exactly as ad_dock_batch draws them. */
int ad_initial_population(ad_ctx *ctx, const ad_batch *b, int lig, uint32_t lig_id, int run, int pop,
                          uint64_t seed, float *genotypes);

/* ad_dock_stream: docks n ligands stored back to back (the layout of
 * ad_load_ligands_packed, host arrays) in batches of batch_size with double
 * buffering: while batch k docks, a host thread prepares batch k + 1
 * (validation, torsion tree, pair list, pre-screen features, on up to 16
 * threads) and uploads it; each batch is freed after it docked.  This is
 * the paper's overlap of host set-up with GPU docking (Sec. 2.2.2, Fig. 1) for
 * sets too large to load at once.  Ligand i's random-stream id is id0 + i,
 * so out[i] (caller-allocated, n entries) equals ad_dock_batch's result for
 * the same ligand docked with that id, whatever the batching: a campaign
 * resumed at ligand j (id0 = j), or split into shards, reproduces the
 * uninterrupted run.  stats (optional, 3 doubles):
 * seconds of host preparation and upload, of docking, and wall time.  The
 * first failing ligand stops the call with its batch and index in the
 * message; results of earlier batches are already in out. */
int ad_dock_stream(ad_ctx *ctx, int n, const int *n_atoms, const int *n_bonds, const int *type_id,
                   const float *charge, const float *xyz, const int *bonds, const unsigned char *rotatable,
                   int batch_size, const ad_dock_params *p, uint64_t seed, uint32_t id0, ad_dock_result *out,
                   double *stats);

/* ---- docking schedule -------------------------------------------------------
 * Batched uneven docking (Sec. 2.2: many ligands of different sizes against
 * one receptor): the runs of a dock call are split into two atom-capacity
 * buckets (<= 64 and <= 128 atoms), each served by its own kernel variant,
 * in longest-first order, on two streams.  The generation loop is captured
 * once per call into a hipGraph and replayed (use_graph; kernel timing
 * forces eager launches).  The local-search kernel can stage the first
 * stage_pairs pair records of each ligand in LDS; with autotune the size is
 * chosen per bucket by timing short local searches on a copy of the initial
 * population (cached per batch and shape), with stage_pairs >= 0 it is
 * forced (rounded down to a candidate: 0, 128, 256, 512, 1024, 2048).  With
 * pack_small the ADADELTA local search of ligands of at most 32 atoms and 25
 * torsions runs two individuals per wavefront (one per half), in the same
 * launch as the 64-atom bucket's other runs, which then stage no pairs; the
 * reported run energies are re-scored by the one-wavefront evaluation.
 * Graph, autotune and staging change the speed only; packing sums a pose's
 * energy in another order inside the search (the searches of packed
 * ligands differ from unpacked ones at rounding level).  Defaults: graph on,
 * autotune on, pack_small on. */
int ad_set_schedule(ad_ctx *ctx, int use_graph, int autotune, int stage_pairs, int pack_small);
/* stage_pairs[2]: the staging size used per bucket by the last dock call
 * (-1: bucket empty or no local search); graph_used: 1 if it ran as a graph;
 * packed_runs: runs whose local search was packed (any may be null). */
int ad_get_schedule(ad_ctx *ctx, int *stage_pairs, int *graph_used, int *packed_runs);

/* Launch shape of the ADADELTA local-search kernel, per bucket (batching of
 * uneven ligands, Sec. 2.2: work-group residency and pair-loop form chosen by
 * the library's autotuner per atom-count bucket).  Two dimensions, both
 * changing speed only (bitwise the same results):
 *   unroll     1: the pair loop takes one step (a pair per lane) per trip;
 *              2: two steps per trip, both steps' records held in fixed
 *              registers and both steps' positions read before the first
 *              step's force additions (each lane still adds its pairs in
 *              list order);
 *   wg_per_cu  one-wavefront work-groups resident per compute unit: as many
 *              as the kernel's LDS allows (at most 16), or fewer by padding
 *              the dynamic LDS (fewer individuals share a CU's caches).
 * With autotune (ad_set_schedule) each dock call's buckets time unroll
 * {1, 2} x wg_per_cu {all, 3/4, 1/2 of what fits} on a sample of their runs
 * (cached per batch and call shape), then the work queue (ad_set_work_queue),
 * then the pair-staging sizes; a candidate replaces the default only if it
 * is 3 % faster.
 * ad_set_launch_shape forces unroll (1 or 2) and/or wg_per_cu (1..64, capped
 * at what fits); 0 leaves a dimension to the tuner (the default).
 * ad_get_launch_shape: unroll[2] and wg_per_cu[2] used per bucket (<= 64,
 * <= 128 atoms) by the last dock call (-1: bucket empty, no local search, or
 * Solis-Wets).  AD_E_INVALID for values out of range. */
int ad_set_launch_shape(ad_ctx *ctx, int unroll, int wg_per_cu);
int ad_get_launch_shape(ad_ctx *ctx, int *unroll, int *wg_per_cu);

/* Persistent work queue of the generation launches (the batching of many
 * uneven ligands, Sec. 2.2: one launch per generation covers every run of
 * every ligand of a bucket).  Off, every work-group of a GA or local-search
 * launch computes one item (an individual of a run; a local search).  On,
 * each launch takes about as many work-groups as the device keeps resident
 * and they take items in run order (longest first) from a per-generation
 * ticket counter until none is left; items of runs that have stopped
 * (autostop, Solis-Wets) are skipped without a dispatch.  Results are
 * bitwise the same either way.  mode: -1 the autotuner times the ADADELTA
 * local search both ways and keeps the queue only if it is 3 % faster, for a
 * bucket that runs as one chain (ad_set_chains; a bucket split into chains
 * keeps the queue off: the other chains' launches fill a launch's tail, the
 * queue's only gain) (the default), 0 off, 1 on; the GA launches follow the bucket's choice (with
 * Solis-Wets, whose launches stay one work-group per item, they follow a
 * forced 1).  The ticket counters live in the docking state and are cleared
 * once per dock call, before any launch.  ad_get_work_queue: used[2], the
 * mode per bucket (<= 64, <= 128 atoms) of the last dock call (-1: bucket
 * empty).  AD_E_INVALID for a mode out of range. */
int ad_set_work_queue(ad_ctx *ctx, int mode);
int ad_get_work_queue(ad_ctx *ctx, int *used);

/* Chains of generation launches (the batching of Sec. 2.2 across
 * generations).  Every generation launch ends with a tail in which fewer
 * and fewer work-groups remain, while the next generation of the same runs
 * has to wait for it.  With parts > 1 each bucket's runs are split into
 * that many parts (part k: every parts-th packed ligand and every parts-th
 * one-wavefront run of the longest-first order), and each part's
 * generation launches go to a stream of its own; the parts meet only at the
 * end of the docking call, so one part's launch tail overlaps the other
 * part's launches.  Calls whose runs stop on their own (autostop,
 * Solis-Wets) decide every run's status after every generation, where the
 * parts would have to meet: they keep one part per bucket.  Results are
 * bitwise the same for any number of parts.  parts 1..4 (default 2);
 * ad_get_chains: parts[2], the parts per bucket of the last dock call (0:
 * bucket empty).  AD_E_INVALID for values out of range. */
int ad_set_chains(ad_ctx *ctx, int parts);
int ad_get_chains(ad_ctx *ctx, int *parts);

/* ---- diagnostics ----------------------------------------------------------
 * Kernel timing with HIP events recorded around every launch of the docking
 * and scoring kernels, on the stream the launch goes to, for throughput and
 * roofline reporting.  Kinds: 0 initial population, 1 GA generation,
 * 2 local-search generation (and ad_local_search), 3 scoring.  Per kind:
 * ms, the sum of the launches' durations; launches, their count; busy_ms,
 * the time during which at least one launch of the kind ran (the union of
 * their intervals: launches of different chains overlap, ad_set_chains, so
 * busy_ms <= ms).  Times are accumulated when a call completes;
 * ad_get_kernel_timing reads (and with reset != 0 clears) them.  Timing
 * adds two event records per launch and runs the generation loop eagerly
 * (no graph). */
#define AD_KERNEL_KINDS 4
typedef struct {
  double ms[AD_KERNEL_KINDS];
  int64_t launches[AD_KERNEL_KINDS];
  double busy_ms[AD_KERNEL_KINDS];
} ad_kernel_times;
int ad_set_kernel_timing(ad_ctx *ctx, int enable);
int ad_get_kernel_timing(ad_ctx *ctx, ad_kernel_times *out, int reset);

/* Microbenchmarks of the rates the kernels' rooflines are set against (the
 * measurement of the method's cost, Sec. 3; diagnostics, never called by the
 * docking path).  kind:
 *   0  FP32 vector FMA, non-packed (as the library is built): FLOP/s
 *   1  FP64 vector FMA: FLOP/s
 *   2  FP32 exp2 (the transcendental unit): results/s
 *   3  LDS ds_add_f64 on consecutive addresses, one-wavefront work-groups:
 *      lane additions/s
 *   4  random 16-byte gathers from a device buffer of `bytes` bytes
 *      (4 KiB .. 16 GiB, used up to the largest power-of-two record count
 *      that fits; L2-sized or map-sized): bytes/s
 * Each runs about 16 work-groups per CU on the context's stream, best of
 * three timed launches after a warm-up; the call allocates and frees its
 * own device buffers and synchronises.  *result receives the rate.
 * AD_E_INVALID for a bad kind or size, AD_E_OOM, AD_E_HIP. */
int ad_microbench(ad_ctx *ctx, int kind, size_t bytes, double *result);


/* ---- learned pre-screen ---------------------------------------------------
 * In the screening setting (many ligands against one receptor, Sec. 1 and
 * Sec. 2.2) a learned model ranks the ligands by predicted docking score so
 * that full docking runs only on the best-ranked share.  The model reads the
 * ligand graph only (no pose): atom features (32 per atom: one-hot type
 * 0..15, charge, |charge|, one-hot degree 0,1,2,3,>=4, rotatable bonds at the
 * atom / 2, constant 1 at index 31), 3 message-passing layers of width 128
 *   H0 = r(relu(X W0 + b0)),  M = r(A H),  H' = r(relu([H | M] W_l + b_l))
 * (A = bond adjacency), sum pooling g = r(sum H3) and an MLP
 *   z1 = r(relu(g U1 + c1)), z2 = r(relu(z1 U2 + c2)), p = z2 U3 + c3
 * with 256-wide hidden layers.  r() rounds to bfloat16 (nearest even): GEMM
 * operands are BF16, accumulation FP32 (gfx950 MFMA).  Training minimises
 *   mean (p - y)^2 + lam * mean over pairs y_i < y_j of softplus((p_i - p_j)/tau)
 * on standardised labels y with Adam on FP32 master weights.
 *
 * Parameters are one float vector of ad_prescreen_n_params() entries:
 * W0[32][128], b0[128], then for l = 1..3 W_l[256][128] (rows 0..127 act on
 * H, 128..255 on M), b_l[128], then U1[128][256], c1[256], U2[256][256],
 * c2[256], U3[256], c3[1]; all matrices row-major [in][out].
 * Ligands must have atoms with at most 8 bonds (AD_E_INVALID otherwise). */
typedef struct ad_prescreen ad_prescreen;
typedef struct {
  int batch_size;        /* minibatch size for training, 2..4096 (256) */
  double lr;             /* Adam step (1e-3) */
  double lam, tau;       /* ranking-loss weight (1.0) and temperature (0.5) */
  double beta1, beta2;   /* Adam moments (0.9, 0.999) */
  double eps;            /* Adam epsilon (1e-8) */
  double label_max;      /* labels above are clipped to it before use (HUGE_VAL: none);
                            docking energies of ligands that do not fit are large and
                            positive, and only the low end is ranked */
} ad_prescreen_cfg;

int ad_prescreen_n_params(void);
/* cfg may be null (defaults above).  Weights He-uniform from `seed` (the
 * output layer U3 scaled by 1/100), biases zero.  The model lives on the
 * context's device and uses its stream. */
int ad_prescreen_create(ad_ctx *ctx, const ad_prescreen_cfg *cfg, uint64_t seed, ad_prescreen **out);
void ad_prescreen_destroy(ad_prescreen *ps);
/* host float [n_params]; set_params also clears the Adam moments and step */
int ad_prescreen_set_params(ad_prescreen *ps, const float *params);
int ad_prescreen_get_params(ad_prescreen *ps, float *params);
/* label scale: predictions are mean + sd * p (set by ad_prescreen_train) */
int ad_prescreen_set_scale(ad_prescreen *ps, double mean, double sd);
int ad_prescreen_get_scale(ad_prescreen *ps, double *mean, double *sd);
/* Predicted score of ligands lig_idx[0..n) of batch b (lig_idx null: 0..n-1)
 * into scores (host, [n]).  Synchronous. */
int ad_prescreen_predict(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx, float *scores);
/* One minibatch (2 <= n <= 4096): forward, loss on labels clipped to
 * label_max and standardised with the current scale, backward.  Outputs (host, each optional): loss, grad
 * [n_params] and the standardised predictions pred_std [n].  No update. */
int ad_prescreen_grad(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx, const float *labels,
                      float *loss, float *grad, float *pred_std);
/* Trains for `epochs` passes over n labelled ligands: clips the labels to
 * label_max, sets the scale to their mean and standard deviation, shuffles with `seed` each epoch and
 * takes one Adam step per full minibatch (a tail shorter than batch_size is
 * skipped).  loss_curve (optional, host [epochs]) receives each epoch's mean
 * minibatch loss.  Synchronous. */
int ad_prescreen_train(ad_prescreen *ps, const ad_batch *b, int n, const int *lig_idx, const float *labels,
                       int epochs, uint64_t seed, float *loss_curve);

#ifdef __cplusplus
}
#endif
#endif
