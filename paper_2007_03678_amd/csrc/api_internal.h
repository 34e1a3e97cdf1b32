// Context / batch objects of the C ABI and the kernel launch interface.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "ad_internal.h"

namespace ad {

struct EvalConst {
  FFConst ff;
  GridArgs grid;
  BatchArgs batch;
};

// Arguments of the map-building kernel (passed through device memory).
struct MapBuildArgs {
  const float *rec_xyz;
  const int *rec_type;
  const float *rec_q;
  int n_rec;
  int nx, ny, nz, n_maps;
  double ox, oy, oz, h;
  int map_type[kMaxTypes];
  double A[kMaxTypes][kMaxTypes], B[kMaxTypes][kMaxTypes], r0[kMaxTypes][kMaxTypes];
  int hb[kMaxTypes][kMaxTypes];
  double solpar[kMaxTypes], vol[kMaxTypes];
  double w_el_ke, w_sol, qasp, diel_A, diel_B, diel_k, diel_lB, two_s2, half_smooth, cutoff2, cap, r_floor;
  float *out4;   // [n_maps][nz][ny][nx] float4 records
  float *soa;    // [n_maps+2][nz][ny][nx] or null
};

struct DockArgs {
  float *geno;
  float *energy;
  unsigned long long *evals;
  const int *run_order;
  const uint32_t *lig_id;   // random-stream id of each docked ligand
  const int *lig_map;       // batch index of each docked ligand (null: identity)
  int n_runs, nrun, pop, n_ls, ls_iters;
  int n_launch;      // runs covered by a launch: run_order[0..n_launch)
  int stage_pairs;   // local search: pair records staged in LDS per ligand (0: none)
  int n_dual;        // ADADELTA: the first n_dual runs of run_order (whole ligands of at most
                     // kDualAtoms atoms and kDualTor torsions) take the two-per-wavefront kernel
  // launch shape of the local search (speed only, bitwise the same results):
  // pair-loop unroll (1 or 2) and extra dynamic LDS per work-group that caps
  // the work-groups resident per CU (0: as many as the kernel's LDS allows)
  int ls_unroll, ls_pad;
  // persistent work queue (null: one work-group per item): per-generation
  // ticket counters of the GA and local-search launches (index = generation,
  // zero when the docking call starts) and the grids their launches take
  unsigned int *q_ga, *q_ls;
  int q_grid_ga, q_grid_ls;
  // Solis-Wets local search
  int ls_method;     // 0 ADADELTA, 1 Solis-Wets
  float sw_rho, sw_rho_lb, sw_sig_t, sw_sig_ang;
  int sw_max_succ, sw_max_fail;
  // per-run stopping (variable-cost local search or autostop); null active:
  // every run takes every generation
  unsigned int *active;    // [n_runs] 1 while the run continues
  int *last_gen;           // [n_runs] last completed generation
  float *hist;             // [n_runs][10] best energy after each generation (ring)
  int *n_active;           // [G + 1] runs still active after each generation
  int autostop, max_gens;
  double stop_std;
  long long max_evals, max_gen_cost;
  uint32_t k0, k1;
  double cx_rate, mut_rate, tour_p, rho, eps, mut_t, mut_theta, mut_rot;
};

// ligands packed two individuals per wavefront in the local search
constexpr int kDualAtoms = 32, kDualTor = 25;
// chains of generation launches of one docking call, both buckets
constexpr int kMaxChains = 8;
// The ADADELTA local search keeps its pick permutation (pop - 1 ints) in
// the torsion-transform area of the evaluation LDS, which is free until the
// search starts, when it fits (and the launch has no staged pairs);
// otherwise in dynamic LDS.  Capacity: the packed layout's area,
// kDualTor x 12 doubles.
constexpr int kPermAlias = kDualTor * 12 * 2;
__host__ __device__ inline bool perm_aliased(int pop, int stage_pairs) {
  return stage_pairs <= 0 && pop - 1 <= kPermAlias;
}

hipError_t launch_dock_init(const EvalConst &C, int cap, const DockArgs &D, hipStream_t s);
hipError_t launch_ga_generation(const EvalConst &C, int cap, const DockArgs &D, int gen, hipStream_t s);
hipError_t launch_ls_generation(const EvalConst &C, int cap, const DockArgs &D, int gen, hipStream_t s);
size_t ls_dynamic_lds(const EvalConst &C, const DockArgs &D);
// LDS of one local-search work-group of the bucket (static + dynamic, pad
// excluded): the tuner sizes its occupancy candidates from it
size_t ls_workgroup_lds(const EvalConst &C, int cap, const DockArgs &D);
// work-groups of the bucket's GA (kind 0) or local-search (kind 1) kernel
// that the current device keeps resident at once, for D's launch shape: the
// grid of a queued launch
int queue_grid(const EvalConst &C, int cap, const DockArgs &D, int kind);
hipError_t launch_dock_finalize(const DockArgs &D, int buf, float *best_E, float *best_G, hipStream_t s);
hipError_t launch_run_status(const DockArgs &D, int gen, hipStream_t s);
hipError_t launch_solis_wets(const EvalConst &C, int cap, const DockArgs &D, int n, const int *lig_idx, float *geno,
                             float *E, int *used, hipStream_t s);
hipError_t launch_init_genotypes(const GridArgs &G, int n_tor, uint32_t k0, uint32_t k1, uint32_t lig_id, int run,
                                 int pop, float *out, hipStream_t s);
hipError_t launch_score(const EvalConst &C, int cap, int n, const int *lig_idx, const float *geno, float *E, float *G,
                        float *T, hipStream_t s);
hipError_t launch_local_search(const EvalConst &C, int cap, int n, const int *lig_idx, float *geno, float *E,
                               int iters, double rho, double eps, hipStream_t s);
hipError_t launch_build_maps(const MapBuildArgs *dev_args, size_t nn, hipStream_t s);

// static staging block of ad_score_poses_noalloc (sections at fixed offsets,
// each a multiple of 256 bytes)
constexpr int kNoAllocPoses = 4096;
constexpr int kNoAllocDevices = 64;
constexpr size_t kNoAllocIdx = 0;
constexpr size_t kNoAllocGeno = kNoAllocIdx + (size_t)kNoAllocPoses * 4;
constexpr size_t kNoAllocE = kNoAllocGeno + (size_t)kNoAllocPoses * kStride * 4;
constexpr size_t kNoAllocG = kNoAllocE + (size_t)kNoAllocPoses * 4;
constexpr size_t kNoAllocT = kNoAllocG + (size_t)kNoAllocPoses * kStride * 4;
constexpr size_t kNoAllocBytes = kNoAllocT + (size_t)kNoAllocPoses * 3 * 4;
static_assert(kNoAllocGeno % 256 == 0 && kNoAllocE % 256 == 0 && kNoAllocG % 256 == 0 && kNoAllocT % 256 == 0 &&
                  kNoAllocBytes % 256 == 0,
              "noalloc sections are 256-byte aligned");
// once per device, with that device current: takes the device address of the
// static block (kept per device); noalloc_scratch returns it (null before)
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
hipError_t launch_relayout(const float *soa, float *out4, size_t nn, int n_maps, hipStream_t s);

}  // namespace ad

struct ad_batch {
  ad_ctx *ctx = nullptr;
  uint64_t uid = 0;   // unique per context (keys the autotuner's cache)
  int device = 0;
  int n_lig = 0;
  int cap = 64;   // atom capacity of the kernels that serve this batch (64 or 128)
  ad::LigDesc *lig = nullptr;
  ad::AtomGeo *geo = nullptr;
  ad::AtomInfo *info = nullptr;
  ad::PairRec *pairs = nullptr;
  ad::TorRec *tors = nullptr;
  std::vector<ad::LigDesc> lig_host;
  std::vector<int> depth_sum;
  // pre-screen inputs (internal atom order): BF16 features [atoms][32] and
  // neighbour slots [atoms][8]; ps_ok = every atom has <= 8 neighbours
  uint16_t *ps_x = nullptr;
  uint8_t *ps_nbr = nullptr;
  bool ps_ok = true;
  int n_atoms_total = 0;
  int map_of_type[AD_MAX_TYPES];   // map index of each type used by the batch at load time (-1: unused)
};

// a bucket's local-search schedule: staged pair records, pair-loop unroll,
// work-groups resident per CU, persistent work queue
struct LsChoice {
  int stage = 0, unroll = 1, wg_per_cu = 0, queue = 0;
};

struct ad_ctx {
  static constexpr int kScratchSlots = 4;
  // live children (batches, pre-screens): ad_destroy releases their device
  // memory and detaches them, so they may be freed after the context in any
  // order (the free then only deletes the handle)
  std::mutex child_mu;
  std::set<ad_batch *> batches;
  std::set<ad_prescreen *> prescreens;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  ad_forcefield ff;
  ad::FFConst ffc;
  std::vector<ad::LJRec> lj_host;
  ad::LJRec *lj_dev = nullptr;
  double *trig_dev = nullptr;   // sin, cos at multiples of pi/64 (torsion rotations)
  // resident grid
  bool has_grid = false;
  int grid_n[3] = {0, 0, 0};
  double spacing = 0, origin[3] = {0, 0, 0};
  int n_maps = 0;
  int map_types[AD_MAX_TYPES];
  int type_to_map[AD_MAX_TYPES];
  float *maps4 = nullptr;
  size_t maps4_bytes = 0;
  // grow-only scratch buffers
  void *scratch[kScratchSlots] = {nullptr, nullptr, nullptr, nullptr};
  size_t scratch_bytes[kScratchSlots] = {0, 0, 0, 0};
  // kernel timing (HIP events around launches on `stream`)
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pending[AD_KERNEL_KINDS];   // (start, stop) pool indices
  size_t ev_used = 0;
  double t_ms[AD_KERNEL_KINDS] = {0, 0, 0, 0};
  double t_busy[AD_KERNEL_KINDS] = {0, 0, 0, 0};   // union of the launch intervals
  int64_t t_launches[AD_KERNEL_KINDS] = {0, 0, 0, 0};
  // docking state buffers
  void *dock_buf = nullptr;
  size_t dock_bytes = 0;
  // docking schedule: hipGraph replay of the generation loop, autotuned LDS
  // pair staging per atom-capacity bucket (or a forced value), and a second
  // stream so the two buckets' launches overlap
  bool use_graph = true;
  bool autotune = true;
  int forced_stage = -1;
  bool pack_small = true;   // two small ligands' individuals per wavefront in the local search
  // chains of generation launches (ad_set_chains): every bucket's runs in
  // `chains` parts, each on its own stream
  static constexpr int kMaxChainsPerBucket = 4;
  static constexpr int kAuxStreams = 2 * kMaxChainsPerBucket - 1;
  int chains = 2;
  int last_chains[2] = {0, 0};
  hipStream_t aux_streams[kAuxStreams] = {};
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::map<std::vector<int64_t>, LsChoice> tune_cache;
  int forced_unroll = 0, forced_wgcu = 0;   // 0: tuned
  int forced_queue = -1;                     // -1: tuned, 0 off, 1 on
  int last_stage[2] = {-1, -1};
  int last_unroll[2] = {-1, -1}, last_wgcu[2] = {-1, -1}, last_queue[2] = {-1, -1};
  int last_graph = 0;
  int last_packed = 0;      // runs of the last dock call packed two individuals per wavefront
  uint64_t next_batch_uid = 1;
  std::string err;

  int fail(int code, const std::string &msg);
  // timing helpers: mark() before / after a launch of `kind`; collect() after a sync
  // on stream s (null: the context's stream); the first event of a call is
  // the reference the intervals are measured from
  int timing_begin(int kind, hipStream_t s = nullptr);
  void timing_end(int kind, int start, hipStream_t s = nullptr);
  void timing_collect();
  int hip_fail(hipError_t e, const char *where);
  void *scratch_alloc(size_t bytes, int slot);
  ad::EvalConst eval_const(const ad_batch *b) const;
  void free_dock_buffers() {
    if (dock_buf) hipFree(dock_buf);
    dock_buf = nullptr;
    dock_bytes = 0;
  }
};

// Child registry of a context (api.cpp): register / unregister under the
// context's lock; batch_release frees a batch's device memory (idempotent).
void register_batch(ad_ctx *c, ad_batch *b);
void unregister_batch(ad_ctx *c, ad_batch *b);
void batch_release(ad_batch *b);
// pre-screen counterparts (prescreen.hip)
void register_prescreen(ad_ctx *c, ad_prescreen *ps);
void prescreen_release(ad_prescreen *ps);

// Ligand loading without the context's error state (api.cpp): the host
// preparation and upload of ad_load_ligands, and the ligand views of the
// back-to-back layout.  Errors come back in *err.
int load_ligands_impl(ad_ctx *c, int n, const ad_ligand *ligs, uint64_t uid, ad_batch **out, std::string *err);
int packed_views(int n, const int *n_atoms, const int *n_bonds, const int *type_id, const float *charge,
                 const float *xyz, const int *bonds, const unsigned char *rotatable, std::vector<ad_ligand> *out,
                 std::string *err);

namespace ad {
void fill_map_build_args(void *out, const ad_forcefield &ff, const ad_grid_desc *g, int n_rec, const float *xyz,
                         const int *type, const float *q, float *out4, float *soa);
size_t map_build_args_size();
}  // namespace ad
