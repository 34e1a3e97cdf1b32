// Docking entry points: Lamarckian GA with ADADELTA local search on the GPU.
//
// All runs of all ligands advance together, one generation per pair of
// launches (GA step + local-search step) on the context's stream; the
// number of generations is fixed up front from the evaluation cap (every
// generation costs exactly pop-1 + n_ls*ls_iters evaluations), so the host
// never waits on the device inside the loop.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <chrono>
#include <thread>
#include <vector>

#include "api_internal.h"

using namespace ad;

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return (ctx)->hip_fail(_e, #expr); \
  } while (0)

namespace {

int check_params(ad_ctx *c, const ad_dock_params *p) {
  if (!p) return c->fail(AD_E_INVALID, "null params");
  if (p->ls_method != 0 && p->ls_method != 1)
    return c->fail(AD_E_UNSUPPORTED, "ls_method must be 0 (ADADELTA) or 1 (Solis-Wets)");
  if (p->autostop != 0 && p->autostop != 1) return c->fail(AD_E_INVALID, "autostop must be 0 or 1");
  if (p->ls_method == 1 &&
      (!(p->sw_rho > 0.0) || !(p->sw_rho_lb > 0.0) || !std::isfinite(p->sw_rho) || p->sw_max_succ < 1 ||
       p->sw_max_fail < 1 || !(p->sw_sigma_t >= 0.0) || !(p->sw_sigma_ang >= 0.0) || !std::isfinite(p->sw_sigma_t) ||
       !std::isfinite(p->sw_sigma_ang)))
    return c->fail(AD_E_INVALID, "bad Solis-Wets parameters");
  if (p->autostop && (!(p->stop_std >= 0.0) || !std::isfinite(p->stop_std)))
    return c->fail(AD_E_INVALID, "bad autostop threshold");
  if (p->nrun < 1 || p->pop < 2 || p->pop > AD_MAX_POP || p->max_gens < 0 || p->max_evals < 0 || p->ls_iters < 0)
    return c->fail(AD_E_INVALID, "need nrun >= 1, 2 <= pop <= 4096, max_gens, max_evals, ls_iters >= 0");
  const double r[] = {p->ls_rate, p->cx_rate, p->mut_rate, p->tour_p};
  for (double v : r)
    if (!(v >= 0.0 && v <= 1.0)) return c->fail(AD_E_INVALID, "rates must lie in [0, 1]");
  if (!(p->rho >= 0.0 && p->rho < 1.0) || !(p->eps > 0.0) || !std::isfinite(p->eps))
    return c->fail(AD_E_INVALID, "bad ADADELTA rho / eps");
  const double m[] = {p->mut_t, p->mut_theta, p->mut_rot};
  for (double v : m)
    if (!(v >= 0.0) || !std::isfinite(v)) return c->fail(AD_E_INVALID, "bad mutation step");
  return AD_OK;
}

int n_local_search(const ad_dock_params *p) {
  int n = (int)std::floor(p->ls_rate * p->pop + 0.5);
  return std::max(0, std::min(n, p->pop - 1));
}

// generations that fit the caps; every generation costs the same
int generations(const ad_dock_params *p, int n_ls) {
  const int64_t per_gen = (int64_t)(p->pop - 1) + (int64_t)n_ls * p->ls_iters;
  int64_t g = p->max_gens;
  if (p->max_evals < p->pop) return 0;
  if (per_gen > 0) g = std::min<int64_t>(g, (p->max_evals - p->pop) / per_gen);
  return (int)g;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// auxiliary streams for `n` chains beyond the first, and the fork / join
// events
int ensure_aux(ad_ctx *c, int n) {
  if (!c->ev_fork && (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess))
    return c->fail(AD_E_HIP, "cannot create the docking events");
  for (int i = 0; i < n && i < ad_ctx::kAuxStreams; ++i)
    if (!c->aux_streams[i] && hipStreamCreateWithFlags(&c->aux_streams[i], hipStreamNonBlocking) != hipSuccess)
      return c->fail(AD_E_HIP, "cannot create an auxiliary stream");
  return AD_OK;
}

// LDS pair-staging candidates of the local-search kernel, within the
// work-group's LDS budget
std::vector<int> stage_candidates(const EvalConst &C, const DockArgs &D, int cap, int max_pairs) {
  std::vector<int> out = {0};
  for (int ns : {128, 256, 512, 1024, 2048}) {
    DockArgs t = D;
    t.stage_pairs = ns;
    if (ls_workgroup_lds(C, cap, t) > 64 * 1024) break;
    out.push_back(ns);
    if (ns >= max_pairs) break;   // every pair of the bucket already staged
  }
  return out;
}

// Launch schedule of one bucket's local search, chosen by timing: the shape
// (pair loop one or two steps per trip; work-groups resident per CU: as many
// as the LDS allows, three quarters or half of that, set by padding the
// dynamic LDS), the persistent work queue (a bucket of one chain only) and
// the number of pair records staged in LDS.  Timing runs the bucket's
// local search (few iterations) from the evaluated initial population on a
// copy of the population buffers, once per candidate (best of three), on a
// strided sample of its runs; the docking state itself is not touched.
// Every candidate computes bitwise the same values, so the choice affects
// speed only.  A candidate replaces the default (one step per trip, full
// occupancy, no queue, no staging) only if it is 3 % faster.  Forced values (ad_set_schedule,
// ad_set_launch_shape) are taken as given.
constexpr int kLdsPerCU = 160 * 1024;
constexpr int kMaxWgPerCU = 16;   // 4 one-wavefront work-groups per SIMD (the kernel's VGPR budget)

int natural_wg_per_cu(size_t lds) { return std::max(1, std::min(kMaxWgPerCU, (int)(kLdsPerCU / std::max<size_t>(lds, 1)))); }

// dynamic-LDS pad that leaves `target` work-groups per CU (0: none needed)
int pad_for(size_t lds, int target) {
  if (target <= 0 || target >= natural_wg_per_cu(lds)) return 0;
  const size_t want = ((size_t)(kLdsPerCU / target) / 512) * 512;   // an LDS granule below 1/target of the CU
  return want > lds ? (int)(want - lds) : 0;
}

int choose_schedule(ad_ctx *c, const ad_batch *b, const int *sel, int n_lig, const EvalConst &C, const DockArgs &Dk,
                    int cap, int max_pairs, bool stage_ok, bool chained, LsChoice *out) {
  const int bk = cap > 64 ? 1 : 0;
  LsChoice best;
  best.stage = 0;
  best.unroll = c->forced_unroll > 0 ? c->forced_unroll : 1;
  best.wg_per_cu = 0;
  const size_t lds0 = ls_workgroup_lds(C, cap, Dk);
  const int natural = natural_wg_per_cu(lds0);
  const std::vector<int> stage_cand = stage_ok ? stage_candidates(C, Dk, cap, max_pairs) : std::vector<int>{0};
  if (c->forced_wgcu > 0) best.wg_per_cu = std::min(c->forced_wgcu, natural);
  if (c->forced_stage >= 0)
    for (int ns : stage_cand)
      if (ns <= c->forced_stage) best.stage = ns;
  best.queue = c->forced_queue > 0 ? 1 : 0;
  const bool tune_shape = c->autotune && (c->forced_unroll <= 0 || c->forced_wgcu <= 0);
  const bool tune_stage = c->autotune && c->forced_stage < 0 && stage_cand.size() > 1;
  // The queue's gain is a launch's tail, which a bucket split into several
  // chains already fills from the other chains' launches; the timing sample
  // (one launch of a part of the runs) shows the tail but not the chains, so
  // the queue is tuned only for a bucket that runs as one chain.
  const bool tune_queue = c->autotune && c->forced_queue < 0 && !chained;
  if (!tune_shape && !tune_stage && !tune_queue) {
    if (best.wg_per_cu <= 0) best.wg_per_cu = natural;
    *out = best;
    return AD_OK;
  }
  std::vector<int64_t> key = {(int64_t)b->uid, cap, Dk.pop, Dk.n_ls, Dk.n_launch, n_lig, Dk.n_dual,
                              c->forced_unroll, c->forced_wgcu, c->forced_stage, c->forced_queue, chained ? 1 : 0};
  if (sel) {
    uint64_t h = 1469598103934665603ull;
    for (int l = 0; l < n_lig; ++l) h = (h ^ (uint64_t)sel[l]) * 1099511628211ull;
    key.push_back((int64_t)h);
  }
  auto it = c->tune_cache.find(key);
  if (it != c->tune_cache.end()) {
    *out = it->second;
    return AD_OK;
  }
  // timing sample: single-wavefront runs when the bucket has any (packed
  // runs take the same shape), else its first whole packed ligands
  const int n_single = Dk.n_launch - Dk.n_dual;
  const size_t pop_floats = (size_t)Dk.n_runs * Dk.pop;
  const size_t sz_g = align256(pop_floats * kStride * sizeof(float));
  const size_t sz_e = align256(pop_floats * sizeof(float));
  const size_t sz_v = align256((size_t)Dk.n_runs * sizeof(unsigned long long));
  const size_t sz_o = align256((size_t)Dk.n_launch * sizeof(int));
  const size_t sz_q = 256;
  char *blk = (char *)c->scratch_alloc(sz_g + sz_e + sz_v + sz_o + sz_q, 3);
  if (!blk) return c->fail(AD_E_OOM, "cannot allocate autotuning buffers");
  std::vector<int> host_order(Dk.n_launch), sample;
  HIP_TRY(c, hipMemcpyAsync(host_order.data(), Dk.run_order, Dk.n_launch * sizeof(int), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  DockArgs T = Dk;
  if (n_single > 0) {
    const int K = std::min(n_single, std::max(1, 3072 / std::max(1, Dk.n_ls)) * 2);
    for (int k = 0; k < K; ++k) sample.push_back(host_order[Dk.n_dual + (size_t)k * n_single / K]);
    T.n_dual = 0;
  } else {
    const int lig_runs = std::max(1, std::min(Dk.n_dual / Dk.nrun, std::max(1, 6144 / std::max(1, Dk.nrun * Dk.n_ls))));
    sample.assign(host_order.begin(), host_order.begin() + (size_t)lig_runs * Dk.nrun);
    T.n_dual = (int)sample.size();
  }
  T.geno = (float *)blk;
  T.energy = (float *)(blk + sz_g);
  T.evals = (unsigned long long *)(blk + sz_g + sz_e);
  int *d_sample = (int *)(blk + sz_g + sz_e + sz_v);
  unsigned int *d_q = (unsigned int *)(blk + sz_g + sz_e + sz_v + sz_o);
  T.run_order = d_sample;
  T.q_ga = nullptr;
  T.n_launch = (int)sample.size();
  T.ls_iters = std::min(Dk.ls_iters, 24);
  HIP_TRY(c, hipMemcpyAsync(d_sample, sample.data(), sample.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  int rc = AD_OK;
  auto time_ms = [&](const LsChoice &ch, float *ms_out) {
    T.stage_pairs = ch.stage;
    T.ls_unroll = ch.unroll;
    T.ls_pad = pad_for(ls_workgroup_lds(C, cap, T), ch.wg_per_cu);
    T.q_ls = ch.queue ? d_q : nullptr;
    T.q_grid_ls = ch.queue ? queue_grid(C, cap, T, 1) : 0;
    float ms_min = INFINITY;
    for (int rep = 0; rep < 3 && rc == AD_OK; ++rep) {
      hipError_t e = hipMemcpyAsync(T.geno, Dk.geno, pop_floats * kStride * sizeof(float), hipMemcpyDeviceToDevice,
                                    c->stream);
      if (e == hipSuccess && ch.queue) e = hipMemsetAsync(d_q, 0, sizeof(unsigned int), c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(T.energy, Dk.energy, pop_floats * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
      if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
      if (e == hipSuccess) e = launch_ls_generation(C, cap, T, 0, c->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) rc = c->hip_fail(e, "autotuning launch");
      ms_min = std::min(ms_min, ms);
    }
    *ms_out = ms_min;
  };
  if (best.wg_per_cu <= 0) best.wg_per_cu = natural;
  float best_ms = INFINITY;
  time_ms(best, &best_ms);
  if (tune_shape) {
    std::vector<int> unrolls = c->forced_unroll > 0 ? std::vector<int>{c->forced_unroll} : std::vector<int>{1, 2};
    std::vector<int> occ = c->forced_wgcu > 0 ? std::vector<int>{best.wg_per_cu}
                                              : std::vector<int>{natural, (3 * natural + 2) / 4, (natural + 1) / 2};
    const LsChoice base = best;
    for (int u : unrolls)
      for (int w : occ) {
        LsChoice ch = base;
        ch.unroll = u;
        ch.wg_per_cu = std::max(1, w);
        if (ch.unroll == base.unroll && ch.wg_per_cu == base.wg_per_cu) continue;
        float ms;
        time_ms(ch, &ms);
        if (rc) break;
        if (ms < 0.97f * best_ms) {
          best_ms = ms;
          best = ch;
        }
      }
  }
  if (tune_queue && rc == AD_OK) {
    // the persistent work queue against one work-group per item, with the
    // shape chosen so far
    LsChoice ch = best;
    ch.queue = 1 - best.queue;
    float ms;
    time_ms(ch, &ms);
    if (rc == AD_OK && ms < 0.97f * best_ms) {
      best_ms = ms;
      best = ch;
    }
  }
  if (tune_stage && rc == AD_OK) {
    // staged records run the plain (unroll 1) loop; a larger staging size
    // must win by 3 % (timing noise and the LDS it takes from co-resident
    // work-groups of other launches)
    for (int ns : stage_cand) {
      if (ns == 0) continue;
      LsChoice ch = best;
      ch.stage = ns;
      ch.unroll = 1;
      float ms;
      time_ms(ch, &ms);
      if (rc) break;
      if (ms < 0.97f * best_ms) {
        best_ms = ms;
        best = ch;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  (void)bk;
  c->tune_cache[key] = best;
  *out = best;
  return AD_OK;
}

}  // namespace

// Docks n_lig ligands of batch b: sel[l] is the batch index of the l-th
// (null: 0..n_lig-1); ids[l] its random-stream id (null: the batch index).
int dock_impl(ad_ctx *c, const ad_batch *b, int n_lig, const int *sel, const ad_dock_params *p, uint64_t seed,
              const uint32_t *lig_ids, ad_dock_result *out, float *run_energy, float *run_genotype) {
  if (!c) return AD_E_INVALID;
  if (!b) return c->fail(AD_E_INVALID, "null batch");
  if (b->ctx != c) return c->fail(AD_E_INVALID, "batch belongs to another context");
  if (!c->has_grid) return c->fail(AD_E_STATE, "no grid loaded");
  for (int t = 0; t < AD_MAX_TYPES; ++t)
    if (b->map_of_type[t] >= 0 && c->type_to_map[t] != b->map_of_type[t])
      return c->fail(AD_E_STATE, "grid maps changed since the batch was loaded; reload the ligands");
  int rc = check_params(c, p);
  if (rc) return rc;
  if (n_lig < 0) return c->fail(AD_E_INVALID, "n < 0");
  if (n_lig == 0) return AD_OK;
  if (!out) return c->fail(AD_E_INVALID, "null result array");
  if (sel)
    for (int l = 0; l < n_lig; ++l)
      if (sel[l] < 0 || sel[l] >= b->n_lig) return c->fail(AD_E_INVALID, "ligand index out of range");
  auto bidx = [&](int l) { return sel ? sel[l] : l; };
  int cap = 64;
  for (int l = 0; l < n_lig; ++l)
    if (b->lig_host[bidx(l)].n_atoms > 64) cap = 128;
  if ((int64_t)n_lig * p->nrun * p->pop > (int64_t)1 << 31)
    return c->fail(AD_E_INVALID, "n_lig * nrun * pop too large for one batch");
  const int n_runs = n_lig * p->nrun;
  const int n_ls = n_local_search(p);
  // Fixed-cost schedule (ADADELTA without autostop): every run takes exactly
  // G generations.  Otherwise runs stop on their own (k_run_status) and G
  // is the most that the cheapest generations (no local-search evaluation)
  // could reach.
  const bool per_run = p->ls_method == 1 || p->autostop;
  int G = generations(p, n_ls);
  if (per_run) {
    ad_dock_params q = *p;
    q.ls_iters = 0;
    G = generations(&q, n_ls);
  }

  // device state, carved out of one grow-only buffer
  const size_t sz_geno = align256((size_t)2 * n_runs * p->pop * kStride * sizeof(float));
  const size_t sz_E = align256((size_t)2 * n_runs * p->pop * sizeof(float));
  const size_t sz_ev = align256((size_t)n_runs * sizeof(unsigned long long));
  const size_t sz_ord = align256((size_t)n_runs * sizeof(int));
  const size_t sz_id = align256((size_t)n_lig * sizeof(uint32_t));
  const size_t sz_bE = align256((size_t)n_runs * sizeof(float));
  const size_t sz_bG = align256((size_t)n_runs * kStride * sizeof(float));
  const size_t sz_lG = align256((size_t)n_lig * kStride * sizeof(float));
  const size_t sz_lE = align256((size_t)n_lig * sizeof(float));
  const size_t sz_lT = align256((size_t)n_lig * 3 * sizeof(float));
  const size_t sz_li = align256((size_t)n_lig * sizeof(int));
  const size_t sz_map = sel ? align256((size_t)n_lig * sizeof(int)) : 0;
  const size_t sz_rl = align256((size_t)n_runs * sizeof(int));
  const size_t sz_act = per_run ? align256((size_t)n_runs * sizeof(unsigned int)) : 0;
  const size_t sz_lgen = per_run ? align256((size_t)n_runs * sizeof(int)) : 0;
  const size_t sz_hist = per_run ? align256((size_t)n_runs * 10 * sizeof(float)) : 0;
  const size_t sz_nact = per_run ? align256((size_t)(G + 1) * sizeof(int)) : 0;
  // work-queue tickets: [chain][GA, local search][generation 0..G]
  static_assert(kMaxChains == 2 * ad_ctx::kMaxChainsPerBucket, "two buckets");
  const size_t sz_q = align256((size_t)2 * kMaxChains * (G + 1) * sizeof(unsigned int));
  const size_t total = sz_geno + sz_E + sz_ev + sz_ord + sz_id + sz_bE + sz_bG + sz_lG + sz_lE + sz_lT + sz_li +
                       sz_map + sz_rl + sz_act + sz_lgen + sz_hist + sz_nact + sz_q;
  hipSetDevice(c->device);
  if (c->dock_bytes < total) {
    hipStreamSynchronize(c->stream);
    c->free_dock_buffers();
    if (hipMalloc(&c->dock_buf, total) != hipSuccess) return c->fail(AD_E_OOM, "cannot allocate docking state");
    c->dock_bytes = total;
  }
  char *base = (char *)c->dock_buf;
  size_t o = 0;
  auto carve = [&](size_t sz) {
    char *ptr = base + o;
    o += sz;
    return ptr;
  };
  DockArgs D;
  memset(&D, 0, sizeof(D));
  D.ls_unroll = 1;
  D.geno = (float *)carve(sz_geno);
  D.energy = (float *)carve(sz_E);
  D.evals = (unsigned long long *)carve(sz_ev);
  int *d_order = (int *)carve(sz_ord);
  uint32_t *d_id = (uint32_t *)carve(sz_id);
  float *d_bE = (float *)carve(sz_bE);
  float *d_bG = (float *)carve(sz_bG);
  float *d_lG = (float *)carve(sz_lG);
  float *d_lE = (float *)carve(sz_lE);
  float *d_lT = (float *)carve(sz_lT);
  int *d_li = (int *)carve(sz_li);
  int *d_map = sel ? (int *)carve(sz_map) : nullptr;
  int *d_rl = (int *)carve(sz_rl);
  D.active = per_run ? (unsigned int *)carve(sz_act) : nullptr;
  D.last_gen = per_run ? (int *)carve(sz_lgen) : nullptr;
  D.hist = per_run ? (float *)carve(sz_hist) : nullptr;
  D.n_active = per_run ? (int *)carve(sz_nact) : nullptr;
  unsigned int *d_q = (unsigned int *)carve(sz_q);
  D.run_order = d_order;
  D.n_dual = 0;
  D.lig_id = d_id;
  D.lig_map = d_map;
  D.ls_method = p->ls_method;
  D.sw_rho = (float)p->sw_rho;
  D.sw_rho_lb = (float)p->sw_rho_lb;
  D.sw_sig_t = (float)p->sw_sigma_t;
  D.sw_sig_ang = (float)p->sw_sigma_ang;
  D.sw_max_succ = p->sw_max_succ;
  D.sw_max_fail = p->sw_max_fail;
  D.autostop = p->autostop;
  D.max_gens = p->max_gens;
  D.stop_std = p->stop_std;
  D.max_evals = (long long)p->max_evals;
  D.max_gen_cost = (long long)(p->pop - 1) + (long long)n_ls * p->ls_iters;
  D.n_runs = n_runs;
  D.nrun = p->nrun;
  D.pop = p->pop;
  D.n_ls = n_ls;
  D.ls_iters = p->ls_iters;
  D.k0 = (uint32_t)seed;
  D.k1 = (uint32_t)(seed >> 32);
  D.cx_rate = p->cx_rate;
  D.mut_rate = p->mut_rate;
  D.tour_p = p->tour_p;
  D.rho = p->rho;
  D.eps = p->eps;
  D.mut_t = p->mut_t;
  D.mut_theta = p->mut_theta;
  D.mut_rot = p->mut_rot;

  // runs grouped by kernel atom capacity (bucket 0: <= 64 atoms, bucket 1:
  // <= 128), each bucket in longest-processing-time order so the last
  // work-groups of every launch are the cheap ones.  ADADELTA runs of small
  // ligands (at most kDualAtoms atoms and kDualTor torsions) go first in
  // bucket 0, as whole ligands: their local search packs two individuals per
  // wavefront.  A bucket is split into `parts` chains (ad_set_chains): part k
  // takes every parts-th packed ligand and every parts-th one-wavefront run
  // of that order, and runs its generations on a stream of its own.
  const bool pack = c->pack_small && p->ls_method == 0 && n_ls > 0 && p->ls_iters > 0;
  std::vector<double> cost(n_lig);
  std::vector<int> bucket_of(n_lig), packed(n_lig);
  for (int l = 0; l < n_lig; ++l) {
    const LigDesc &d = b->lig_host[bidx(l)];
    cost[l] = d.n_pairs + 4.0 * d.n_atoms + 2.0 * d.n_tor;
    bucket_of[l] = d.n_atoms > 64 ? 1 : 0;
    packed[l] = pack && d.n_atoms <= kDualAtoms && d.n_tor <= kDualTor;
  }
  struct Chain {
    int bk, start, n, n_dual;
    DockArgs D;
  };
  std::vector<Chain> chains;
  std::vector<int> order;
  order.reserve(n_runs);
  int n_dual = 0;
  for (int bk = 0; bk < 2; ++bk) {
    std::vector<int> ligs;
    for (int l = 0; l < n_lig; ++l)
      if (bucket_of[l] == bk) ligs.push_back(l);
    std::stable_sort(ligs.begin(), ligs.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    std::vector<int> lig_packed, singles;
    for (int l : ligs) {
      if (packed[l]) lig_packed.push_back(l);
      else
        for (int r = 0; r < p->nrun; ++r) singles.push_back(l * p->nrun + r);
    }
    // runs that stop on their own meet after every generation (status
    // kernel), where split launches would only add tails: one part
    const int units = (int)(lig_packed.size() + singles.size());
    const int parts = per_run ? 1 : std::max(1, std::min(c->chains, units));
    for (int pt = 0; pt < parts; ++pt) {
      Chain ch{bk, (int)order.size(), 0, 0, D};
      for (size_t k = pt; k < lig_packed.size(); k += parts)
        for (int r = 0; r < p->nrun; ++r) order.push_back(lig_packed[k] * p->nrun + r);
      ch.n_dual = (int)order.size() - ch.start;
      for (size_t k = pt; k < singles.size(); k += parts) order.push_back(singles[k]);
      ch.n = (int)order.size() - ch.start;
      n_dual += ch.n_dual;
      if (ch.n > 0) chains.push_back(ch);
    }
  }
  std::vector<uint32_t> ids(n_lig);
  for (int l = 0; l < n_lig; ++l) ids[l] = lig_ids ? lig_ids[l] : (uint32_t)bidx(l);
  HIP_TRY(c, hipMemcpyAsync(d_order, order.data(), n_runs * sizeof(int), hipMemcpyHostToDevice, c->stream));
  if (sel) HIP_TRY(c, hipMemcpyAsync(d_map, sel, n_lig * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_id, ids.data(), n_lig * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(D.evals, 0, (size_t)n_runs * sizeof(unsigned long long), c->stream));
  if (per_run) {
    HIP_TRY(c, hipMemsetAsync(D.active, 1, (size_t)n_runs * sizeof(unsigned int), c->stream));
    HIP_TRY(c, hipMemsetAsync(D.last_gen, 0, (size_t)n_runs * sizeof(int), c->stream));
    HIP_TRY(c, hipMemsetAsync(D.n_active, 0, (size_t)(G + 1) * sizeof(int), c->stream));
  }

  const EvalConst C = c->eval_const(b);
  int max_pairs[2] = {0, 0};
  for (int l = 0; l < n_lig; ++l)
    max_pairs[bucket_of[l]] = std::max(max_pairs[bucket_of[l]], b->lig_host[bidx(l)].n_pairs);
  const int n_chains = (int)chains.size();
  for (Chain &ch : chains) {
    ch.D.run_order = d_order + ch.start;
    ch.D.n_launch = ch.n;
    ch.D.stage_pairs = 0;
    ch.D.n_dual = ch.n_dual;
  }
  {
    const int t0 = c->timing_begin(0);
    for (const Chain &ch : chains) HIP_TRY(c, launch_dock_init(C, ch.bk ? 128 : 64, ch.D, c->stream));
    c->timing_end(0, t0);
  }
  const bool do_ls = n_ls > 0 && p->ls_iters > 0;
  HIP_TRY(c, hipMemsetAsync(d_q, 0, sz_q, c->stream));
  for (int bk = 0; bk < 2; ++bk) {
    c->last_stage[bk] = -1;
    c->last_unroll[bk] = -1;
    c->last_wgcu[bk] = -1;
    c->last_queue[bk] = -1;
    c->last_chains[bk] = 0;
    int first = -1;
    for (int i = 0; i < n_chains; ++i)
      if (chains[i].bk == bk) {
        if (first < 0) first = i;
        ++c->last_chains[bk];
      }
    if (first < 0) continue;
    const int cap_b = bk ? 128 : 64;
    // the GA launches take the bucket's queue mode: the local search's
    // (tuned or forced) under ADADELTA, else the forced one.  The tuner
    // times the bucket's first part; every part takes its choice.
    int queue = c->forced_queue > 0 ? 1 : 0;
    LsChoice ch;
    bool tuned = false;
    if (do_ls && p->ls_method == 1) {   // Solis-Wets: its own kernel, one fixed shape
      c->last_stage[bk] = 0;
    } else if (do_ls) {
      // packed runs stage no pairs; their launch still takes the tuned shape
      bool stage_ok = true;
      int bk_chains = 0;
      for (const Chain &x : chains)
        if (x.bk == bk) {
          ++bk_chains;
          if (x.n_dual > 0) stage_ok = false;
        }
      rc = choose_schedule(c, b, sel, n_lig, C, chains[first].D, cap_b, max_pairs[bk], stage_ok, bk_chains > 1, &ch);
      if (rc) return rc;
      tuned = true;
      c->last_stage[bk] = ch.stage;
      c->last_unroll[bk] = ch.unroll;
      c->last_wgcu[bk] = ch.wg_per_cu;
      queue = ch.queue;
    }
    for (int i = 0; i < n_chains; ++i) {
      if (chains[i].bk != bk) continue;
      DockArgs &Dc = chains[i].D;
      if (tuned) {
        Dc.stage_pairs = ch.stage;
        Dc.ls_unroll = ch.unroll;
        Dc.ls_pad = pad_for(ls_workgroup_lds(C, cap_b, Dc), ch.wg_per_cu);
      }
      if (queue) {
        Dc.q_ga = d_q + (size_t)(2 * i) * (G + 1);
        Dc.q_grid_ga = queue_grid(C, cap_b, Dc, 0);
        if (tuned) {
          Dc.q_ls = d_q + (size_t)(2 * i + 1) * (G + 1);
          Dc.q_grid_ls = queue_grid(C, cap_b, Dc, 1);
        }
        if (Dc.q_grid_ga <= 0 || (tuned && Dc.q_grid_ls <= 0))
          return c->fail(AD_E_HIP, "cannot size the work-queue grid");
      }
    }
    c->last_queue[bk] = queue;
  }

  // the generation loop: chain 0 on the context's stream, the others on
  // auxiliary streams; the chains meet only at the end (with per-run
  // stopping, after every generation, for the status kernel).  Eager with
  // kernel timing (an event pair around every launch, on its stream),
  // otherwise captured once into a graph and replayed.
  rc = ensure_aux(c, n_chains - 1);
  if (rc) return rc;
  std::vector<hipStream_t> cs(n_chains);
  for (int i = 0; i < n_chains; ++i) cs[i] = i == 0 ? c->stream : c->aux_streams[i - 1];
  auto fork = [&]() -> hipError_t {
    if (n_chains < 2) return hipSuccess;
    hipError_t e = hipEventRecord(c->ev_fork, c->stream);
    for (int i = 1; i < n_chains && e == hipSuccess; ++i) e = hipStreamWaitEvent(cs[i], c->ev_fork, 0);
    return e;
  };
  auto join = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (int i = 1; i < n_chains && e == hipSuccess; ++i) {
      e = hipEventRecord(c->ev_join, cs[i]);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->ev_join, 0);
    }
    return e;
  };
  // one generation of chain i (GA, then local search), each launch timed
  auto generation = [&](int i, int gen) -> hipError_t {
    const Chain &ch = chains[i];
    const int cap_i = ch.bk ? 128 : 64;
    const int t1 = c->timing_begin(1, cs[i]);
    hipError_t e = launch_ga_generation(C, cap_i, ch.D, gen, cs[i]);
    c->timing_end(1, t1, cs[i]);
    if (e == hipSuccess && do_ls) {
      const int t2 = c->timing_begin(2, cs[i]);
      e = launch_ls_generation(C, cap_i, ch.D, gen, cs[i]);
      c->timing_end(2, t2, cs[i]);
    }
    return e;
  };
  const bool graph = c->use_graph && !c->timing && G > 0 && !per_run;
  c->last_graph = graph ? 1 : 0;
  c->last_packed = n_dual;
  if (per_run) {
    // generations until every run has stopped: the status kernel decides
    // per run after each generation; the host looks every 16 generations
    HIP_TRY(c, launch_run_status(D, 0, c->stream));
    for (int gen = 1; gen <= G; ++gen) {
      HIP_TRY(c, fork());
      for (int i = 0; i < n_chains; ++i) HIP_TRY(c, generation(i, gen));
      HIP_TRY(c, join());
      HIP_TRY(c, launch_run_status(D, gen, c->stream));
      if (gen % 16 == 0 || gen == G) {
        int n_act = 0;
        HIP_TRY(c, hipMemcpyAsync(&n_act, D.n_active + gen, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (n_act == 0) break;
      }
    }
  } else if (!graph) {
    // generation-major, so every stream is fed as the loop goes
    HIP_TRY(c, fork());
    for (int gen = 1; gen <= G; ++gen)
      for (int i = 0; i < n_chains; ++i) HIP_TRY(c, generation(i, gen));
    HIP_TRY(c, join());
  } else {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = fork();
    for (int gen = 1; gen <= G && e == hipSuccess; ++gen)
      for (int i = 0; i < n_chains && e == hipSuccess; ++i) e = generation(i, gen);
    if (e == hipSuccess) e = join();
    const hipError_t e_end = hipStreamEndCapture(c->stream, &g);
    if (e != hipSuccess || e_end != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return c->hip_fail(e != hipSuccess ? e : e_end, "capture of the generation loop");
    }
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (ge) hipGraphExecDestroy(ge);
    hipGraphDestroy(g);
    if (e != hipSuccess) return c->hip_fail(e, "generation-loop graph");
  }
  HIP_TRY(c, launch_dock_finalize(D, G & 1, d_bE, d_bG, c->stream));
  if (n_dual > 0) {
    // the packed local search sums a pose's energy in another order (one
    // wavefront half); report every run's best energy as the one-wavefront
    // evaluation gives it, so that it re-scores bitwise (ad_score_poses)
    std::vector<int> rl(n_runs);
    for (int R = 0; R < n_runs; ++R) rl[R] = bidx(R / p->nrun);
    HIP_TRY(c, hipMemcpyAsync(d_rl, rl.data(), n_runs * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_score(C, cap, n_runs, d_rl, d_bG, d_bE, nullptr, nullptr, c->stream));
  }

  std::vector<float> bE(n_runs), bG((size_t)n_runs * kStride);
  std::vector<unsigned long long> ev(n_runs);
  std::vector<int> run_gens(n_runs, G);
  if (per_run)
    HIP_TRY(c, hipMemcpyAsync(run_gens.data(), D.last_gen, n_runs * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bE.data(), d_bE, n_runs * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bG.data(), d_bG, (size_t)n_runs * kStride * sizeof(float), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(ev.data(), D.evals, n_runs * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timing_collect();

  // best run per ligand (lowest energy, lowest run index on ties), then its
  // score terms from one more scoring launch
  std::vector<int> best_run(n_lig), lidx(n_lig);
  std::vector<float> lG((size_t)n_lig * kStride);
  for (int l = 0; l < n_lig; ++l) {
    int br = 0;
    for (int r = 1; r < p->nrun; ++r) {
      float e = bE[l * p->nrun + r], eb = bE[l * p->nrun + br];
      if (e < eb || (std::isnan(eb) && !std::isnan(e))) br = r;
    }
    best_run[l] = br;
    lidx[l] = bidx(l);
    memcpy(&lG[(size_t)l * kStride], &bG[(size_t)(l * p->nrun + br) * kStride], kStride * sizeof(float));
  }
  HIP_TRY(c, hipMemcpyAsync(d_lG, lG.data(), lG.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_li, lidx.data(), n_lig * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_score(C, cap, n_lig, d_li, d_lG, d_lE, nullptr, d_lT, c->stream));
  std::vector<float> lT((size_t)n_lig * 3);
  HIP_TRY(c, hipMemcpyAsync(lT.data(), d_lT, lT.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));

  for (int l = 0; l < n_lig; ++l) {
    ad_dock_result &r = out[l];
    const int R = l * p->nrun + best_run[l];
    r.best_energy = bE[R];
    r.best_score = lT[(size_t)l * 3 + 2];
    memcpy(r.best_genotype, &lG[(size_t)l * kStride], kStride * sizeof(float));
    r.best_run = best_run[l];
    r.generations = run_gens[R];
    int64_t e = 0;
    for (int q = 0; q < p->nrun; ++q) e += (int64_t)ev[l * p->nrun + q];
    r.evals = e;
  }
  if (run_energy) memcpy(run_energy, bE.data(), n_runs * sizeof(float));
  if (run_genotype) memcpy(run_genotype, bG.data(), (size_t)n_runs * kStride * sizeof(float));
  return AD_OK;
}

extern "C" int ad_dock_batch(ad_ctx *c, const ad_batch *b, const ad_dock_params *p, uint64_t seed,
                             const uint32_t *lig_ids, ad_dock_result *out, float *run_energy, float *run_genotype) {
  if (!c) return AD_E_INVALID;
  if (!b) return c->fail(AD_E_INVALID, "null batch");
  return dock_impl(c, b, b->n_lig, nullptr, p, seed, lig_ids, out, run_energy, run_genotype);
}

extern "C" int ad_dock_select(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, const ad_dock_params *p,
                              uint64_t seed, ad_dock_result *out, float *run_energy, float *run_genotype) {
  if (!c) return AD_E_INVALID;
  if (n > 0 && !lig_idx) return c->fail(AD_E_INVALID, "null ligand index list");
  return dock_impl(c, b, n, lig_idx, p, seed, nullptr, out, run_energy, run_genotype);
}

extern "C" int ad_dock_stream(ad_ctx *c, int n, const int *n_atoms, const int *n_bonds, const int *type_id,
                              const float *charge, const float *xyz, const int *bonds, const unsigned char *rotatable,
                              int batch_size, const ad_dock_params *p, uint64_t seed, uint32_t id0,
                              ad_dock_result *out, double *stats) {
  if (!c) return AD_E_INVALID;
  if (!c->has_grid) return c->fail(AD_E_STATE, "load or build grids before ligands");
  if (batch_size < 1) return c->fail(AD_E_INVALID, "batch_size must be >= 1");
  if (n > 0 && !out) return c->fail(AD_E_INVALID, "null result array");
  int rc = check_params(c, p);
  if (rc) return rc;
  std::vector<ad_ligand> v;
  std::string err;
  rc = packed_views(n, n_atoms, n_bonds, type_id, charge, xyz, bonds, rotatable, &v, &err);
  if (rc) return c->fail(rc, err);
  using clk = std::chrono::steady_clock;
  const auto t_wall = clk::now();
  double prep_s = 0.0, dock_s = 0.0;
  // batch k: ligands [k * batch_size, ...); its host preparation and upload
  // run on a worker thread while batch k - 1 docks
  auto load = [&](int k, ad_batch **b, std::string *e) -> int {
    const auto t0 = clk::now();
    const int lo = k * batch_size, cnt = std::min(batch_size, n - lo);
    const int r = load_ligands_impl(c, cnt, v.data() + lo, c->next_batch_uid++, b, e);
    prep_s += std::chrono::duration<double>(clk::now() - t0).count();
    return r;
  };
  const int n_batches = (n + batch_size - 1) / batch_size;
  ad_batch *cur = nullptr;
  if (n_batches > 0) {
    rc = load(0, &cur, &err);
    if (rc) return c->fail(rc, err);
  }
  for (int k = 0; k < n_batches; ++k) {
    const int lo = k * batch_size, cnt = std::min(batch_size, n - lo);
    ad_batch *next = nullptr;
    int rc_next = AD_OK;
    std::string err_next;
    std::thread worker;
    if (k + 1 < n_batches) worker = std::thread([&]() { rc_next = load(k + 1, &next, &err_next); });
    // random-stream id = id0 + index in the set: results do not depend on the batching
    std::vector<uint32_t> ids(cnt);
    for (int l = 0; l < cnt; ++l) ids[l] = id0 + (uint32_t)(lo + l);
    const auto t0 = clk::now();
    rc = dock_impl(c, cur, cnt, nullptr, p, seed, ids.data(), out + lo, nullptr, nullptr);
    dock_s += std::chrono::duration<double>(clk::now() - t0).count();
    if (worker.joinable()) worker.join();
    ad_free_batch(cur);
    cur = next;
    if (rc) {
      if (cur) ad_free_batch(cur);
      return rc;
    }
    if (rc_next) {
      if (cur) ad_free_batch(cur);
      return c->fail(rc_next, "batch " + std::to_string(k + 1) + ", " + err_next);
    }
  }
  if (stats) {
    stats[0] = prep_s;
    stats[1] = dock_s;
    stats[2] = std::chrono::duration<double>(clk::now() - t_wall).count();
  }
  return AD_OK;
}

extern "C" int ad_set_schedule(ad_ctx *c, int use_graph, int autotune, int stage_pairs, int pack_small) {
  if (!c) return AD_E_INVALID;
  c->use_graph = use_graph != 0;
  c->pack_small = pack_small != 0;
  c->autotune = autotune != 0;
  c->forced_stage = stage_pairs < 0 ? -1 : stage_pairs;
  return AD_OK;
}

extern "C" int ad_set_launch_shape(ad_ctx *c, int unroll, int wg_per_cu) {
  if (!c) return AD_E_INVALID;
  if (unroll < 0 || unroll > 2 || wg_per_cu < 0 || wg_per_cu > 64)
    return c->fail(AD_E_INVALID, "launch shape: unroll 0 (tune), 1 or 2; wg_per_cu 0 (tune) or 1..64");
  c->forced_unroll = unroll;
  c->forced_wgcu = wg_per_cu;
  return AD_OK;
}

extern "C" int ad_get_launch_shape(ad_ctx *c, int *unroll, int *wg_per_cu) {
  if (!c) return AD_E_INVALID;
  for (int bk = 0; bk < 2; ++bk) {
    if (unroll) unroll[bk] = c->last_unroll[bk];
    if (wg_per_cu) wg_per_cu[bk] = c->last_wgcu[bk];
  }
  return AD_OK;
}

extern "C" int ad_set_work_queue(ad_ctx *c, int mode) {
  if (!c) return AD_E_INVALID;
  if (mode < -1 || mode > 1) return c->fail(AD_E_INVALID, "work queue: -1 (tune), 0 (off) or 1 (on)");
  c->forced_queue = mode;
  return AD_OK;
}

extern "C" int ad_get_work_queue(ad_ctx *c, int *used) {
  if (!c) return AD_E_INVALID;
  if (used)
    for (int bk = 0; bk < 2; ++bk) used[bk] = c->last_queue[bk];
  return AD_OK;
}

extern "C" int ad_set_chains(ad_ctx *c, int parts) {
  if (!c) return AD_E_INVALID;
  if (parts < 1 || parts > ad_ctx::kMaxChainsPerBucket) return c->fail(AD_E_INVALID, "chains: parts 1..4 per bucket");
  c->chains = parts;
  return AD_OK;
}

extern "C" int ad_get_chains(ad_ctx *c, int *parts) {
  if (!c) return AD_E_INVALID;
  if (parts)
    for (int bk = 0; bk < 2; ++bk) parts[bk] = c->last_chains[bk];
  return AD_OK;
}

extern "C" int ad_get_schedule(ad_ctx *c, int *stage_pairs, int *graph_used, int *packed_runs) {
  if (!c) return AD_E_INVALID;
  if (packed_runs) *packed_runs = c->last_packed;
  if (stage_pairs) {
    stage_pairs[0] = c->last_stage[0];
    stage_pairs[1] = c->last_stage[1];
  }
  if (graph_used) *graph_used = c->last_graph;
  return AD_OK;
}

extern "C" int ad_initial_population(ad_ctx *c, const ad_batch *b, int lig, uint32_t lig_id, int run, int pop,
                                     uint64_t seed, float *genotypes) {
  if (!c) return AD_E_INVALID;
  if (!b || b->ctx != c) return c->fail(AD_E_INVALID, "bad batch");
  if (!c->has_grid) return c->fail(AD_E_STATE, "no grid loaded");
  if (lig < 0 || lig >= b->n_lig || run < 0 || pop < 1 || pop > AD_MAX_POP || !genotypes)
    return c->fail(AD_E_INVALID, "bad arguments");
  hipSetDevice(c->device);
  float *d = (float *)c->scratch_alloc((size_t)pop * kStride * sizeof(float), 2);
  if (!d) return c->fail(AD_E_OOM, "cannot allocate");
  const EvalConst C = c->eval_const(b);
  HIP_TRY(c, launch_init_genotypes(C.grid, b->lig_host[lig].n_tor, (uint32_t)seed, (uint32_t)(seed >> 32), lig_id,
                                   run, pop, d, c->stream));
  HIP_TRY(c, hipMemcpyAsync(genotypes, d, (size_t)pop * kStride * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return AD_OK;
}
