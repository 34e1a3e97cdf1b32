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
  if (p->ls_method != 0) return c->fail(AD_E_UNSUPPORTED, "only ADADELTA local search (ls_method 0) is built");
  if (p->autostop != 0) return c->fail(AD_E_UNSUPPORTED, "autostop is not built");
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

}  // namespace

extern "C" int ad_dock_batch(ad_ctx *c, const ad_batch *b, const ad_dock_params *p, uint64_t seed,
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
  if (!out) return c->fail(AD_E_INVALID, "null result array");
  const int n_lig = b->n_lig;
  if (n_lig == 0) return AD_OK;
  if ((int64_t)n_lig * p->nrun * p->pop > (int64_t)1 << 31)
    return c->fail(AD_E_INVALID, "n_lig * nrun * pop too large for one batch");
  const int n_runs = n_lig * p->nrun;
  const int n_ls = n_local_search(p);
  const int G = generations(p, n_ls);

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
  const size_t total = sz_geno + sz_E + sz_ev + sz_ord + sz_id + sz_bE + sz_bG + sz_lG + sz_lE + sz_lT + sz_li;
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
  D.run_order = d_order;
  D.lig_id = d_id;
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

  // runs of expensive ligands first, so the last work-groups of each launch
  // are the cheap ones (longest-processing-time order)
  std::vector<int> order(n_runs);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(n_lig);
  for (int l = 0; l < n_lig; ++l)
    cost[l] = b->lig_host[l].n_pairs + 4.0 * b->lig_host[l].n_atoms + 2.0 * b->lig_host[l].n_tor;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return cost[x / p->nrun] > cost[y / p->nrun]; });
  std::vector<uint32_t> ids(n_lig);
  for (int l = 0; l < n_lig; ++l) ids[l] = lig_ids ? lig_ids[l] : (uint32_t)l;
  HIP_TRY(c, hipMemcpyAsync(d_order, order.data(), n_runs * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_id, ids.data(), n_lig * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(D.evals, 0, (size_t)n_runs * sizeof(unsigned long long), c->stream));

  const EvalConst C = c->eval_const(b);
  {
    const int t0 = c->timing_begin(0);
    HIP_TRY(c, launch_dock_init(C, b->cap, D, c->stream));
    c->timing_end(0, t0);
  }
  for (int gen = 1; gen <= G; ++gen) {
    const int t1 = c->timing_begin(1);
    HIP_TRY(c, launch_ga_generation(C, b->cap, D, gen, c->stream));
    c->timing_end(1, t1);
    if (n_ls > 0 && p->ls_iters > 0) {
      const int t2 = c->timing_begin(2);
      HIP_TRY(c, launch_ls_generation(C, b->cap, D, gen, c->stream));
      c->timing_end(2, t2);
    }
  }
  HIP_TRY(c, launch_dock_finalize(D, G & 1, d_bE, d_bG, c->stream));

  std::vector<float> bE(n_runs), bG((size_t)n_runs * kStride);
  std::vector<unsigned long long> ev(n_runs);
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
    lidx[l] = l;
    memcpy(&lG[(size_t)l * kStride], &bG[(size_t)(l * p->nrun + br) * kStride], kStride * sizeof(float));
  }
  HIP_TRY(c, hipMemcpyAsync(d_lG, lG.data(), lG.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_li, lidx.data(), n_lig * sizeof(int), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_score(C, b->cap, n_lig, d_li, d_lG, d_lE, nullptr, d_lT, c->stream));
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
    r.generations = G;
    int64_t e = 0;
    for (int q = 0; q < p->nrun; ++q) e += (int64_t)ev[l * p->nrun + q];
    r.evals = e;
  }
  if (run_energy) memcpy(run_energy, bE.data(), n_runs * sizeof(float));
  if (run_genotype) memcpy(run_genotype, bG.data(), (size_t)n_runs * kStride * sizeof(float));
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
