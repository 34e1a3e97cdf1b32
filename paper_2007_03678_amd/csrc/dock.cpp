// Docking entry points (Lamarckian GA + ADADELTA).
#include "api_internal.h"

extern "C" int ad_dock_batch(ad_ctx *c, const ad_batch *b, const ad_dock_params *p, uint64_t seed,
                             const uint32_t *lig_ids, ad_dock_result *out, float *run_energy, float *run_genotype) {
  if (!c) return AD_E_INVALID;
  return c->fail(AD_E_UNSUPPORTED, "docking not built yet");
}

extern "C" int ad_initial_population(ad_ctx *c, const ad_batch *b, int lig, uint32_t lig_id, int run, int pop,
                                     uint64_t seed, float *genotypes) {
  if (!c) return AD_E_INVALID;
  return c->fail(AD_E_UNSUPPORTED, "docking not built yet");
}
