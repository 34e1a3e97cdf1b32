// C-ABI entry points of libaddock: argument validation, device memory,
// host<->device staging and kernel launches on the context's stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <thread>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace ad;

static_assert(kNoAllocPoses == AD_NOALLOC_MAX_POSES, "static staging limit matches the header");

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
int ad_ctx::fail(int code, const std::string &msg) {
  err = msg;
  return code;
}

int ad_ctx::hip_fail(hipError_t e, const char *where) {
  err = std::string(where) + ": " + hipGetErrorString(e);
  return AD_E_HIP;
}

#define HIP_TRY(ctx, expr)                                  \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return (ctx)->hip_fail(_e, #expr); \
  } while (0)

// fn(i) for i in [0, n) on up to 16 host threads (contiguous blocks)
template <typename F>
void parallel_for(int n, F fn) {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({hw, 16, std::max(1, n / 64)});
  if (nt <= 1) {
    for (int i = 0; i < n; ++i) fn(i);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      const int lo = (int)((long long)n * t / nt), hi = (int)((long long)n * (t + 1) / nt);
      for (int i = lo; i < hi; ++i) fn(i);
    });
  for (auto &x : th) x.join();
}

void *ad_ctx::scratch_alloc(size_t bytes, int slot) {
  // per-slot grow-only device buffers; calls on one context are serialised
  if (slot < 0 || slot >= kScratchSlots) return nullptr;
  bytes = (bytes + 255) & ~(size_t)255;
  if (scratch_bytes[slot] >= bytes && scratch[slot]) return scratch[slot];
  if (scratch[slot]) {
    hipStreamSynchronize(stream);
    hipFree(scratch[slot]);
    scratch[slot] = nullptr;
    scratch_bytes[slot] = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, std::max(bytes, (size_t)256)) != hipSuccess) return nullptr;
  scratch[slot] = p;
  scratch_bytes[slot] = bytes;
  return p;
}

EvalConst ad_ctx::eval_const(const ad_batch *b) const {
  EvalConst C;
  C.ff = ffc;
  C.grid.maps = maps4;
  C.grid.nx = grid_n[0];
  C.grid.ny = grid_n[1];
  C.grid.nz = grid_n[2];
  C.grid.n_maps = n_maps;
  C.grid.ox = origin[0];
  C.grid.oy = origin[1];
  C.grid.oz = origin[2];
  C.grid.h = spacing;
  C.grid.inv_h = 1.0 / spacing;
  C.batch.lig = b->lig;
  C.batch.geo = b->geo;
  C.batch.info = b->info;
  C.batch.pairs = b->pairs;
  C.batch.tors = b->tors;
  C.batch.lj = lj_dev;
  C.batch.trig = trig_dev;
  C.batch.n_lig = b->n_lig;
  C.batch.n_types = ff.n_types;
  return C;
}

static bool finite_d(double v) { return std::isfinite(v); }

static int check_ff(const ad_forcefield *ff, std::string *msg) {
  if (!ff) return *msg = "null force field", AD_E_INVALID;
  if (ff->n_types < 1 || ff->n_types > AD_MAX_TYPES) return *msg = "n_types must be 1..16", AD_E_INVALID;
  for (int t = 0; t < ff->n_types; ++t) {
    if (!(ff->Rii[t] > 0) || !(ff->epsii[t] >= 0) || !finite_d(ff->vol[t]) || !finite_d(ff->solpar[t]) ||
        ff->hbrole[t] < 0 || ff->hbrole[t] > 2 || !finite_d(ff->Rii[t]) || !finite_d(ff->epsii[t]))
      return *msg = "bad per-type force-field value", AD_E_INVALID;
    if (ff->hbrole[t] == 2 && (!(ff->Rhb[t] > 0) || !(ff->epshb[t] >= 0) || !finite_d(ff->Rhb[t])))
      return *msg = "bad H-bond parameters", AD_E_INVALID;
  }
  const double s[] = {ff->w_vdw, ff->w_hb, ff->w_el, ff->w_sol, ff->w_tor, ff->coulomb, ff->diel_A, ff->diel_eps0,
                      ff->diel_lambda, ff->diel_k, ff->sigma, ff->qasp, ff->smooth, ff->cutoff, ff->cap,
                      ff->r_floor, ff->k_out};
  for (double v : s)
    if (!finite_d(v)) return *msg = "non-finite force-field scalar", AD_E_INVALID;
  if (!(ff->sigma > 0) || !(ff->smooth >= 0) || !(ff->r_floor > 0) || !(ff->cutoff > 0) || !(ff->k_out >= 0))
    return *msg = "bad force-field scalar", AD_E_INVALID;
  return AD_OK;
}

static int check_grid_desc(const ad_grid_desc *g, int n_types, std::string *msg) {
  if (!g) return *msg = "null grid descriptor", AD_E_INVALID;
  if (g->nx < 2 || g->ny < 2 || g->nz < 2) return *msg = "grid needs >= 2 points per axis", AD_E_INVALID;
  if ((double)g->nx * g->ny * g->nz > 2.0e9) return *msg = "grid too large", AD_E_INVALID;
  // the kernels index the map records in 32 bits with 24-bit products:
  // (m * nz + k) * (nx * ny) + j * nx + i, both factors below 2^24
  if ((double)g->nx * g->ny >= 16777216.0 || (double)std::max(g->n_maps, 1) * g->nz >= 16777216.0 ||
      (double)std::max(g->n_maps, 1) * g->nx * g->ny * g->nz >= 4294967296.0)
    return *msg = "grid too large for the map indexing (nx*ny < 2^24, n_maps*nz < 2^24, n_maps*nx*ny*nz < 2^32)",
           AD_E_INVALID;
  if (!(g->spacing > 0) || !finite_d(g->spacing)) return *msg = "spacing must be > 0", AD_E_INVALID;
  for (int d = 0; d < 3; ++d)
    if (!finite_d(g->origin[d])) return *msg = "non-finite origin", AD_E_INVALID;
  if (g->n_maps < 0 || g->n_maps > AD_MAX_TYPES) return *msg = "n_maps must be 0..16", AD_E_INVALID;
  if (g->n_maps > 0 && !g->map_types) return *msg = "null map_types", AD_E_INVALID;
  for (int m = 0; m < g->n_maps; ++m) {
    if (g->map_types[m] < 0 || g->map_types[m] >= n_types) return *msg = "map type out of range", AD_E_INVALID;
    for (int k = 0; k < m; ++k)
      if (g->map_types[k] == g->map_types[m]) return *msg = "duplicate map type", AD_E_INVALID;
  }
  return AD_OK;
}

extern "C" int ad_grid_check(const ad_grid_desc *g, int n_types, char *msg, int msg_len) {
  std::string err;
  int rc = AD_OK;
  if (n_types < 1 || n_types > AD_MAX_TYPES) {
    rc = AD_E_INVALID;
    err = "n_types must be 1..16";
  } else {
    rc = check_grid_desc(g, n_types, &err);
  }
  if (msg && msg_len > 0) {
    strncpy(msg, rc ? err.c_str() : "", (size_t)msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return rc;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int ad_create(ad_ctx **out, int device, const ad_forcefield *ff, void *hip_stream) {
  if (!out) return AD_E_INVALID;
  *out = nullptr;
  std::string msg;
  int rc = check_ff(ff, &msg);
  if (rc) return rc;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return AD_E_DEVICE;
  if (device < 0 || device >= count) return AD_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return AD_E_DEVICE;
  // device address of ad_score_poses_noalloc's static block, once per device
  if (noalloc_scratch_init(device) != hipSuccess) return AD_E_HIP;
  ad_ctx *c = new ad_ctx();
  c->device = device;
  c->ff = *ff;
  c->ffc = make_ffconst(*ff);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return AD_E_HIP;
    }
    c->own_stream = true;
  }
  build_lj_table(*ff, &c->lj_host);
  if (hipMalloc(&c->lj_dev, c->lj_host.size() * sizeof(LJRec)) != hipSuccess ||
      hipMemcpy(c->lj_dev, c->lj_host.data(), c->lj_host.size() * sizeof(LJRec), hipMemcpyHostToDevice) !=
          hipSuccess) {
    ad_destroy(c);
    return AD_E_OOM;
  }
  {
    double trig[kTrigN][2];
    for (int j = 0; j < kTrigN; ++j) {
      const double a = j * (3.14159265358979323846 / (kTrigN / 2));
      trig[j][0] = std::sin(a);
      trig[j][1] = std::cos(a);
    }
    if (hipMalloc(&c->trig_dev, sizeof(trig)) != hipSuccess ||
        hipMemcpy(c->trig_dev, trig, sizeof(trig), hipMemcpyHostToDevice) != hipSuccess) {
      ad_destroy(c);
      return AD_E_OOM;
    }
  }
  for (int t = 0; t < AD_MAX_TYPES; ++t) c->type_to_map[t] = -1;
  *out = c;
  return AD_OK;
}

extern "C" void ad_destroy(ad_ctx *c) {
  if (!c) return;
  hipSetDevice(c->device);
  if (c->stream) hipStreamSynchronize(c->stream);
  {
    // children still alive give up their device memory and their link to
    // the context; freeing them later only deletes the handle
    std::lock_guard<std::mutex> lk(c->child_mu);
    for (ad_batch *b : c->batches) {
      batch_release(b);
      b->ctx = nullptr;
    }
    for (ad_prescreen *ps : c->prescreens) prescreen_release(ps);
    c->batches.clear();
    c->prescreens.clear();
  }
  for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
  if (c->maps4) hipFree(c->maps4);
  if (c->lj_dev) hipFree(c->lj_dev);
  if (c->trig_dev) hipFree(c->trig_dev);
  for (int s = 0; s < ad_ctx::kScratchSlots; ++s)
    if (c->scratch[s]) hipFree(c->scratch[s]);
  c->free_dock_buffers();
  if (c->own_stream && c->stream) hipStreamDestroy(c->stream);
  for (int i = 0; i < ad_ctx::kAuxStreams; ++i)
    if (c->aux_streams[i]) hipStreamDestroy(c->aux_streams[i]);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  delete c;
}

extern "C" const char *ad_last_error(const ad_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" int ad_set_stream(ad_ctx *c, void *hip_stream) {
  if (!c) return AD_E_INVALID;
  hipSetDevice(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->own_stream) hipStreamDestroy(c->stream);
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
    c->own_stream = false;
  } else {
    HIP_TRY(c, hipStreamCreate(&c->stream));
    c->own_stream = true;
  }
  return AD_OK;
}

extern "C" int ad_synchronize(ad_ctx *c) {
  if (!c) return AD_E_INVALID;
  hipSetDevice(c->device);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return AD_OK;
}

// ---------------------------------------------------------------------------
// grids
// ---------------------------------------------------------------------------
static int set_grid_meta(ad_ctx *c, const ad_grid_desc *g) {
  c->grid_n[0] = g->nx;
  c->grid_n[1] = g->ny;
  c->grid_n[2] = g->nz;
  c->spacing = g->spacing;
  for (int d = 0; d < 3; ++d) c->origin[d] = g->origin[d];
  c->n_maps = g->n_maps;
  for (int t = 0; t < AD_MAX_TYPES; ++t) c->type_to_map[t] = -1;
  for (int m = 0; m < g->n_maps; ++m) {
    c->map_types[m] = g->map_types[m];
    c->type_to_map[g->map_types[m]] = m;
  }
  return AD_OK;
}

static int ensure_maps4(ad_ctx *c, size_t nn, int n_maps) {
  size_t bytes = std::max((size_t)16, nn * (size_t)std::max(n_maps, 1) * 16);
  if (c->maps4 && c->maps4_bytes >= bytes) return AD_OK;
  if (c->maps4) {
    hipStreamSynchronize(c->stream);
    hipFree(c->maps4);
    c->maps4 = nullptr;
    c->maps4_bytes = 0;
  }
  if (hipMalloc(&c->maps4, bytes) != hipSuccess) return c->fail(AD_E_OOM, "cannot allocate grid maps");
  c->maps4_bytes = bytes;
  return AD_OK;
}

extern "C" int ad_load_grids(ad_ctx *c, const ad_grid_desc *g, const float *maps, int ptrs_on_device) {
  if (!c) return AD_E_INVALID;
  std::string msg;
  int rc = check_grid_desc(g, c->ff.n_types, &msg);
  if (rc) return c->fail(rc, msg);
  if (!maps) return c->fail(AD_E_INVALID, "null maps");
  hipSetDevice(c->device);
  const size_t nn = (size_t)g->nx * g->ny * g->nz;
  const size_t total = nn * (size_t)(g->n_maps + 2);
  if (!ptrs_on_device) {
    for (size_t i = 0; i < total; ++i)
      if (!std::isfinite(maps[i])) return c->fail(AD_E_INVALID, "non-finite map value");
  }
  rc = ensure_maps4(c, nn, g->n_maps);
  if (rc) return rc;
  const float *src = maps;
  if (!ptrs_on_device) {
    float *tmp = (float *)c->scratch_alloc(total * sizeof(float), 0);
    if (!tmp) return c->fail(AD_E_OOM, "cannot allocate staging buffer");
    HIP_TRY(c, hipMemcpyAsync(tmp, maps, total * sizeof(float), hipMemcpyHostToDevice, c->stream));
    src = tmp;
  }
  if (g->n_maps > 0) HIP_TRY(c, launch_relayout(src, c->maps4, nn, g->n_maps, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  set_grid_meta(c, g);
  c->has_grid = true;
  return AD_OK;
}

extern "C" int ad_build_grids(ad_ctx *c, const ad_grid_desc *g, int n_rec, const float *rec_xyz, const int *rec_type,
                              const float *rec_charge, float *maps_out) {
  if (!c) return AD_E_INVALID;
  std::string msg;
  int rc = check_grid_desc(g, c->ff.n_types, &msg);
  if (rc) return c->fail(rc, msg);
  if (n_rec < 0 || (n_rec > 0 && (!rec_xyz || !rec_type || !rec_charge)))
    return c->fail(AD_E_INVALID, "bad receptor arrays");
  for (int a = 0; a < n_rec; ++a) {
    if (rec_type[a] < 0 || rec_type[a] >= c->ff.n_types) return c->fail(AD_E_INVALID, "receptor type out of range");
    if (!std::isfinite(rec_charge[a]) || !std::isfinite(rec_xyz[3 * a]) || !std::isfinite(rec_xyz[3 * a + 1]) ||
        !std::isfinite(rec_xyz[3 * a + 2]))
      return c->fail(AD_E_INVALID, "non-finite receptor data");
  }
  hipSetDevice(c->device);
  const size_t nn = (size_t)g->nx * g->ny * g->nz;
  rc = ensure_maps4(c, nn, g->n_maps);
  if (rc) return rc;
  // receptor staging: xyz, type, charge in one scratch block
  size_t o_xyz = 0, o_t = ((size_t)3 * n_rec * 4 + 255) & ~(size_t)255;
  size_t o_q = o_t + (((size_t)n_rec * 4 + 255) & ~(size_t)255);
  size_t o_args = o_q + (((size_t)n_rec * 4 + 255) & ~(size_t)255);
  size_t bytes = o_args + ((map_build_args_size() + 255) & ~(size_t)255);
  char *blk = (char *)c->scratch_alloc(bytes, 1);
  if (!blk) return c->fail(AD_E_OOM, "cannot allocate receptor staging");
  float *soa = nullptr;
  if (maps_out) {
    soa = (float *)c->scratch_alloc(nn * (size_t)(g->n_maps + 2) * sizeof(float), 0);
    if (!soa) return c->fail(AD_E_OOM, "cannot allocate map output staging");
  }
  std::vector<char> hargs(map_build_args_size());
  fill_map_build_args(hargs.data(), c->ff, g, n_rec, (const float *)(blk + o_xyz), (const int *)(blk + o_t),
                      (const float *)(blk + o_q), c->maps4, soa);
  if (n_rec > 0) {
    HIP_TRY(c, hipMemcpyAsync(blk + o_xyz, rec_xyz, (size_t)3 * n_rec * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(blk + o_t, rec_type, (size_t)n_rec * 4, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(blk + o_q, rec_charge, (size_t)n_rec * 4, hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(blk + o_args, hargs.data(), hargs.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_build_maps(reinterpret_cast<const MapBuildArgs *>(blk + o_args), nn, c->stream));
  if (maps_out)
    HIP_TRY(c, hipMemcpyAsync(maps_out, soa, nn * (size_t)(g->n_maps + 2) * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  set_grid_meta(c, g);
  c->has_grid = true;
  return AD_OK;
}

// ---------------------------------------------------------------------------
// ligands
// ---------------------------------------------------------------------------
extern "C" int ad_ligand_check(const ad_ligand *lig, int n_types, char *msg, int msg_len) {
  std::string err;
  int rc;
  if (!lig) {
    rc = AD_E_INVALID;
    err = "null ligand";
  } else if (n_types < 1 || n_types > AD_MAX_TYPES) {
    rc = AD_E_INVALID;
    err = "n_types must be 1..16";
  } else {
    ad_forcefield ff;
    memset(&ff, 0, sizeof(ff));
    ff.n_types = n_types;
    rc = prepare_ligand(*lig, ff, nullptr, nullptr, &err);
  }
  if (msg && msg_len > 0) {
    strncpy(msg, rc ? err.c_str() : "", (size_t)msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return rc;
}

// The work of ad_load_ligands without touching the context's error state
// (ad_dock_stream runs it on a worker thread while the context docks).
int load_ligands_impl(ad_ctx *c, int n, const ad_ligand *ligs, uint64_t uid, ad_batch **out, std::string *err) {
  *out = nullptr;
  // host preparation (validation, torsion tree, pair list, features) runs on
  // all host threads; the first failing ligand (lowest index) is reported
  std::vector<PreparedLigand> prep(n);
  std::vector<int> prep_rc(n, AD_OK);
  std::vector<std::string> prep_err(n);
  parallel_for(n, [&](int i) { prep_rc[i] = prepare_ligand(ligs[i], c->ff, c->type_to_map, &prep[i], &prep_err[i]); });
  for (int i = 0; i < n; ++i)
    if (prep_rc[i]) {
      *err = "ligand " + std::to_string(i) + ": " + prep_err[i];
      return prep_rc[i];
    }
  ad_batch *b = new ad_batch();
  b->ctx = c;
  b->uid = uid;
  b->device = c->device;
  b->n_lig = n;
  std::vector<LigDesc> lig(n);
  std::vector<AtomGeo> geo;
  std::vector<AtomInfo> info;
  std::vector<PairRec> pairs;
  std::vector<TorRec> tors;
  int cap = 64;
  for (int i = 0; i < n; ++i) {
    const PreparedLigand &P = prep[i];
    LigDesc &d = lig[i];
    d.n_atoms = P.n_atoms;
    d.n_tor = P.n_tor;
    d.n_pairs = (int)P.pairs.size();
    d.n_frag = P.n_frag;
    d.atom_off = (int)geo.size();
    d.pair_off = (int)pairs.size();
    d.tor_off = (int)tors.size();
    d.max_depth = P.max_depth;
    geo.insert(geo.end(), P.geo.begin(), P.geo.end());
    info.insert(info.end(), P.info.begin(), P.info.end());
    pairs.insert(pairs.end(), P.pairs.begin(), P.pairs.end());
    tors.insert(tors.end(), P.tors.begin(), P.tors.end());
    if (P.n_atoms > 64) cap = 128;
  }
  pairs.resize(pairs.size() + 2 * kWave, PairRec{0, 0.0f, 0.0f, 0.0f});   // spare records: the kernels prefetch 128 ahead
  b->cap = cap;
  b->lig_host = lig;
  b->depth_sum.resize(n);
  for (int i = 0; i < n; ++i) b->depth_sum[i] = prep[i].depth_sum;
  for (int t = 0; t < AD_MAX_TYPES; ++t) b->map_of_type[t] = -1;
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < ligs[i].n_atoms; ++a) b->map_of_type[ligs[i].type_id[a]] = c->type_to_map[ligs[i].type_id[a]];
  hipSetDevice(c->device);
  auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
    if (hipMalloc(dst, std::max(bytes, (size_t)256)) != hipSuccess) return false;
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
    return true;
  };
  std::vector<std::vector<uint16_t>> fx(n);
  std::vector<std::vector<uint8_t>> fn(n);
  std::vector<char> f_ok(n, 1);
  parallel_for(n, [&](int i) {
    if (!featurize(ligs[i], prep[i].perm, &fx[i], &fn[i])) {
      f_ok[i] = 0;
      fx[i].assign((size_t)prep[i].n_atoms * kFeat, 0);
      fn[i].assign((size_t)prep[i].n_atoms * kMaxDeg, 0xff);
    }
  });
  std::vector<uint16_t> psx;
  std::vector<uint8_t> psn;
  psx.reserve(geo.size() * kFeat);
  psn.reserve(geo.size() * kMaxDeg);
  for (int i = 0; i < n; ++i) {
    if (!f_ok[i]) b->ps_ok = false;
    psx.insert(psx.end(), fx[i].begin(), fx[i].end());
    psn.insert(psn.end(), fn[i].begin(), fn[i].end());
  }
  b->n_atoms_total = (int)geo.size();
  bool ok = up((void **)&b->ps_x, psx.data(), psx.size() * sizeof(uint16_t)) &&
            up((void **)&b->ps_nbr, psn.data(), psn.size()) &&
            up((void **)&b->lig, lig.data(), lig.size() * sizeof(LigDesc)) &&
            up((void **)&b->geo, geo.data(), geo.size() * sizeof(AtomGeo)) &&
            up((void **)&b->info, info.data(), info.size() * sizeof(AtomInfo)) &&
            up((void **)&b->pairs, pairs.data(), pairs.size() * sizeof(PairRec)) &&
            up((void **)&b->tors, tors.data(), tors.size() * sizeof(TorRec));
  if (!ok) {
    ad_free_batch(b);
    *err = "cannot upload ligand batch";
    return AD_E_OOM;
  }
  register_batch(c, b);
  *out = b;
  return AD_OK;
}

extern "C" int ad_load_ligands(ad_ctx *c, int n, const ad_ligand *ligs, ad_batch **out) {
  if (!c || !out) return AD_E_INVALID;
  *out = nullptr;
  if (n < 0 || (n > 0 && !ligs)) return c->fail(AD_E_INVALID, "bad ligand array");
  if (!c->has_grid) return c->fail(AD_E_STATE, "load or build grids before ligands");
  std::string err;
  const int rc = load_ligands_impl(c, n, ligs, c->next_batch_uid++, out, &err);
  return rc ? c->fail(rc, err) : AD_OK;
}

// Views of n ligands stored back to back (the ad_load_ligands_packed layout).
int packed_views(int n, const int *n_atoms, const int *n_bonds, const int *type_id, const float *charge,
                 const float *xyz, const int *bonds, const unsigned char *rotatable, std::vector<ad_ligand> *out,
                 std::string *err) {
  if (n < 0 || (n > 0 && (!n_atoms || !n_bonds || !type_id || !charge || !xyz))) {
    *err = "bad packed ligand arrays";
    return AD_E_INVALID;
  }
  std::vector<ad_ligand> &v = *out;
  v.assign(n, ad_ligand{});
  size_t a = 0, bo = 0;
  for (int i = 0; i < n; ++i) {
    if (n_atoms[i] < 1 || n_bonds[i] < 0) {
      *err = "ligand " + std::to_string(i) + ": bad counts";
      return AD_E_INVALID;
    }
    if (n_bonds[i] > 0 && (!bonds || !rotatable)) {
      *err = "null bond arrays";
      return AD_E_INVALID;
    }
    v[i].n_atoms = n_atoms[i];
    v[i].n_bonds = n_bonds[i];
    v[i].type_id = type_id + a;
    v[i].charge = charge + a;
    v[i].xyz = xyz + 3 * a;
    v[i].bonds = n_bonds[i] ? bonds + 2 * bo : nullptr;
    v[i].rotatable = n_bonds[i] ? rotatable + bo : nullptr;
    a += (size_t)n_atoms[i];
    bo += (size_t)n_bonds[i];
  }
  return AD_OK;
}

extern "C" int ad_load_ligands_packed(ad_ctx *c, int n, const int *n_atoms, const int *n_bonds, const int *type_id,
                                      const float *charge, const float *xyz, const int *bonds,
                                      const unsigned char *rotatable, ad_batch **out) {
  if (!c || !out) return AD_E_INVALID;
  *out = nullptr;
  std::vector<ad_ligand> v;
  std::string err;
  const int rc = packed_views(n, n_atoms, n_bonds, type_id, charge, xyz, bonds, rotatable, &v, &err);
  if (rc) return c->fail(rc, err);
  return ad_load_ligands(c, n, v.data(), out);
}

void register_batch(ad_ctx *c, ad_batch *b) {
  std::lock_guard<std::mutex> lk(c->child_mu);
  c->batches.insert(b);
}

void unregister_batch(ad_ctx *c, ad_batch *b) {
  std::lock_guard<std::mutex> lk(c->child_mu);
  c->batches.erase(b);
}

// Frees the batch's device memory (the host descriptors stay readable).
void batch_release(ad_batch *b) {
  hipSetDevice(b->device);
  if (b->ctx && b->ctx->stream) hipStreamSynchronize(b->ctx->stream);
  void *bufs[] = {b->lig, b->geo, b->info, b->pairs, b->tors, b->ps_x, b->ps_nbr};
  for (void *p : bufs)
    if (p) hipFree(p);
  b->lig = nullptr;
  b->geo = nullptr;
  b->info = nullptr;
  b->pairs = nullptr;
  b->tors = nullptr;
  b->ps_x = nullptr;
  b->ps_nbr = nullptr;
}

extern "C" void ad_free_batch(ad_batch *b) {
  if (!b) return;
  // a batch detached by ad_destroy has no device memory left
  if (b->ctx) {
    unregister_batch(b->ctx, b);
    batch_release(b);
  }
  delete b;
}

extern "C" int ad_batch_info(const ad_batch *b, int lig, int *n_atoms, int *n_torsions, int *n_pairs,
                             int *n_fragments, int *depth_sum) {
  if (!b || lig < 0 || lig >= b->n_lig) return AD_E_INVALID;
  const LigDesc &d = b->lig_host[lig];
  if (n_atoms) *n_atoms = d.n_atoms;
  if (n_torsions) *n_torsions = d.n_tor;
  if (n_pairs) *n_pairs = d.n_pairs;
  if (n_fragments) *n_fragments = d.n_frag;
  if (depth_sum) *depth_sum = b->depth_sum[lig];
  return AD_OK;
}

// ---------------------------------------------------------------------------
// scoring and local search
// ---------------------------------------------------------------------------
static int check_batch(ad_ctx *c, const ad_batch *b) {
  if (!b) return c->fail(AD_E_INVALID, "null batch");
  if (b->ctx != c) return c->fail(AD_E_INVALID, "batch belongs to another (or a destroyed) context");
  if (!c->has_grid) return c->fail(AD_E_STATE, "no grid loaded");
  // the batch's atoms carry map indices: the resident grid must still assign them
  for (int t = 0; t < AD_MAX_TYPES; ++t)
    if (b->map_of_type[t] >= 0 && c->type_to_map[t] != b->map_of_type[t])
      return c->fail(AD_E_STATE, "grid maps changed since the batch was loaded; reload the ligands");
  return AD_OK;
}

// Kernel atom capacity of an evaluation shape (32: the packed kernels), or
// -1 for an unknown shape.
static int shape_cap(const ad_batch *b, int shape) {
  switch (shape) {
    case AD_SHAPE_AUTO: return b->cap;
    case AD_SHAPE_WAVE64: return 64;
    case AD_SHAPE_WAVE128: return 128;
    case AD_SHAPE_PACKED: return 32;
    default: return -1;
  }
}

// Host-side check of the ligands a shaped call names (host index arrays).
static int check_shape_poses(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, int shape) {
  for (int p = 0; p < n; ++p)
    if (lig_idx[p] < 0 || lig_idx[p] >= b->n_lig) return c->fail(AD_E_INVALID, "lig_idx out of range");
  const int cap = shape_cap(b, shape);
  for (int p = 0; p < n; ++p) {
    const LigDesc &d = b->lig_host[lig_idx[p]];
    if (d.n_atoms > std::max(cap, kDualAtoms) || (cap == kDualAtoms && d.n_tor > kDualTor))
      return c->fail(AD_E_INVALID, "pose " + std::to_string(p) + ": ligand too large for the evaluation shape");
    if (shape == AD_SHAPE_PACKED && (p & 1) && lig_idx[p] != lig_idx[p - 1])
      return c->fail(AD_E_INVALID, "packed shape: poses 2w and 2w+1 must name the same ligand");
  }
  return AD_OK;
}

extern "C" int ad_score_poses(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, const float *genotypes,
                              float *energy, float *grad, float *terms, int ptrs_on_device) {
  return ad_score_poses_shape(c, b, n, lig_idx, genotypes, energy, grad, terms, ptrs_on_device, AD_SHAPE_AUTO);
}

extern "C" int ad_score_poses_shape(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, const float *genotypes,
                                    float *energy, float *grad, float *terms, int ptrs_on_device, int shape) {
  if (!c) return AD_E_INVALID;
  int rc = check_batch(c, b);
  if (rc) return rc;
  if (n < 0) return c->fail(AD_E_INVALID, "n < 0");
  const int cap = shape_cap(b, shape);
  if (cap < 0) return c->fail(AD_E_INVALID, "unknown evaluation shape");
  if (n == 0) return AD_OK;
  if (!lig_idx || !genotypes || !energy) return c->fail(AD_E_INVALID, "null argument");
  hipSetDevice(c->device);
  const EvalConst C = c->eval_const(b);
  if (ptrs_on_device) {
    const int t0 = c->timing_begin(3);
    HIP_TRY(c, launch_score(C, cap, n, lig_idx, genotypes, energy, grad, terms, c->stream));
    c->timing_end(3, t0);
    return AD_OK;
  }
  rc = check_shape_poses(c, b, n, lig_idx, shape);
  if (rc) return rc;
  const size_t nb_idx = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t nb_geo = ((size_t)n * kStride * 4 + 255) & ~(size_t)255;
  const size_t nb_e = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t nb_g = grad ? nb_geo : 0;
  const size_t nb_t = terms ? (((size_t)n * 12 + 255) & ~(size_t)255) : 0;
  char *blk = (char *)c->scratch_alloc(nb_idx + nb_geo + nb_e + nb_g + nb_t, 0);
  if (!blk) return c->fail(AD_E_OOM, "cannot allocate staging");
  int *d_idx = (int *)blk;
  float *d_geo = (float *)(blk + nb_idx);
  float *d_e = (float *)(blk + nb_idx + nb_geo);
  float *d_g = grad ? (float *)(blk + nb_idx + nb_geo + nb_e) : nullptr;
  float *d_t = terms ? (float *)(blk + nb_idx + nb_geo + nb_e + nb_g) : nullptr;
  HIP_TRY(c, hipMemcpyAsync(d_idx, lig_idx, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_geo, genotypes, (size_t)n * kStride * 4, hipMemcpyHostToDevice, c->stream));
  const int t0 = c->timing_begin(3);
  HIP_TRY(c, launch_score(C, cap, n, d_idx, d_geo, d_e, d_g, d_t, c->stream));
  c->timing_end(3, t0);
  HIP_TRY(c, hipMemcpyAsync(energy, d_e, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  if (grad) HIP_TRY(c, hipMemcpyAsync(grad, d_g, (size_t)n * kStride * 4, hipMemcpyDeviceToHost, c->stream));
  if (terms) HIP_TRY(c, hipMemcpyAsync(terms, d_t, (size_t)n * 12, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timing_collect();
  return AD_OK;
}

extern "C" int ad_score_poses_noalloc(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx,
                                      const float *genotypes, float *energy, float *grad, float *terms) {
  // ad_score_poses with host buffers, staged through the device's static
  // block instead of the context's grow-only staging buffer: no device
  // allocation, no event creation (kernel timing does not cover this call)
  if (!c) return AD_E_INVALID;
  int rc = check_batch(c, b);
  if (rc) return rc;
  if (n < 0) return c->fail(AD_E_INVALID, "n < 0");
  if (n > kNoAllocPoses)
    return c->fail(AD_E_INVALID, "ad_score_poses_noalloc: n = " + std::to_string(n) + " exceeds the static limit of " +
                                     std::to_string(kNoAllocPoses) + " poses per call");
  if (n == 0) return AD_OK;
  if (!lig_idx || !genotypes || !energy) return c->fail(AD_E_INVALID, "null argument");
  rc = check_shape_poses(c, b, n, lig_idx, AD_SHAPE_AUTO);
  if (rc) return rc;
  const int cap = shape_cap(b, AD_SHAPE_AUTO);
  HIP_TRY(c, hipSetDevice(c->device));
  char *blk = (char *)noalloc_scratch(c->device);
  if (!blk) return c->fail(AD_E_STATE, "static staging block not set up on this device");
  const EvalConst C = c->eval_const(b);
  int *d_idx = (int *)(blk + kNoAllocIdx);
  float *d_geo = (float *)(blk + kNoAllocGeno);
  float *d_e = (float *)(blk + kNoAllocE);
  float *d_g = grad ? (float *)(blk + kNoAllocG) : nullptr;
  float *d_t = terms ? (float *)(blk + kNoAllocT) : nullptr;
  // every staged section is written before it is read (inputs by the copies
  // below, outputs by the kernel for every pose), so nothing needs clearing
  HIP_TRY(c, hipMemcpyAsync(d_idx, lig_idx, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_geo, genotypes, (size_t)n * kStride * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_score(C, cap, n, d_idx, d_geo, d_e, d_g, d_t, c->stream));
  HIP_TRY(c, hipMemcpyAsync(energy, d_e, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  if (grad) HIP_TRY(c, hipMemcpyAsync(grad, d_g, (size_t)n * kStride * 4, hipMemcpyDeviceToHost, c->stream));
  if (terms) HIP_TRY(c, hipMemcpyAsync(terms, d_t, (size_t)n * 12, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return AD_OK;
}

extern "C" int ad_local_search(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, float *genotypes,
                               float *energy, const ad_dock_params *p, int iters, int ptrs_on_device) {
  return ad_local_search_shape(c, b, n, lig_idx, genotypes, energy, p, iters, ptrs_on_device, AD_SHAPE_AUTO);
}

extern "C" int ad_local_search_shape(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, float *genotypes,
                                     float *energy, const ad_dock_params *p, int iters, int ptrs_on_device,
                                     int shape) {
  if (!c) return AD_E_INVALID;
  int rc = check_batch(c, b);
  if (rc) return rc;
  if (n < 0 || iters < 0 || !p) return c->fail(AD_E_INVALID, "bad local-search arguments");
  if (!(p->rho >= 0 && p->rho < 1) || !(p->eps > 0)) return c->fail(AD_E_INVALID, "bad ADADELTA rho / eps");
  const int cap = shape_cap(b, shape);
  if (cap < 0) return c->fail(AD_E_INVALID, "unknown evaluation shape");
  if (n == 0) return AD_OK;
  if (!lig_idx || !genotypes || !energy) return c->fail(AD_E_INVALID, "null argument");
  hipSetDevice(c->device);
  const EvalConst C = c->eval_const(b);
  if (ptrs_on_device) {
    const int t0 = c->timing_begin(2);
    HIP_TRY(c, launch_local_search(C, cap, n, lig_idx, genotypes, energy, iters, p->rho, p->eps, c->stream));
    c->timing_end(2, t0);
    return AD_OK;
  }
  rc = check_shape_poses(c, b, n, lig_idx, shape);
  if (rc) return rc;
  const size_t nb_idx = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t nb_geo = ((size_t)n * kStride * 4 + 255) & ~(size_t)255;
  char *blk = (char *)c->scratch_alloc(nb_idx + nb_geo + nb_idx, 0);
  if (!blk) return c->fail(AD_E_OOM, "cannot allocate staging");
  int *d_idx = (int *)blk;
  float *d_geo = (float *)(blk + nb_idx);
  float *d_e = (float *)(blk + nb_idx + nb_geo);
  HIP_TRY(c, hipMemcpyAsync(d_idx, lig_idx, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_geo, genotypes, (size_t)n * kStride * 4, hipMemcpyHostToDevice, c->stream));
  const int t0 = c->timing_begin(2);
  HIP_TRY(c, launch_local_search(C, cap, n, d_idx, d_geo, d_e, iters, p->rho, p->eps, c->stream));
  c->timing_end(2, t0);
  HIP_TRY(c, hipMemcpyAsync(genotypes, d_geo, (size_t)n * kStride * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(energy, d_e, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timing_collect();
  return AD_OK;
}

extern "C" int ad_solis_wets(ad_ctx *c, const ad_batch *b, int n, const int *lig_idx, float *genotypes,
                             float *energy, int *evals_used, const ad_dock_params *p, int max_evals, uint64_t seed) {
  if (!c) return AD_E_INVALID;
  int rc = check_batch(c, b);
  if (rc) return rc;
  if (n < 0 || max_evals < 0 || !p) return c->fail(AD_E_INVALID, "bad local-search arguments");
  if (!(p->sw_rho > 0.0) || !(p->sw_rho_lb > 0.0) || p->sw_max_succ < 1 || p->sw_max_fail < 1 ||
      !(p->sw_sigma_t >= 0.0) || !(p->sw_sigma_ang >= 0.0))
    return c->fail(AD_E_INVALID, "bad Solis-Wets parameters");
  if (n > 65536) return c->fail(AD_E_INVALID, "at most 65536 poses per call");
  if (n == 0) return AD_OK;
  if (!lig_idx || !genotypes || !energy) return c->fail(AD_E_INVALID, "null argument");
  for (int q = 0; q < n; ++q)
    if (lig_idx[q] < 0 || lig_idx[q] >= b->n_lig) return c->fail(AD_E_INVALID, "lig_idx out of range");
  hipSetDevice(c->device);
  const EvalConst C = c->eval_const(b);
  DockArgs D;
  memset(&D, 0, sizeof(D));
  D.ls_iters = max_evals;
  D.k0 = (uint32_t)seed;
  D.k1 = (uint32_t)(seed >> 32);
  D.sw_rho = (float)p->sw_rho;
  D.sw_rho_lb = (float)p->sw_rho_lb;
  D.sw_sig_t = (float)p->sw_sigma_t;
  D.sw_sig_ang = (float)p->sw_sigma_ang;
  D.sw_max_succ = p->sw_max_succ;
  D.sw_max_fail = p->sw_max_fail;
  const size_t nb_idx = ((size_t)n * 4 + 255) & ~(size_t)255;
  const size_t nb_geo = ((size_t)n * kStride * 4 + 255) & ~(size_t)255;
  char *blk = (char *)c->scratch_alloc(3 * nb_idx + nb_geo, 0);
  if (!blk) return c->fail(AD_E_OOM, "cannot allocate staging");
  int *d_idx = (int *)blk;
  float *d_geo = (float *)(blk + nb_idx);
  float *d_e = (float *)(blk + nb_idx + nb_geo);
  int *d_used = (int *)(blk + 2 * nb_idx + nb_geo);
  HIP_TRY(c, hipMemcpyAsync(d_idx, lig_idx, (size_t)n * 4, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(d_geo, genotypes, (size_t)n * kStride * 4, hipMemcpyHostToDevice, c->stream));
  const int t0 = c->timing_begin(2);
  HIP_TRY(c, launch_solis_wets(C, b->cap, D, n, d_idx, d_geo, d_e, d_used, c->stream));
  c->timing_end(2, t0);
  HIP_TRY(c, hipMemcpyAsync(genotypes, d_geo, (size_t)n * kStride * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(energy, d_e, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  if (evals_used) HIP_TRY(c, hipMemcpyAsync(evals_used, d_used, (size_t)n * 4, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->timing_collect();
  return AD_OK;
}

// ---------------------------------------------------------------------------
// map-builder argument block (force field in double)
// ---------------------------------------------------------------------------
namespace ad {
size_t map_build_args_size() { return sizeof(MapBuildArgs); }

void fill_map_build_args(void *out, const ad_forcefield &ff, const ad_grid_desc *g, int n_rec, const float *xyz,
                         const int *type, const float *q, float *out4, float *soa) {
  MapBuildArgs &A = *reinterpret_cast<MapBuildArgs *>(out);
  memset(&A, 0, sizeof(A));
  A.rec_xyz = xyz;
  A.rec_type = type;
  A.rec_q = q;
  A.n_rec = n_rec;
  A.nx = g->nx;
  A.ny = g->ny;
  A.nz = g->nz;
  A.n_maps = g->n_maps;
  A.ox = g->origin[0];
  A.oy = g->origin[1];
  A.oz = g->origin[2];
  A.h = g->spacing;
  for (int m = 0; m < g->n_maps; ++m) A.map_type[m] = g->map_types[m];
  for (int i = 0; i < ff.n_types; ++i)
    for (int j = 0; j < ff.n_types; ++j) {
      int acc = -1;
      if (ff.hbrole[i] == 1 && ff.hbrole[j] == 2) acc = j;
      if (ff.hbrole[i] == 2 && ff.hbrole[j] == 1) acc = i;
      if (acc >= 0) {
        double R = ff.Rhb[acc], e = ff.epshb[acc], R10 = std::pow(R, 10.0);
        A.A[i][j] = ff.w_hb * 5.0 * e * R10 * R * R;
        A.B[i][j] = ff.w_hb * 6.0 * e * R10;
        A.r0[i][j] = R;
        A.hb[i][j] = 1;
      } else {
        double R = 0.5 * (ff.Rii[i] + ff.Rii[j]), e = std::sqrt(ff.epsii[i] * ff.epsii[j]);
        double R6 = std::pow(R, 6.0);
        A.A[i][j] = ff.w_vdw * e * R6 * R6;
        A.B[i][j] = ff.w_vdw * 2.0 * e * R6;
        A.r0[i][j] = R;
        A.hb[i][j] = 0;
      }
    }
  for (int t = 0; t < ff.n_types; ++t) {
    A.solpar[t] = ff.solpar[t];
    A.vol[t] = ff.vol[t];
  }
  A.w_el_ke = ff.w_el * ff.coulomb;
  A.w_sol = ff.w_sol;
  A.qasp = ff.qasp;
  A.diel_A = ff.diel_A;
  A.diel_B = ff.diel_eps0 - ff.diel_A;
  A.diel_k = ff.diel_k;
  A.diel_lB = ff.diel_lambda * A.diel_B;
  A.two_s2 = 2.0 * ff.sigma * ff.sigma;
  A.half_smooth = 0.5 * ff.smooth;
  A.cutoff2 = ff.cutoff * ff.cutoff;
  A.cap = ff.cap;
  A.r_floor = ff.r_floor;
  A.out4 = out4;
  A.soa = soa;
}
}  // namespace ad

// Docking entry points are implemented in dock.cpp.

// ---------------------------------------------------------------------------
// kernel timing
// ---------------------------------------------------------------------------
int ad_ctx::timing_begin(int kind, hipStream_t s) {
  if (!timing) return -1;
  while (ev_used + 3 > ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    ev_pool.push_back(e);
  }
  // pool slot 0 of a call: the reference event, on the context's stream
  // before anything the call launches
  if (ev_used == 0) {
    if (hipEventRecord(ev_pool[0], stream) != hipSuccess) return -1;
    ev_used = 1;
  }
  const int i = (int)ev_used;
  ev_used += 2;
  if (hipEventRecord(ev_pool[i], s ? s : stream) != hipSuccess) return -1;
  (void)kind;
  return i;
}

void ad_ctx::timing_end(int kind, int start, hipStream_t s) {
  if (start < 0) return;
  if (hipEventRecord(ev_pool[start + 1], s ? s : stream) != hipSuccess) return;
  ev_pending[kind].push_back({start, start + 1});
}

void ad_ctx::timing_collect() {
  if (ev_used == 0) return;
  hipStreamSynchronize(stream);   // launches on other streams are joined into it
  for (int k = 0; k < AD_KERNEL_KINDS; ++k) {
    std::vector<std::pair<float, float>> iv;
    for (auto &pr : ev_pending[k]) {
      float t0 = 0.f, t1 = 0.f;
      if (hipEventElapsedTime(&t0, ev_pool[0], ev_pool[pr.first]) == hipSuccess &&
          hipEventElapsedTime(&t1, ev_pool[0], ev_pool[pr.second]) == hipSuccess) {
        t_ms[k] += t1 - t0;
        t_launches[k] += 1;
        iv.push_back({t0, t1});
      }
    }
    ev_pending[k].clear();
    // busy time: the union of the intervals
    std::sort(iv.begin(), iv.end());
    double busy = 0.0, lo = 0.0, hi = -1.0;
    for (auto &x : iv) {
      if (x.first > hi) {
        if (hi > lo) busy += hi - lo;
        lo = x.first;
        hi = x.second;
      } else if (x.second > hi) {
        hi = x.second;
      }
    }
    if (hi > lo) busy += hi - lo;
    t_busy[k] += busy;
  }
  ev_used = 0;
}

extern "C" int ad_set_kernel_timing(ad_ctx *c, int enable) {
  if (!c) return AD_E_INVALID;
  hipSetDevice(c->device);
  c->timing_collect();
  c->timing = enable != 0;
  return AD_OK;
}

extern "C" int ad_get_kernel_timing(ad_ctx *c, ad_kernel_times *out, int reset) {
  if (!c || !out) return AD_E_INVALID;
  hipSetDevice(c->device);
  c->timing_collect();
  for (int k = 0; k < AD_KERNEL_KINDS; ++k) {
    out->ms[k] = c->t_ms[k];
    out->launches[k] = c->t_launches[k];
    out->busy_ms[k] = c->t_busy[k];
    if (reset) {
      c->t_ms[k] = 0;
      c->t_launches[k] = 0;
      c->t_busy[k] = 0;
    }
  }
  return AD_OK;
}
