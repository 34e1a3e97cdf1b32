// HIP kernels for gfx950: fused pose + energy + gradient evaluation, local
// search, GA generations, grid-map construction and grid re-layout.
//
// Execution model: one 64-lane wavefront (one work-group) per individual.
// Lanes map to atoms (atom i on lane i % 64, up to two per lane), to
// torsions (lane k < 32) and to intramolecular pairs (strided).  Posed
// coordinates and per-atom force accumulators live in LDS; pair records,
// torsion records and the grid maps are read through L1/L2.  The ADADELTA
// search of small ligands (at most 32 atoms, 25 torsions) packs two
// individuals per wavefront, one per 32-lane half (ls_dual).
//
// Precision: geometry (pose, distances, grid coordinates and trilinear
// weights), the energy accumulation and the gradient back-projection run in
// FP64 -- on CDNA the FP64 FMA rate equals the non-packed FP32 rate, and the
// energy of a clashing pose is steep enough that FP32 coordinates would move
// it by more than 1e-5 relative.  The pair potentials themselves
// (transcendental heavy) run in FP32 with the hardware rsq / rcp / exp2.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "api_internal.h"

namespace ad {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Wavefront scans with DPP lane moves (no LDS crossbar round trips): rows of
// 16 lanes by row_shr 1, 2, 4, 8, then row_bcast 15 / 31 across rows.  The
// summation order is fixed, so results are bitwise reproducible.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// row shift with bound_ctrl: lanes whose source lies outside the row read 0,
// so no zeroed destination is needed
template <int CTRL>
__device__ __forceinline__ double dpp_shr_f64(double v) {
  const int l = (int)__double2loint(v), h = (int)__double2hiint(v);
  const int lo = __builtin_amdgcn_update_dpp(l, l, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(h, h, CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_incl_scan(double v) {
  v += dpp_shr_f64<0x111>(v);    // row_shr:1
  v += dpp_shr_f64<0x112>(v);    // row_shr:2
  v += dpp_shr_f64<0x114>(v);    // row_shr:4
  v += dpp_shr_f64<0x118>(v);    // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// value of lane 63 (uniform)
__device__ __forceinline__ double wave_last(double v) {
  const int lo = __builtin_amdgcn_readlane((int)__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane((int)__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) { return wave_last(wave_incl_scan(v)); }

// The same over groups of W lanes: W = 64 is the whole wavefront; W = 32
// splits it into two halves (lanes 0-31 and 32-63) that scan and sum
// independently (`half` = lane >> 5).
template <int W>
__device__ __forceinline__ double grp_incl_scan(double v) {
  v += dpp_shr_f64<0x111>(v);    // row_shr:1
  v += dpp_shr_f64<0x112>(v);    // row_shr:2
  v += dpp_shr_f64<0x114>(v);    // row_shr:4
  v += dpp_shr_f64<0x118>(v);    // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  if (W == 64) v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

template <int W>
__device__ __forceinline__ double grp_last(double v, int half) {
  if (W == 64) return wave_last(v);
  const int l = (int)__double2loint(v), h = (int)__double2hiint(v);
  const int lo0 = __builtin_amdgcn_readlane(l, 31), hi0 = __builtin_amdgcn_readlane(h, 31);
  const int lo1 = __builtin_amdgcn_readlane(l, 63), hi1 = __builtin_amdgcn_readlane(h, 63);
  return half ? __hiloint2double(hi1, lo1) : __hiloint2double(hi0, lo0);
}

template <int W>
__device__ __forceinline__ double grp_sum(double v, int half) { return grp_last<W>(grp_incl_scan<W>(v), half); }

__device__ __forceinline__ float lane_f32(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// lane k of this lane's group
template <int W>
__device__ __forceinline__ float grp_lane_f32(float v, int k, int half) {
  if (W == 64) return lane_f32(v, k);
  const float a = lane_f32(v, k), b = lane_f32(v, 32 + k);
  return half ? b : a;
}

__device__ __forceinline__ float fast_rsq(float x) { return __builtin_amdgcn_rsqf(x); }

// sin and cos of an FP64 angle from a table at multiples of pi/64
// (BatchArgs::trig, filled on the host).  Cody-Waite reduction x = k pi/64 +
// r (pi/64 split into 33 + 33 + 53 significant bits, each term applied with
// one FMA) leaves |r| <= pi/128; then sin x = s_k cos r + c_k sin r and
// cos x = c_k cos r - s_k sin r, with the Taylor series of sin r (through
// r^9) and cos r (through r^8): truncation below 1e-19 on that interval.
// Arguments beyond 1e5 rad take the library routine.  The constants are read
// from a table in LDS (`kSinCosTable`, copied by every evaluating kernel):
// held in registers they would stay live across a local search's whole
// iteration loop and cost occupancy.
enum { kSc64OverPi = 0, kScC1 = 1, kScC2 = 2, kScC3 = 3, kScSin = 4, kScCos = 8, kScN = 12 };
__device__ const double kSinCosTable[kScN] = {
    20.371832715762604,      // 64/pi
    0.049087385210441425,    // pi/64, first 33 bits
    1.8990939082199894e-12,  // next 33 bits
    6.319582027487346e-23,   // remainder
    // sin r = r + r z (-1/3! + z (1/5! + z (-1/7! + z / 9!))), z = r^2
    -0.16666666666666666, 0.008333333333333333, -0.0001984126984126984, 2.7557319223985893e-06,
    // cos r = 1 + z (-1/2! + z (1/4! + z (-1/6! + z / 8!)))
    -0.5, 0.041666666666666664, -0.001388888888888889, 2.48015873015873e-05};

// Arguments outside [-1e5, 1e5] (and NaN): the library routine, kept out of
// line so that its own constants are not hoisted into callers' loops.
__device__ __attribute__((noinline)) void sincos_f64_far(double x, double *sn, double *cs) { sincos(x, sn, cs); }

__device__ __forceinline__ void sincos_f64(double x, double *sn, double *cs, const double *T, const double *trig) {
  if (!(fabs(x) <= 1.0e5)) {
    sincos_f64_far(x, sn, cs);
    return;
  }
  const double k = rint(x * T[kSc64OverPi]);
  double r = fma(-k, T[kScC1], x);
  r = fma(-k, T[kScC2], r);
  r = fma(-k, T[kScC3], r);
  const double z = r * r;
  double ps = fma(T[kScSin + 3], z, T[kScSin + 2]);
  ps = fma(ps, z, T[kScSin + 1]);
  ps = fma(ps, z, T[kScSin]);
  const double sr = fma(ps * z, r, r);
  double pc = fma(T[kScCos + 3], z, T[kScCos + 2]);
  pc = fma(pc, z, T[kScCos + 1]);
  pc = fma(pc, z, T[kScCos]);
  const double cr = fma(pc, z, 1.0);
  const int j = ((int)k) & (kTrigN - 1);
  const double sk = trig[2 * j], ck = trig[2 * j + 1];
  *sn = fma(sk, cr, ck * sr);
  *cs = fma(ck, cr, -(sk * sr));
}

// 1/sqrt(a) in FP64: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt_f64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  const double h = 0.5 * a;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11) and the stream layout of the search:
// key = (seed lo, seed hi), counter = (ligand id, run, generation,
// individual << 16 | stream << 10 | word >> 2), word = lane word & 3.
// ---------------------------------------------------------------------------
enum : uint32_t { kStInit = 0, kStSelect = 1, kStCross = 2, kStMutate = 3, kStLsPick = 4 };

__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

struct Rng {
  uint32_t k0, k1, lig, run, gen;
  __device__ uint32_t word(uint32_t indiv, uint32_t stream, uint32_t w) const {
    uint4 o = philox(make_uint4(lig, run, gen, (indiv << 16) | (stream << 10) | (w >> 2)), k0, k1);
    uint32_t s = w & 3;
    return s == 0 ? o.x : (s == 1 ? o.y : (s == 2 ? o.z : o.w));
  }
  __device__ uint4 block(uint32_t indiv, uint32_t stream, uint32_t blk) const {
    return philox(make_uint4(lig, run, gen, (indiv << 16) | (stream << 10) | blk), k0, k1);
  }
};
__device__ __forceinline__ double unif(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }
__device__ __forceinline__ uint32_t randint(uint32_t x, uint32_t n) {
  return (uint32_t)(((uint64_t)x * n) >> 32);
}

// ---------------------------------------------------------------------------
// Quaternion helpers (w, x, y, z), FP64.
// ---------------------------------------------------------------------------
struct Q4 {
  double w, x, y, z;
};
__device__ __forceinline__ Q4 qmul(Q4 a, Q4 b) {
  return {a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
          a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w};
}
__device__ __forceinline__ Q4 qnormalize(Q4 q) {
  double n = sqrt(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  double in = 1.0 / n;
  return {q.w * in, q.x * in, q.y * in, q.z * in};
}
// q <- exp(w/2) (x) q, renormalised
__device__ __forceinline__ Q4 apply_rotvec(Q4 q, double wx, double wy, double wz) {
  double th = sqrt(wx * wx + wy * wy + wz * wz);
  double s, c;
  sincos(0.5 * th, &s, &c);
  double f = th > 1e-300 ? s / th : 0.5;
  Q4 r = {c, f * wx, f * wy, f * wz};
  return qnormalize(qmul(r, q));
}
__device__ __forceinline__ double wrap_angle(double th) {
  const double twopi = 6.283185307179586476925;
  return th - twopi * floor((th + 3.14159265358979323846) / twopi);
}

// ---------------------------------------------------------------------------
// Shared memory of one evaluating wavefront.  CAP = atom capacity (64/128).
// ---------------------------------------------------------------------------
template <int CAP, int NT = kMaxTor>
struct EvalLds {
  // prefix-sum slots: at most one per torsion range end and start, plus the
  // totals, and never more than the atoms
  static constexpr int kSlots = 2 * NT + 1 < CAP ? 2 * NT + 1 : CAP;
  double x[3][CAP];   // posed coordinates (component-major)
  double g[CAP][3];   // dE/dx accumulators
  union {
    double tm[NT][12];        // torsion rigid transforms T_k = (R_k | w_k) (pose phase)
    double pre[kSlots][6];    // inclusive prefix sums of (g, (x-t) x g) at the slot atoms (gradient phase)
  };
  int tpar[NT];               // parent torsion of each torsion (-1: root fragment)
  double geno[kStride];        // genotype being evaluated
  double grad[kStride];        // output gradient
  double rot[9];               // global rotation matrix of the pose
  double sc[kScN];             // sin / cos constants (kSinCosTable)
};

// A zero the compiler cannot see through, produced anew by every call.  An
// address or bound derived from it is recomputed inside a local search's
// iteration loop instead of being hoisted into a register for the whole
// loop (one instruction against one register of occupancy).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// Per-kernel set-up of the evaluation LDS (before the first barrier).
template <int CAP, int NT>
__device__ __forceinline__ void init_eval_lds(EvalLds<CAP, NT> &S, int lane) {
  if (lane < kScN) S.sc[lane] = kSinCosTable[lane];
}

// Ligand being evaluated, with the lane's atom records (reference
// coordinates, map, charge, owner torsion; atom c * W + lane) and its
// torsion's indices for the gradient phase held in registers for a whole
// local search.  The torsion axis records of the pose phase and the pair
// records are re-read from L1-resident global memory inside every evaluation:
// holding those as well takes the kernel past 128 VGPRs, one wavefront per
// SIMD fewer.
template <int CAP>
struct LaneLig {
  static constexpr int kAPL = CAP >= 64 ? CAP / 64 : 1;
  LigDesc L;
  double y[kAPL][3];
  int map[kAPL], owner[kAPL], slot[kAPL];
  float q[kAPL];
  int ts, te, ta, tb;   // ts, te: prefix-sum slots of the torsion's range (TorRec s_slot, e_slot)
  double tinv;
  __device__ void load(const EvalConst &C, int li, int lane) {
    L = C.batch.lig[li];
    constexpr int W = CAP >= 64 ? 64 : 32;
#pragma unroll
    for (int c = 0; c < kAPL; ++c) {
      const int i = c * W + lane;
      if (i < L.n_atoms) {
        const AtomGeo &ag = C.batch.geo[L.atom_off + i];
        const AtomInfo &ai = C.batch.info[L.atom_off + i];
        y[c][0] = ag.y[0]; y[c][1] = ag.y[1]; y[c][2] = ag.y[2];
        map[c] = ai.map; q[c] = ai.q; owner[c] = ai.owner; slot[c] = ai.slot;
      } else {
        y[c][0] = y[c][1] = y[c][2] = 0.0;
        map[c] = 0; q[c] = 0.0f; owner[c] = -1; slot[c] = -1;
      }
    }
    if (lane < L.n_tor) {
      const TorRec &tr = C.batch.tors[L.tor_off + lane];
      ts = tr.s_slot; te = tr.e_slot; ta = tr.a; tb = tr.b; tinv = tr.inv_len;
    } else {
      ts = te = ta = tb = 0; tinv = 0.0;
    }
  }
};

// Trilinear interpolation of map_m + q map_e + |q| map_d with its gradient,
// plus the out-of-box restraint.  FP64 (near the map cap the corner values
// are ~1e5 while their differences, the gradient, are small).
__device__ __forceinline__ double grid_energy(const GridArgs &G, double k_out, int m, float qf, const double x[3],
                                              double g[3]) {
  const double q = qf, aq = fabs(q);
  const double u[3] = {(x[0] - G.ox) * G.inv_h, (x[1] - G.oy) * G.inv_h, (x[2] - G.oz) * G.inv_h};
  const int n[3] = {G.nx, G.ny, G.nz};
  double f[3], uc[3];
  int i0[3];
  bool clamped[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double top = (double)(n[d] - 1 + opaque_zero());
    clamped[d] = !(u[d] >= 0.0 && u[d] <= top);    // NaN counts as clamped
    uc[d] = fmin(fmax(u[d], 0.0), top);             // NaN -> 0 (fmax drops NaN)
    int ii = (int)floor(uc[d]);
    ii = min(max(ii, 0), n[d] - 2);
    i0[d] = ii;
    f[d] = uc[d] - (double)ii;
  }
  // record index in 32 bits with 24-bit products: the host keeps nx * ny
  // below 2^24 and the whole map set below 2^32 records
  const uint32_t sy = (uint32_t)G.nx, sz = (uint32_t)G.nx * (uint32_t)G.ny;
  const uint32_t base = __umul24(__umul24((uint32_t)m, (uint32_t)G.nz) + (uint32_t)i0[2], sz) +
                        __umul24((uint32_t)i0[1], sy) + (uint32_t)i0[0];
  const float4 *M = reinterpret_cast<const float4 *>(G.maps) + base;
  double v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const uint32_t off = ((c & 1) ? 1u : 0u) + ((c & 2) ? sy : 0u) + ((c & 4) ? sz : 0u);
    const float4 r = M[off];
    v[c] = fma(aq, (double)r.z, fma(q, (double)r.y, (double)r.x));
  }
  const double fx = f[0], fy = f[1], fz = f[2];
  // along x (corner c: bit 0 = x, bit 1 = y, bit 2 = z), then y, then z
  const double d00 = v[1] - v[0], d10 = v[3] - v[2], d01 = v[5] - v[4], d11 = v[7] - v[6];
  const double a00 = fma(fx, d00, v[0]), a10 = fma(fx, d10, v[2]);
  const double a01 = fma(fx, d01, v[4]), a11 = fma(fx, d11, v[6]);
  const double e0 = a10 - a00, e1 = a11 - a01;
  const double b0 = fma(fy, e0, a00), b1 = fma(fy, e1, a01);
  const double c0 = fma(fy, d10 - d00, d00), c1 = fma(fy, d11 - d01, d01);
  double E = fma(fz, b1 - b0, b0);
  const double dEdu[3] = {fma(fz, c1 - c0, c0), fma(fz, e1 - e0, e0), b1 - b0};
  const double o[3] = {G.ox, G.oy, G.oz};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!clamped[d]) {
      g[d] = dEdu[d] * G.inv_h;
    } else {
      double dd = x[d] - (o[d] + G.h * uc[d]);
      E += k_out * dd * dd;
      g[d] = 2.0 * k_out * dd;
    }
  }
  return E;
}

// One intramolecular pair in FP32: returns the energy, writes dE/dr / r.
__device__ __forceinline__ float pair_energy(const FFConst &K, const LJRec &lj, float qq, float dsv, float r2,
                                             float *fscale) {
  const bool floored = !(r2 >= K.r_floor2);
  const float r2c = floored ? K.r_floor2 : r2;   // NaN -> the floor
  const float inv_r = fast_rsq(r2c);
  const float r = r2c * inv_r;
  // smoothed 12-6 / 12-10
  const float dr = r - lj.r0;
  const float sh = __builtin_amdgcn_fmed3f(dr, -K.half_smooth, K.half_smooth);
  const float rr = r - sh;
  const float slope = fabsf(dr) > K.half_smooth ? 1.0f : 0.0f;
  const float inv = fast_rcp(rr);
  const float i2 = inv * inv, i6 = i2 * i2 * i2, i12 = i6 * i6;
  const bool hb = lj.hb != 0.0f;
  const float im = hb ? i6 * i2 * i2 : i6;
  const float mm = hb ? 10.0f : 6.0f;
  const float e_lj = lj.A * i12 - lj.B * im;
  const float d_lj = slope * (mm * lj.B * im - 12.0f * lj.A * i12) * inv;
  // distance-dependent dielectric electrostatics: qq D / (N r), D = 1 + k e, N = A D + B
  const float ex = fast_exp2(-K.diel_lB_log2e * r);
  const float D = 1.0f + K.diel_k * ex;
  const float N = K.diel_A * D + K.diel_B;
  const float inv_Nr = fast_rcp(N * r);
  const float e_el = qq * D * inv_Nr;
  const float d_el = -qq * (D * N + K.diel_c1 * r * ex) * inv_Nr * inv_Nr;
  // desolvation
  const float gds = fast_exp2(-K.ds_log2e * r2c);
  const float e_ds = dsv * gds;
  const float d_ds = -e_ds * r * K.inv_s2;
  // a select on the factor, not on the whole force, keeps the force terms
  // out of a branch
  *fscale = (d_lj + d_el + d_ds) * (floored ? 0.0f : inv_r);
  return e_lj + e_el + e_ds;
}

// Rodrigues rotation matrix of angle th about unit u (row major 3x3).
__device__ __forceinline__ void rot_matrix(const double u[3], double c, double s, double R[9]) {
  const double t = 1.0 - c;
  R[0] = c + t * u[0] * u[0];
  R[1] = t * u[0] * u[1] - s * u[2];
  R[2] = t * u[0] * u[2] + s * u[1];
  R[3] = t * u[1] * u[0] + s * u[2];
  R[4] = c + t * u[1] * u[1];
  R[5] = t * u[1] * u[2] - s * u[0];
  R[6] = t * u[2] * u[0] - s * u[1];
  R[7] = t * u[2] * u[1] + s * u[0];
  R[8] = c + t * u[2] * u[2];
}

// Evaluate the genotype in S.geno.  Returns the total energy (every lane);
// with GRAD the gradient is written to S.grad[0..39]; terms (lane 0) gets
// {inter, intra}.  Ends with the LDS in a consistent state (barrier).
// Pairs staged in LDS by a local search (see k_ls_generation): the first `n`
// pair records of the ligand and the whole type-pair table, at byte offset
// `off` of the work-group's dynamic LDS.
struct PairStage {
  int off, n;
};

template <int CAP, bool GRAD, bool STAGE = false, int W = 64, int NT = kMaxTor, int UNROLL = 1>
__device__ double evaluate(const EvalConst &C, const LaneLig<CAP> &LL, EvalLds<CAP, NT> &S, int lane, double *inter_out,
                           double *intra_out, PairStage st = PairStage{0, 0}, int half = 0) {
  constexpr int APL = CAP / W;
  static_assert(LaneLig<CAP>::kAPL == APL && (CAP >= 64) == (W == 64), "LaneLig holds atom c * W + lane");
  const LigDesc &L = LL.L;
  // keep the ligand records below from being hoisted out of a caller's loop,
  // and recompute the lane's addresses per evaluation (opaque_zero)
  asm volatile("" ::: "memory");
  lane += opaque_zero();
  // global rigid transform x = R y + t (y relative to the centre): R from the
  // normalised quaternion, one element per lane, kept in LDS
  const double t0 = S.geno[0], t1 = S.geno[1], t2 = S.geno[2];
  if (lane < 9) {
    const double qw0 = S.geno[3], qx0 = S.geno[4], qy0 = S.geno[5], qz0 = S.geno[6];
    const double inv = rsqrt_f64(qw0 * qw0 + qx0 * qx0 + qy0 * qy0 + qz0 * qz0);
    const double w = qw0 * inv, x = qx0 * inv, y = qy0 * inv, z = qz0 * inv;
    double v;
    switch (lane) {
      case 0: v = 1 - 2 * (y * y + z * z); break;
      case 1: v = 2 * (x * y - w * z); break;
      case 2: v = 2 * (x * z + w * y); break;
      case 3: v = 2 * (x * y + w * z); break;
      case 4: v = 1 - 2 * (x * x + z * z); break;
      case 5: v = 2 * (y * z - w * x); break;
      case 6: v = 2 * (x * z - w * y); break;
      case 7: v = 2 * (y * z + w * x); break;
      default: v = 1 - 2 * (x * x + y * y); break;
    }
    S.rot[lane] = v;
  }
  // torsion transforms T_k(y) = R_k (y - o_k) + o_k in the reference frame
  if (lane < L.n_tor) {
    const TorRec &tr = C.batch.tors[L.tor_off + lane];
    const double to[3] = {tr.o[0], tr.o[1], tr.o[2]};
    const double tu[3] = {tr.u[0], tr.u[1], tr.u[2]};
    double sn, cs, Rk[9];
    sincos_f64(S.geno[7 + lane], &sn, &cs, S.sc + opaque_zero(), C.batch.trig);
    rot_matrix(tu, cs, sn, Rk);
#pragma unroll
    for (int e = 0; e < 9; ++e) S.tm[lane][e] = Rk[e];
#pragma unroll
    for (int r = 0; r < 3; ++r)
      S.tm[lane][9 + r] = to[r] - (Rk[3 * r] * to[0] + Rk[3 * r + 1] * to[1] + Rk[3 * r + 2] * to[2]);
    S.tpar[lane] = tr.parent;
  }
  __syncthreads();
  // atoms: pose and inter-molecular energy
  double e_inter = 0.0;
#pragma unroll
  for (int c = 0; c < APL; ++c) {
    const int i = c * W + lane;
    if (i < L.n_atoms) {
      // torsions moving the atom, deepest first, then the global transform
      double y0 = LL.y[c][0], y1 = LL.y[c][1], y2 = LL.y[c][2];
      for (int k = LL.owner[c]; k >= 0; k = S.tpar[k]) {
        const double *M = S.tm[k];
        const double n0 = fma(M[0], y0, fma(M[1], y1, fma(M[2], y2, M[9])));
        const double n1 = fma(M[3], y0, fma(M[4], y1, fma(M[5], y2, M[10])));
        const double n2 = fma(M[6], y0, fma(M[7], y1, fma(M[8], y2, M[11])));
        y0 = n0; y1 = n1; y2 = n2;
      }
      double x[3];
#pragma unroll
      for (int r = 0; r < 3; ++r) x[r] = S.rot[3 * r] * y0 + S.rot[3 * r + 1] * y1 + S.rot[3 * r + 2] * y2;
      x[0] += t0; x[1] += t1; x[2] += t2;
      double g[3];
      e_inter += grid_energy(C.grid, C.ff.k_out, LL.map[c], LL.q[c], x, g);
      S.x[0][i] = x[0]; S.x[1][i] = x[1]; S.x[2][i] = x[2];
      if (GRAD) { S.g[i][0] = g[0]; S.g[i][1] = g[1]; S.g[i][2] = g[2]; }
    }
  }
  __syncthreads();
  // intramolecular pairs, 64 per step in list order
  double e_intra = 0.0;
  const PairRec *pr = C.batch.pairs + L.pair_off;
  const LJRec *ljt = C.batch.lj;
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  const LJRec *s_lj = reinterpret_cast<const LJRec *>(dyn_lds + st.off);
  const PairRec *s_pr = reinterpret_cast<const PairRec *>(dyn_lds + st.off + C.ff.n_types * C.ff.n_types * 16);
  // two-deep prefetch: the record of the step after next is loaded while the
  // type-pair record of the next step is fetched with the next record (which
  // arrived one step earlier), so neither load waits at its use.  The batch's
  // pair array ends with 128 spare records, so these loads stay in bounds;
  // past the ligand's list they read records that are not used
  PairRec rec_a, rec_b;
  LJRec lj_a;
  if (lane < L.n_pairs) {
    rec_a = (STAGE && lane < st.n) ? s_pr[lane] : pr[lane];
    rec_b = (STAGE && lane + W < st.n) ? s_pr[lane + W] : pr[lane + W];
    lj_a = STAGE ? s_lj[rec_a.ijt >> 16] : ljt[rec_a.ijt >> 16];
  }
  // 32-bit byte offsets from the ligand's list (a list and its spare records
  // span far less than 4 GiB)
  auto pair_at = [&](int q) -> PairRec {
    return (STAGE && q < st.n) ? s_pr[q]
                               : *reinterpret_cast<const PairRec *>(reinterpret_cast<const char *>(pr) +
                                                                    (uint32_t)q * (uint32_t)sizeof(PairRec));
  };
  auto lj_of = [&](const PairRec &r) -> LJRec { return STAGE ? s_lj[r.ijt >> 16] : ljt[r.ijt >> 16]; };
  // One pair step.  A lane with `live` false (past the list, in the second
  // step of a trip) computes on a record that is not the ligand's and keeps
  // its sum and the forces unchanged; its atom indices are cut to the array
  // (the ligand's own indices are below CAP, a power of two).
  static_assert((CAP & (CAP - 1)) == 0, "atom index mask");
  struct PairGeo {
    int i, j;
    double dx, dy, dz;
  };
  auto pair_geo = [&](const PairRec &rec) -> PairGeo {
    const int i = rec.ijt & (CAP - 1), j = (rec.ijt >> 8) & (CAP - 1);
    return PairGeo{i, j, S.x[0][i] - S.x[0][j], S.x[1][i] - S.x[1][j], S.x[2][i] - S.x[2][j]};
  };
  auto pair_terms = [&](const PairRec &rec, const LJRec &lj, const PairGeo &g, bool live) {
    const float r2 = (float)(g.dx * g.dx + g.dy * g.dy + g.dz * g.dz);
    float fs;
    const double e = (double)pair_energy(C.ff, lj, rec.qq, rec.dsv, r2, &fs);
    e_intra = live ? e_intra + e : e_intra;   // a select: the terms stay out of the branch below
    if (GRAD && live) {
      const double f = (double)fs;
      const double fx = f * g.dx, fy = f * g.dy, fz = f * g.dz;
      atomicAdd(&S.g[g.i][0], fx);
      atomicAdd(&S.g[g.i][1], fy);
      atomicAdd(&S.g[g.i][2], fz);
      atomicAdd(&S.g[g.j][0], -fx);
      atomicAdd(&S.g[g.j][1], -fy);
      atomicAdd(&S.g[g.j][2], -fz);
    }
  };
  auto do_pair = [&](const PairRec &rec, const LJRec &lj, bool live) { pair_terms(rec, lj, pair_geo(rec), live); };
  // The step count is the same for every lane of the group (the last step
  // masks the lanes past the list), so step k of every lane is one and the
  // same instruction in either loop form below: the form (a launch-shape
  // option of the local search) then changes neither a lane's order of pairs
  // nor the order in which the lanes' force additions reach an accumulator.
  const int n_steps = (L.n_pairs + W - 1) / W;
  if (UNROLL == 1) {
    for (int step = 0; step < n_steps; ++step) {
      const int p = step * W + lane;
      if (p >= L.n_pairs) continue;
      const PairRec rec = rec_a;
      const LJRec lj = lj_a;
      rec_a = rec_b;
      rec_b = pair_at(p + 2 * W);
      lj_a = lj_of(rec_a);
      do_pair(rec, lj, true);
    }
  } else {
    // Two steps per trip with fixed register roles: rec_a holds the record
    // of the trip's first step and rec_b that of its second, each reloaded
    // in place two steps ahead, so no record is moved between registers
    // (a move of a record still in flight would wait for its load).  Every
    // step but the last covers whole groups, so only the second step of a
    // trip and a final odd step mask lanes; the second step computes on every
    // lane and masks only its sum and forces, so its loads are issued a step
    // ahead of their use.
    int step = 0;
    for (; step + 1 < n_steps; step += 2) {
      const int p = step * W + lane;   // below n_pairs: not the last step
      const PairRec c0 = rec_a;
      const LJRec j0 = lj_a;
      const LJRec lj_b = lj_of(rec_b);
      rec_a = pair_at(p + 2 * W);
      const PairRec c1 = rec_b;
      // both steps' positions are read before the first step's force
      // additions, which the LDS would otherwise serve first
      const PairGeo g0 = pair_geo(c0), g1 = pair_geo(c1);
      pair_terms(c0, j0, g0, true);
      const int p1 = p + W;
      const bool live = p1 < L.n_pairs;
      rec_b = pair_at(live ? p1 + 2 * W : p);   // past the list: read a valid record, unused
      lj_a = lj_of(rec_a);
      pair_terms(c1, lj_b, g1, live);
    }
    if (step < n_steps && step * W + lane < L.n_pairs) do_pair(rec_a, lj_a, true);
  }
  // one wavefront sum unless the caller wants the two parts
  double total;
  if (inter_out || intra_out) {
    const double inter = grp_sum<W>(e_inter, half), intra = grp_sum<W>(e_intra, half);
    if (inter_out) *inter_out = inter;
    if (intra_out) *intra_out = intra;
    total = inter + intra;
  } else {
    total = grp_sum<W>(e_inter + e_intra, half);
  }
  if (!GRAD) return total;
  __syncthreads();
  // gradient back-projection: prefix sums over the internal atom order of
  // v_i = (g_i, (x_i - t) x g_i); each torsion's moving set is a range
  double carry[6] = {0, 0, 0, 0, 0, 0};
  double vv[APL][6];
#pragma unroll
  for (int c = 0; c < APL; ++c) {
    const int i = c * W + lane;
    if (i < L.n_atoms) {
      const double gx = S.g[i][0], gy = S.g[i][1], gz = S.g[i][2];
      const double rx = S.x[0][i] - t0, ry = S.x[1][i] - t1, rz = S.x[2][i] - t2;
      vv[c][0] = gx; vv[c][1] = gy; vv[c][2] = gz;
      vv[c][3] = ry * gz - rz * gy;
      vv[c][4] = rz * gx - rx * gz;
      vv[c][5] = rx * gy - ry * gx;
    } else {
#pragma unroll
      for (int e = 0; e < 6; ++e) vv[c][e] = 0.0;
    }
  }
  __syncthreads();   // tm (pose phase) is dead; pre aliases it
#pragma unroll
  for (int c = 0; c < APL; ++c) {
    const int i = c * W + lane;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      double s = grp_incl_scan<W>(vv[c][e]) + carry[e];
      if (i < L.n_atoms && LL.slot[c] >= 0) S.pre[LL.slot[c]][e] = s;
      carry[e] = grp_last<W>(s, half);
    }
  }
  __syncthreads();
  if (lane < kStride && lane < W) {
    double gv = 0.0;
    if (lane < 6) gv = S.pre[0][lane];   // dE/dt and dE/domega: totals (the last atom's slot)
    S.grad[lane] = gv;
  }
  if (lane < L.n_tor) {
    const int ts = LL.ts, te = LL.te, ta = LL.ta, tb = LL.tb;
    const double tinv_len = LL.tinv;
    double F[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) F[e] = S.pre[te][e] - (ts >= 0 ? S.pre[ts][e] : 0.0);
    const double ax = S.x[0][ta] - t0, ay = S.x[1][ta] - t1, az = S.x[2][ta] - t2;
    // torque about the axis point a: sum (x_i - t) x g_i - (x_a - t) x sum g_i
    const double tx = F[3] - (ay * F[2] - az * F[1]);
    const double ty = F[4] - (az * F[0] - ax * F[2]);
    const double tz = F[5] - (ax * F[1] - ay * F[0]);
    const double ux = (S.x[0][tb] - S.x[0][ta]) * tinv_len;
    const double uy = (S.x[1][tb] - S.x[1][ta]) * tinv_len;
    const double uz = (S.x[2][tb] - S.x[2][ta]) * tinv_len;
    S.grad[7 + lane] = ux * tx + uy * ty + uz * tz;
  }
  __syncthreads();
  return total;
}

__device__ __forceinline__ bool genotype_finite(const double *geno, int n_tor) {
  bool ok = true;
  for (int e = 0; e < 7 + n_tor; ++e) ok = ok && isfinite(geno[e]);
  return ok;
}

// ---------------------------------------------------------------------------
// ad_score_poses: one work-group (one wavefront) per pose.
// ---------------------------------------------------------------------------
template <int CAP, bool GRAD>
__global__ __launch_bounds__(64) void k_score(EvalConst C, int n, const int *__restrict__ lig_idx,
                                              const float *__restrict__ geno, float *__restrict__ E_out,
                                              float *__restrict__ G_out, float *__restrict__ T_out) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int li = lig_idx[p];
  if (li < 0 || li >= C.batch.n_lig || C.batch.lig[li].n_atoms > CAP) {
    // invalid index (only reachable with device-side indices): NaN result
    if (lane == 0) E_out[(size_t)p] = __builtin_nanf("");
    if (GRAD && G_out && lane < kStride) G_out[(size_t)p * kStride + lane] = __builtin_nanf("");
    if (T_out && lane < 3) T_out[(size_t)p * 3 + lane] = __builtin_nanf("");
    return;
  }
  LaneLig<CAP> LL;
  LL.load(C, li, lane);
  if (lane < kStride) S.geno[lane] = (double)geno[(size_t)p * kStride + lane];
  __syncthreads();
  double inter, intra;
  double E = evaluate<CAP, GRAD>(C, LL, S, lane, &inter, &intra);
  const bool fin = genotype_finite(S.geno, LL.L.n_tor);
  const float nanf = __builtin_nanf("");
  if (lane == 0) E_out[p] = fin ? (float)E : nanf;
  if (T_out && lane < 3) {
    double tv = lane == 0 ? inter : (lane == 1 ? intra : inter + (double)C.ff.w_tor * LL.L.n_tor);
    T_out[(size_t)p * 3 + lane] = fin ? (float)tv : nanf;
  }
  if (GRAD && lane < kStride) {
    double gv = (lane == 6 || lane >= 7 + LL.L.n_tor) ? 0.0 : S.grad[lane];
    G_out[(size_t)p * kStride + lane] = fin ? (float)gv : nanf;
  }
}

// ---------------------------------------------------------------------------
// ADADELTA local search: one wavefront per individual, `iters` evaluations.
// Degrees of freedom on lanes: 0-2 translation, 3-5 rotation vector,
// 7..7+T-1 torsions (lane 6 is the fourth quaternion slot).
// ---------------------------------------------------------------------------
template <int CAP, bool STAGE = false, int W = 64, int NT = kMaxTor, int UNROLL = 1>
__device__ void adadelta_wave(const EvalConst &C, const LaneLig<CAP> &LL, EvalLds<CAP, NT> &S, int lane,
                              float *geno_io, float *E_io, int iters, double rho_d, double eps_d,
                              PairStage st = PairStage{0, 0}, int half = 0, bool write = true) {
  const int T = LL.L.n_tor;
  // genes are FP32 values; the step arithmetic runs in FP32 with native
  // square roots (the accumulated squared gradient in FP64: gradients of
  // clashing poses overflow FP32 when squared)
  const bool gl = lane < kStride && lane < W;   // the lane holds a gene slot
  float gene = gl ? geno_io[lane] : 0.0f;
  float best_gene = gene;
  double best_E = INFINITY;
  double Eg2 = 0.0;
  float Edx2 = 0.0f;
  const bool dof = lane < 6 || (lane >= 7 && lane < 7 + T);
  for (int it = 0; it < iters; ++it) {
    // step constants recomputed from the (scalar) arguments every iteration
    const double zd = (double)opaque_zero();
    const float rho = (float)(rho_d + zd), eps = (float)(eps_d + zd);
    if (gl) S.geno[lane] = (double)gene;
    __syncthreads();
    const double E = evaluate<CAP, true, STAGE, W, NT, UNROLL>(C, LL, S, lane, nullptr, nullptr, st, half);
    const double gd = dof ? S.grad[lane] : 0.0;
    if (E < best_E) {
      best_E = E;
      best_gene = gene;
    }
    Eg2 = (rho_d + zd) * Eg2 + (1.0 - (rho_d + zd)) * gd * gd;
    const float rg = fast_rsq((float)(Eg2 + eps_d));
    const float dx = dof ? -__builtin_amdgcn_sqrtf(Edx2 + eps) * rg * (float)gd : 0.0f;
    Edx2 = rho * Edx2 + (1.0f - rho) * dx * dx;
    // orientation: q <- exp(dw/2) (x) q from the three rotation lanes
    const float w0 = grp_lane_f32<W>(dx, 3, half), w1 = grp_lane_f32<W>(dx, 4, half);
    const float w2 = grp_lane_f32<W>(dx, 5, half);
    const float qw = grp_lane_f32<W>(gene, 3, half), qx = grp_lane_f32<W>(gene, 4, half);
    const float qy = grp_lane_f32<W>(gene, 5, half), qz = grp_lane_f32<W>(gene, 6, half);
    const float th = __builtin_amdgcn_sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
    float sh, ch;
    __sincosf(0.5f * th, &sh, &ch);
    const float f = th > 1e-30f ? sh * fast_rcp(th) : 0.5f;
    const float rx = f * w0, ry = f * w1, rz = f * w2;
    float nw = ch * qw - rx * qx - ry * qy - rz * qz;
    float nx = ch * qx + rx * qw + ry * qz - rz * qy;
    float ny = ch * qy - rx * qz + ry * qw + rz * qx;
    float nz = ch * qz + rx * qy - ry * qx + rz * qw;
    const float inv = fast_rsq(nw * nw + nx * nx + ny * ny + nz * nz);
    if (lane < 3) gene += dx;
    else if (lane == 3) gene = nw * inv;
    else if (lane == 4) gene = nx * inv;
    else if (lane == 5) gene = ny * inv;
    else if (lane == 6) gene = nz * inv;
    else if (lane < 7 + T) {
      float th2 = gene + dx;
      th2 -= 6.2831853071795865f * floorf((th2 + 3.14159265358979f) * 0.15915494309189535f);
      gene = th2;
    }
    __syncthreads();
  }
  if (gl && write) geno_io[lane] = best_gene;
  if (lane == 0 && write) *E_io = (float)best_E;
}

template <int CAP>
__global__ __launch_bounds__(64) void k_local_search(EvalConst C, int n, const int *__restrict__ lig_idx,
                                                     float *__restrict__ geno, float *__restrict__ E, int iters,
                                                     double rho, double eps) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int li = lig_idx[p];
  if (li < 0 || li >= C.batch.n_lig || C.batch.lig[li].n_atoms > CAP) {
    if (lane == 0) E[p] = __builtin_nanf("");
    return;
  }
  LaneLig<CAP> LL;
  LL.load(C, li, lane);
  adadelta_wave<CAP>(C, LL, S, lane, geno + (size_t)p * kStride, E + p, iters, rho, eps);
}

// ---------------------------------------------------------------------------
// Packed evaluation (ad_score_poses_shape / ad_local_search_shape with
// AD_SHAPE_PACKED): poses 2w and 2w + 1 of one ligand (at most kDualAtoms
// atoms and kDualTor torsions) on work-group w, one per 32-lane half, through
// the same evaluate / adadelta_wave instantiation as the packed local search
// of the docking kernel.  A half whose pose is past n recomputes the last
// pose and writes nothing; a half whose pose names another ligand than pose
// 2w writes NaN.
// ---------------------------------------------------------------------------
struct DualPose {
  int half, lane, p, li;
  bool write, ok;
};

__device__ __forceinline__ DualPose dual_pose(const EvalConst &C, int n, const int *lig_idx) {
  DualPose d;
  d.half = threadIdx.x >> 5;
  d.lane = threadIdx.x & 31;
  const int p0 = 2 * (int)blockIdx.x;
  d.write = p0 + d.half < n;
  d.p = min(p0 + d.half, n - 1);
  d.li = lig_idx[p0];   // uniform over the work-group
  const bool lig_ok = d.li >= 0 && d.li < C.batch.n_lig && C.batch.lig[d.li].n_atoms <= kDualAtoms &&
                      C.batch.lig[d.li].n_tor <= kDualTor;
  d.ok = lig_ok && lig_idx[d.p] == d.li;
  if (!lig_ok) d.li = -1;
  return d;
}

template <bool GRAD>
__global__ __launch_bounds__(64) void k_score_dual(EvalConst C, int n, const int *__restrict__ lig_idx,
                                                   const float *__restrict__ geno, float *__restrict__ E_out,
                                                   float *__restrict__ G_out, float *__restrict__ T_out) {
  __shared__ EvalLds<kDualAtoms, kDualTor> S2[2];
  const DualPose d = dual_pose(C, n, lig_idx);
  const int lane = d.lane, half = d.half;
  EvalLds<kDualAtoms, kDualTor> &S = S2[half];
  init_eval_lds(S, lane);
  const float nanf = __builtin_nanf("");
  if (d.li < 0) {   // no valid ligand for the work-group (device-side indices only)
    if (d.write) {
      if (lane == 0) E_out[d.p] = nanf;
      if (GRAD && G_out) {
        G_out[(size_t)d.p * kStride + lane] = nanf;
        if (lane < kStride - 32) G_out[(size_t)d.p * kStride + 32 + lane] = nanf;
      }
      if (T_out && lane < 3) T_out[(size_t)d.p * 3 + lane] = nanf;
    }
    return;
  }
  LaneLig<kDualAtoms> LL;
  LL.load(C, d.li, lane);
  S.geno[lane] = (double)geno[(size_t)d.p * kStride + lane];   // 32 slots: 7 + at most 25 torsions
  __syncthreads();
  double inter, intra;
  const double E = evaluate<kDualAtoms, GRAD, false, 32, kDualTor>(C, LL, S, lane, &inter, &intra,
                                                                   PairStage{0, 0}, half);
  if (!d.write) return;
  const bool fin = d.ok && genotype_finite(S.geno, LL.L.n_tor);
  if (lane == 0) E_out[d.p] = fin ? (float)E : nanf;
  if (T_out && lane < 3) {
    const double tv = lane == 0 ? inter : (lane == 1 ? intra : inter + (double)C.ff.w_tor * LL.L.n_tor);
    T_out[(size_t)d.p * 3 + lane] = fin ? (float)tv : nanf;
  }
  if (GRAD) {
    const double gv = (lane == 6 || lane >= 7 + LL.L.n_tor) ? 0.0 : S.grad[lane];
    G_out[(size_t)d.p * kStride + lane] = fin ? (float)gv : nanf;
    if (lane < kStride - 32) G_out[(size_t)d.p * kStride + 32 + lane] = fin ? 0.0f : nanf;
  }
}

__global__ __launch_bounds__(64) void k_local_search_dual(EvalConst C, int n, const int *__restrict__ lig_idx,
                                                          float *__restrict__ geno, float *__restrict__ E, int iters,
                                                          double rho, double eps) {
  __shared__ EvalLds<kDualAtoms, kDualTor> S2[2];
  const DualPose d = dual_pose(C, n, lig_idx);
  EvalLds<kDualAtoms, kDualTor> &S = S2[d.half];
  init_eval_lds(S, d.lane);
  if (d.li < 0) {
    if (d.write && d.lane == 0) E[d.p] = __builtin_nanf("");
    return;
  }
  LaneLig<kDualAtoms> LL;
  LL.load(C, d.li, d.lane);
  adadelta_wave<kDualAtoms, false, 32, kDualTor>(C, LL, S, d.lane, geno + (size_t)d.p * kStride, E + d.p, iters, rho,
                                                 eps, PairStage{0, 0}, d.half, d.write && d.ok);
  if (d.write && !d.ok && d.lane == 0) E[d.p] = __builtin_nanf("");
}

// ---------------------------------------------------------------------------
// Lamarckian GA on the GPU.  Population state per run R (ligand * nrun +
// run): genotypes [2][n_runs][pop][40] (ping-pong by generation parity) and
// energies [2][n_runs][pop].  Every genotype stored is exactly the one that
// was evaluated (genes are rounded to FP32 before evaluation).
// ---------------------------------------------------------------------------
__device__ __forceinline__ size_t pop_off(const DockArgs &D, int buf, int R) {
  return ((size_t)buf * D.n_runs + R) * D.pop;
}

__device__ __forceinline__ float round_gene(double v) { return (float)v; }

// byte offset of the staged pair area in k_ls_generation's dynamic LDS
__host__ __device__ __forceinline__ int stage_offset(int pop) { return (pop * 4 + 15) & ~15; }

// Draw the generation-0 individual `indiv` of (lig id, run): genes on lanes.
__device__ double init_gene(const GridArgs &G, const Rng &rng, int indiv, int lane, int n_tor) {
  const double PI = 3.14159265358979323846;
  double gene = 0.0;
  if (lane < 3) {
    const double o = lane == 0 ? G.ox : (lane == 1 ? G.oy : G.oz);
    const int n = lane == 0 ? G.nx : (lane == 1 ? G.ny : G.nz);
    gene = o + unif(rng.word(indiv, kStInit, lane)) * G.h * (double)(n - 1);
  }
  // orientation by Shoemake's method (every lane computes it; lanes 3-6 keep a component)
  const uint4 b = rng.block(indiv, kStInit, 0);
  const uint4 b1 = rng.block(indiv, kStInit, 1);
  const double u1 = unif(b.w), u2 = unif(b1.x), u3 = unif(b1.y);
  const double a = sqrt(1.0 - u1), c = sqrt(u1);
  double s2, c2, s3, c3;
  sincos(2.0 * PI * u2, &s2, &c2);
  sincos(2.0 * PI * u3, &s3, &c3);
  if (lane == 3) gene = a * s2;
  if (lane == 4) gene = a * c2;
  if (lane == 5) gene = c * s3;
  if (lane == 6) gene = c * c3;
  if (lane >= 7 && lane < 7 + n_tor) gene = -PI + 2.0 * PI * unif(rng.word(indiv, kStInit, 6 + (lane - 7)));
  return gene;
}

template <int CAP>
__global__ __launch_bounds__(64) void k_init_pop(EvalConst C, DockArgs D) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  const int lane = threadIdx.x;
  const int R = D.run_order[blockIdx.x / D.pop];
  const int i = blockIdx.x % D.pop;
  const int li = R / D.nrun, run = R % D.nrun;
  LaneLig<CAP> LL;
  LL.load(C, D.lig_map ? D.lig_map[li] : li, lane);
  const Rng rng{D.k0, D.k1, D.lig_id[li], (uint32_t)run, 0u};
  const float g = round_gene(init_gene(C.grid, rng, i, lane, LL.L.n_tor));
  if (lane < kStride) S.geno[lane] = (double)g;
  __syncthreads();
  const double E = evaluate<CAP, false>(C, LL, S, lane, nullptr, nullptr);
  const size_t off = pop_off(D, 0, R) + i;
  if (lane < kStride) D.geno[off * kStride + lane] = g;
  if (lane == 0) {
    D.energy[off] = (float)E;
    atomicAdd(&D.evals[R], 1ull);
  }
}

// lowest energy (lowest index on ties; NaN ranks as +inf) over a population
__device__ int wave_argmin(const float *E, int pop, int lane) {
  float bv = INFINITY;
  int bi = 0x7fffffff;
  for (int j = lane; j < pop; j += 64) {
    float v = E[j];
    if (!(v == v)) v = INFINITY;
    if (v < bv || (v == bv && j < bi)) {
      bv = v;
      bi = j;
    }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov < bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  return bi == 0x7fffffff ? 0 : bi;
}

__device__ __forceinline__ int tournament(const float *E, int pop, double tour_p, uint32_t w0, uint32_t w1,
                                          uint32_t w2) {
  const int a = (int)randint(w0, (uint32_t)pop), b = (int)randint(w1, (uint32_t)pop);
  const float ea = E[a], eb = E[b];
  const int better = (ea < eb || (ea == eb && a < b)) ? a : b;
  const int worse = better == a ? b : a;
  return unif(w2) < tour_p ? better : worse;
}

// Work queue of a generation launch.  Without a queue every work-group
// computes one item (the item is its block index).  With a queue (D.q_ga /
// D.q_ls set) the grid holds about as many work-groups as the device keeps
// resident, and each one takes the next item, or chunk of items, from the
// launch's counter (one per generation, zero at the start of the docking
// call) until the counter passes the item count.  Items are taken in item
// order, so the run order's longest-first ranking still decides what starts
// first, and items of stopped runs are skipped without a dispatch.  What an
// item computes does not depend on the work-group that takes it: results
// are bitwise the same with and without the queue.
__device__ __forceinline__ int next_ticket(unsigned int *ctr) {
  int t = 0;
  if (threadIdx.x == 0) t = (int)atomicAdd(ctr, 1u);
  return __builtin_amdgcn_readfirstlane(t);
}

// GA items taken per ticket: the counter is hit once per chunk
constexpr int kGaChunk = 16;

// One GA generation `gen` (>= 1), item = run slot * pop + individual:
// individual 0 keeps the previous best, the others are tournament /
// crossover / mutation children, evaluated.
template <int CAP>
__device__ __forceinline__ void ga_item(const EvalConst &C, const DockArgs &D, int gen, int item, EvalLds<CAP> &S) {
  const int lane = threadIdx.x;
  const int R = D.run_order[item / D.pop];
  if (D.active && !D.active[R]) return;   // the run has stopped
  const int i = item % D.pop;
  const int li = R / D.nrun, run = R % D.nrun;
  const int src = (gen - 1) & 1, dst = gen & 1;
  const float *oldG = D.geno + pop_off(D, src, R) * kStride;
  const float *oldE = D.energy + pop_off(D, src, R);
  float *newG = D.geno + pop_off(D, dst, R) * kStride;
  float *newE = D.energy + pop_off(D, dst, R);
  if (i == 0) {
    const int b = wave_argmin(oldE, D.pop, lane);
    if (lane < kStride) newG[lane] = oldG[(size_t)b * kStride + lane];
    if (lane == 0) newE[0] = oldE[b];
    return;
  }
  LaneLig<CAP> LL;
  LL.load(C, D.lig_map ? D.lig_map[li] : li, lane);
  const int T = LL.L.n_tor;
  const Rng rng{D.k0, D.k1, D.lig_id[li], (uint32_t)run, (uint32_t)gen};
  const uint4 s0 = rng.block(i, kStSelect, 0), s1 = rng.block(i, kStSelect, 1);
  const int A = tournament(oldE, D.pop, D.tour_p, s0.x, s0.y, s0.z);
  const int B = tournament(oldE, D.pop, D.tour_p, s0.w, s1.x, s1.y);
  // two-point crossover over gene blocks {t, q, theta_0..theta_{T-1}}
  const uint4 cx = rng.block(i, kStCross, 0);
  const int nb = 2 + T;
  int lo = 1, hi = 0;   // empty range
  if (unif(cx.x) < D.cx_rate) {
    const int c1 = (int)randint(cx.y, (uint32_t)nb), c2 = (int)randint(cx.z, (uint32_t)nb);
    lo = min(c1, c2);
    hi = max(c1, c2);
  }
  const int blk = lane < 3 ? 0 : (lane < 7 ? 1 : 2 + (lane - 7));
  const bool fromB = blk >= lo && blk <= hi;
  double gene = lane < kStride ? (double)(fromB ? oldG[(size_t)B * kStride + lane] : oldG[(size_t)A * kStride + lane])
                               : 0.0;
  // mutation: slot s uses Philox block s of the mutation stream
  const uint4 mo = rng.block(i, kStMutate, 3);   // orientation slot
  if (unif(mo.x) < D.mut_rate) {
    const double PI = 3.14159265358979323846;
    const double z = 2.0 * unif(mo.y) - 1.0, phi = 2.0 * PI * unif(mo.z), rho = sqrt(1.0 - z * z);
    const double ang = (2.0 * unif(mo.w) - 1.0) * D.mut_rot;
    double sp, cp;
    sincos(phi, &sp, &cp);
    Q4 q = {__shfl(gene, 3), __shfl(gene, 4), __shfl(gene, 5), __shfl(gene, 6)};
    Q4 qn = apply_rotvec(q, ang * rho * cp, ang * rho * sp, ang * z);
    if (lane == 3) gene = qn.w;
    if (lane == 4) gene = qn.x;
    if (lane == 5) gene = qn.y;
    if (lane == 6) gene = qn.z;
  }
  if (lane < 3 || (lane >= 7 && lane < 7 + T)) {
    const int slot = lane < 3 ? lane : 4 + (lane - 7);
    const uint4 m = rng.block(i, kStMutate, slot);
    if (unif(m.x) < D.mut_rate) {
      const double d = 2.0 * unif(m.y) - 1.0;
      gene = lane < 3 ? gene + d * D.mut_t : wrap_angle(gene + d * D.mut_theta);
    }
  }
  const float g = round_gene(gene);
  if (lane < kStride) S.geno[lane] = (double)g;
  __syncthreads();
  const double E = evaluate<CAP, false, false, 64, kMaxTor, 2>(C, LL, S, lane, nullptr, nullptr);
  if (lane < kStride) newG[(size_t)i * kStride + lane] = g;
  if (lane == 0) {
    newE[i] = (float)E;
    atomicAdd(&D.evals[R], 1ull);
  }
}

template <int CAP, bool QUEUE>
__global__ __launch_bounds__(64) void k_ga_generation(EvalConst C, DockArgs D, int gen) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  if (!QUEUE) {
    ga_item<CAP>(C, D, gen, (int)blockIdx.x, S);
    return;
  }
  const int n_items = D.n_launch * D.pop;
  for (int t = next_ticket(D.q_ga + gen); t * kGaChunk < n_items; t = next_ticket(D.q_ga + gen)) {
    const int end = min(n_items, (t + 1) * kGaChunk);
    for (int item = t * kGaChunk; item < end; ++item) {
      ga_item<CAP>(C, D, gen, item, S);
      __syncthreads();
    }
  }
}

// ADADELTA for small ligands (at most kDualAtoms atoms and kDualTor
// torsions): two individuals per wavefront, one per half of 32 lanes
// (atoms, torsions and degrees of freedom on lanes, pairs strided by 32),
// each half with its own LDS.  The halves take individuals of one ligand:
// the packed part of a bucket's run order holds whole ligands (nrun
// consecutive runs each), and work-group w of a ligand takes its items 2w
// and 2w + 1 (item = run slot * n_ls + pick).  A half without an item (odd
// item count) or whose run has stopped computes on a valid individual and
// writes nothing, so both halves pass the same barriers.  `wg` numbers the
// packed work-groups; dynamic LDS: 2 * pop ints (each half's pick
// permutation).
template <int UNROLL>
__device__ __forceinline__ void ls_dual(const EvalConst &C, const DockArgs &D, int gen, int wg,
                                        EvalLds<kDualAtoms, kDualTor> *S2) {
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  const int half = threadIdx.x >> 5, lane = threadIdx.x & 31;
  EvalLds<kDualAtoms, kDualTor> &S = S2[half];
  init_eval_lds(S, lane);
  static_assert(sizeof(S.tm) >= kPermAlias * sizeof(int), "pick permutation alias");
  int *perm = perm_aliased(D.pop, 0) ? reinterpret_cast<int *>(&S.tm[0][0])
                                     : reinterpret_cast<int *>(dyn_lds) + half * D.pop;
  const int items = D.nrun * D.n_ls;
  const int wpl = (items + 1) >> 1;   // work-groups per ligand
  const int chunk = wg / wpl;
  const int k = (wg - chunk * wpl) * 2 + half;
  const int li = D.run_order[chunk * D.nrun] / D.nrun;   // the chunk's ligand (uniform)
  bool live = k < items;
  const int run_slot = live ? k / D.n_ls : 0;
  const int slot = live ? k - run_slot * D.n_ls : 0;
  const int R = D.run_order[chunk * D.nrun + run_slot];
  if (D.active && !D.active[R]) live = false;
  if (__ballot(live) == 0) return;   // both halves idle (stopped runs): nothing to compute
  const int run = R % D.nrun;
  const int m = D.pop - 1;
  for (int j = lane; j < m; j += 32) perm[j] = j + 1;
  __syncthreads();
  const Rng rng{D.k0, D.k1, D.lig_id[li], (uint32_t)run, (uint32_t)gen};
  if (lane == 0 && live) {
    for (int s = 0; s <= slot; ++s) {
      const int r = s + (int)randint(rng.word(0, kStLsPick, s), (uint32_t)(m - s));
      const int t = perm[s];
      perm[s] = perm[r];
      perm[r] = t;
    }
  }
  __syncthreads();
  const int indiv = perm[slot];
  LaneLig<kDualAtoms> LL;
  LL.load(C, D.lig_map ? D.lig_map[li] : li, lane);
  const size_t off = pop_off(D, gen & 1, R) + indiv;
  adadelta_wave<kDualAtoms, false, 32, kDualTor, UNROLL>(C, LL, S, lane, D.geno + off * kStride, D.energy + off,
                                                         D.ls_iters,
                                                 D.rho, D.eps, PairStage{0, 0}, half, live);
  if (lane == 0 && live) atomicAdd(&D.evals[R], (unsigned long long)D.ls_iters);
}

// ADADELTA on the individuals picked for generation `gen`: n_ls distinct
// indices from 1..pop-1 by a partial Fisher-Yates shuffle (word s of the
// pick stream draws the partner of position s).  Item = run slot * n_ls +
// pick, over the bucket's one-wavefront runs (those after the packed ones).
// With STAGE the first D.stage_pairs pair records of the ligand and the
// type-pair table are copied to LDS once and read from there by all
// ls_iters evaluations (the results are bitwise the same either way).
// Dynamic LDS: pop ints (the pick permutation), then the staged records.
template <int CAP, bool STAGE, int UNROLL>
__device__ __forceinline__ void ls_single(const EvalConst &C, const DockArgs &D, int gen, int item, EvalLds<CAP> &S) {
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  static_assert(sizeof(S.tm) >= kPermAlias * sizeof(int), "pick permutation alias");
  int *perm = !STAGE && perm_aliased(D.pop, 0) ? reinterpret_cast<int *>(&S.tm[0][0])
                                               : reinterpret_cast<int *>(dyn_lds);
  const int lane = threadIdx.x;
  const int R = D.run_order[D.n_dual + item / D.n_ls];
  if (D.active && !D.active[R]) return;
  init_eval_lds(S, lane);
  const int slot = item % D.n_ls;
  const int li = R / D.nrun, run = R % D.nrun;
  const int m = D.pop - 1;
  for (int j = lane; j < m; j += 64) perm[j] = j + 1;
  __syncthreads();
  const Rng rng{D.k0, D.k1, D.lig_id[li], (uint32_t)run, (uint32_t)gen};
  if (lane == 0) {
    for (int s = 0; s <= slot; ++s) {
      const int r = s + (int)randint(rng.word(0, kStLsPick, s), (uint32_t)(m - s));
      const int t = perm[s];
      perm[s] = perm[r];
      perm[r] = t;
    }
  }
  __syncthreads();
  const int indiv = perm[slot];
  LaneLig<CAP> LL;
  LL.load(C, D.lig_map ? D.lig_map[li] : li, lane);
  PairStage st{0, 0};
  if (STAGE) {
    st.off = stage_offset(D.pop);
    st.n = min(LL.L.n_pairs, D.stage_pairs);
    const int ntt = C.ff.n_types * C.ff.n_types;
    LJRec *s_lj = reinterpret_cast<LJRec *>(dyn_lds + st.off);
    PairRec *s_pr = reinterpret_cast<PairRec *>(dyn_lds + st.off + ntt * 16);
    for (int k = lane; k < ntt; k += 64) s_lj[k] = C.batch.lj[k];
    const PairRec *src = C.batch.pairs + LL.L.pair_off;
    for (int k = lane; k < st.n; k += 64) s_pr[k] = src[k];
    __syncthreads();
  }
  const size_t off = pop_off(D, gen & 1, R) + indiv;
  adadelta_wave<CAP, STAGE, 64, kMaxTor, UNROLL>(C, LL, S, lane, D.geno + off * kStride, D.energy + off, D.ls_iters,
                                                 D.rho, D.eps, st);
  if (lane == 0) atomicAdd(&D.evals[R], (unsigned long long)D.ls_iters);
}

// One launch covers the bucket's one-wavefront items, then (64-atom variant
// without staging) the packed work-groups of ls_dual, one item each; both
// kinds share one static LDS block.
template <int CAP, bool STAGE, int UNROLL = 1, bool QUEUE = false>
__global__ __launch_bounds__(64) void k_ls_generation(EvalConst C, DockArgs D, int gen) {
  constexpr bool kPack = CAP == 64 && !STAGE;
  constexpr size_t kOne = sizeof(EvalLds<CAP>), kTwo = 2 * sizeof(EvalLds<kDualAtoms, kDualTor>);
  __shared__ __attribute__((aligned(16))) char lds[kPack && kTwo > kOne ? kTwo : kOne];
  const int n_single = (D.n_launch - D.n_dual) * D.n_ls;
  auto run_item = [&](int item) {
    if (kPack && item >= n_single)
      ls_dual<UNROLL>(C, D, gen, item - n_single, reinterpret_cast<EvalLds<kDualAtoms, kDualTor> *>(lds));
    else
      ls_single<CAP, STAGE, UNROLL>(C, D, gen, item, *reinterpret_cast<EvalLds<CAP> *>(lds));
  };
  if (!QUEUE) {
    run_item((int)blockIdx.x);
    return;
  }
  const int n_items = n_single + (kPack ? (D.n_dual / D.nrun) * ((D.nrun * D.n_ls + 1) / 2) : 0);
  for (int t = next_ticket(D.q_ls + gen); t < n_items; t = next_ticket(D.q_ls + gen)) {
    run_item(t);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Solis-Wets local search: one wavefront per individual, energy-only
// evaluations.  Degrees of freedom on lanes as in ADADELTA (0-2
// translation, 3-5 rotation vector, 7.. torsions; DOF index k = lane for
// lane < 6, lane - 1 above).  Deviates: Philox with key (seed lo, seed hi ^
// 0x9E3779B9), counter (ligand id, run, gen << 16 | individual, it << 8 |
// k / 2); Box-Muller from words 0, 1 (cosine branch for even k, sine for
// odd), evaluated in FP32.  Only improvements are accepted.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float sw_normal(uint32_t k0, uint32_t k1, uint32_t lig, uint32_t run, uint32_t gen,
                                           uint32_t indiv, uint32_t it, int k) {
  const uint4 w = philox(make_uint4(lig, run, (gen << 16) | indiv, (it << 8) | (uint32_t)(k >> 1)), k0,
                         k1 ^ 0x9E3779B9u);
  const float u1 = (float)((w.x >> 8) + 1) * (1.0f / 16777216.0f);
  const float u2 = (float)(w.y >> 8) * (1.0f / 16777216.0f);
  const float r = __builtin_sqrtf(-2.0f * 0.69314718055994531f * __builtin_amdgcn_logf(u1));
  float sn, cs;
  __sincosf(6.2831853071795865f * u2, &sn, &cs);
  return (k & 1) ? r * sn : r * cs;
}

// gene of this lane after moving by sgn * (b + d) (rotation lanes combine
// the three rotation-vector components into a quaternion update)
__device__ __forceinline__ float sw_moved(float gene, float step, float sgn, int lane, int T) {
  const float st = sgn * step;
  const float w0 = lane_f32(st, 3), w1 = lane_f32(st, 4), w2 = lane_f32(st, 5);
  const float qw = lane_f32(gene, 3), qx = lane_f32(gene, 4), qy = lane_f32(gene, 5), qz = lane_f32(gene, 6);
  const float th = __builtin_sqrtf(w0 * w0 + w1 * w1 + w2 * w2);
  float sh, ch;
  __sincosf(0.5f * th, &sh, &ch);
  const float f = th > 1e-30f ? sh / th : 0.5f;
  const float rx = f * w0, ry = f * w1, rz = f * w2;
  const float nw = ch * qw - rx * qx - ry * qy - rz * qz;
  const float nx = ch * qx + rx * qw + ry * qz - rz * qy;
  const float ny = ch * qy - rx * qz + ry * qw + rz * qx;
  const float nz = ch * qz + rx * qy - ry * qx + rz * qw;
  const float inv = fast_rsq(nw * nw + nx * nx + ny * ny + nz * nz);
  if (lane < 3) return gene + st;
  if (lane == 3) return nw * inv;
  if (lane == 4) return nx * inv;
  if (lane == 5) return ny * inv;
  if (lane == 6) return nz * inv;
  if (lane < 7 + T) {
    float th2 = gene + st;
    th2 -= 6.2831853071795865f * floorf((th2 + 3.14159265358979f) * 0.15915494309189535f);
    return th2;
  }
  return gene;
}

template <int CAP>
__device__ int sw_wave(const EvalConst &C, const LaneLig<CAP> &LL, EvalLds<CAP> &S, int lane, float *geno_io,
                       float *E_io, const DockArgs &D, uint32_t lig_id, uint32_t run, uint32_t gen, uint32_t indiv) {
  const int T = LL.L.n_tor;
  const bool dof = lane < 6 || (lane >= 7 && lane < 7 + T);
  const int k = lane < 6 ? lane : lane - 1;
  const float sig = lane < 3 ? D.sw_sig_t : D.sw_sig_ang;
  float gene = lane < kStride ? geno_io[lane] : 0.0f;
  double Ex = (double)*E_io;
  float b = 0.0f, rho = D.sw_rho;
  int succ = 0, fail = 0, ev = 0;
  for (uint32_t it = 0; ev < D.ls_iters && rho >= D.sw_rho_lb; ++it) {
    const float dv = dof ? rho * sig * sw_normal(D.k0, D.k1, lig_id, run, gen, indiv, it, k) : 0.0f;
    const float step = b + dv;
    bool ok = false;
    float cand = sw_moved(gene, step, 1.0f, lane, T);
    if (lane < kStride) S.geno[lane] = (double)cand;
    __syncthreads();
    double E = evaluate<CAP, false, false, 64, kMaxTor, 2>(C, LL, S, lane, nullptr, nullptr);
    ++ev;
    if (E < Ex) {
      gene = cand;
      Ex = E;
      b = 0.2f * b + 0.4f * dv;
      ok = true;
    } else if (ev < D.ls_iters) {
      cand = sw_moved(gene, step, -1.0f, lane, T);
      __syncthreads();
      if (lane < kStride) S.geno[lane] = (double)cand;
      __syncthreads();
      E = evaluate<CAP, false, false, 64, kMaxTor, 2>(C, LL, S, lane, nullptr, nullptr);
      ++ev;
      if (E < Ex) {
        gene = cand;
        Ex = E;
        b = b - 0.4f * dv;
        ok = true;
      }
    }
    if (ok) {
      ++succ;
      fail = 0;
    } else {
      b *= 0.5f;
      ++fail;
      succ = 0;
    }
    if (succ >= D.sw_max_succ) {
      rho *= 2.0f;
      succ = 0;
    } else if (fail >= D.sw_max_fail) {
      rho *= 0.5f;
      fail = 0;
    }
    __syncthreads();
  }
  if (lane < kStride) geno_io[lane] = gene;
  if (lane == 0) *E_io = (float)Ex;
  return ev;
}

// Solis-Wets on the individuals picked for generation `gen` (same picks as
// the ADADELTA generation kernel).  Dynamic LDS: pop ints.
template <int CAP>
__global__ __launch_bounds__(64) void k_sw_generation(EvalConst C, DockArgs D, int gen) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
  int *perm = reinterpret_cast<int *>(dyn_lds);
  const int lane = threadIdx.x;
  const int R = D.run_order[blockIdx.x / D.n_ls];
  if (D.active && !D.active[R]) return;
  const int slot = blockIdx.x % D.n_ls;
  const int li = R / D.nrun, run = R % D.nrun;
  const int m = D.pop - 1;
  for (int j = lane; j < m; j += 64) perm[j] = j + 1;
  __syncthreads();
  const Rng rng{D.k0, D.k1, D.lig_id[li], (uint32_t)run, (uint32_t)gen};
  if (lane == 0) {
    for (int s2 = 0; s2 <= slot; ++s2) {
      const int r = s2 + (int)randint(rng.word(0, kStLsPick, s2), (uint32_t)(m - s2));
      const int t = perm[s2];
      perm[s2] = perm[r];
      perm[r] = t;
    }
  }
  __syncthreads();
  const int indiv = perm[slot];
  LaneLig<CAP> LL;
  LL.load(C, D.lig_map ? D.lig_map[li] : li, lane);
  const size_t off = pop_off(D, gen & 1, R) + indiv;
  const int used = sw_wave<CAP>(C, LL, S, lane, D.geno + off * kStride, D.energy + off, D, D.lig_id[li],
                                (uint32_t)run, (uint32_t)gen, (uint32_t)indiv);
  if (lane == 0) atomicAdd(&D.evals[R], (unsigned long long)used);
}

// Standalone Solis-Wets on given poses (ad_solis_wets): the start energy is
// evaluated first (one evaluation), then D.ls_iters - 1 more at most.
// Random streams: ligand id = batch index, run 0, generation 0, individual =
// pose index.
template <int CAP>
__global__ __launch_bounds__(64) void k_solis_wets(EvalConst C, DockArgs D, int n, const int *__restrict__ lig_idx,
                                                   float *__restrict__ geno, float *__restrict__ E,
                                                   int *__restrict__ used) {
  __shared__ EvalLds<CAP> S;
  init_eval_lds(S, threadIdx.x);
  const int p = blockIdx.x;
  const int lane = threadIdx.x;
  const int li = lig_idx[p];
  if (li < 0 || li >= C.batch.n_lig || C.batch.lig[li].n_atoms > CAP) {
    if (lane == 0) {
      E[p] = __builtin_nanf("");
      used[p] = 0;
    }
    return;
  }
  LaneLig<CAP> LL;
  LL.load(C, li, lane);
  float *g = geno + (size_t)p * kStride;
  if (D.ls_iters <= 0) {
    if (lane == 0) {
      E[p] = __builtin_nanf("");
      used[p] = 0;
    }
    return;
  }
  if (lane < kStride) S.geno[lane] = (double)g[lane];
  __syncthreads();
  const double E0 = evaluate<CAP, false, false, 64, kMaxTor, 2>(C, LL, S, lane, nullptr, nullptr);
  __syncthreads();
  if (lane == 0) E[p] = (float)E0;
  __syncthreads();
  DockArgs Dp = D;
  Dp.ls_iters = D.ls_iters - 1;
  const int u = sw_wave<CAP>(C, LL, S, lane, g, E + p, Dp, (uint32_t)li, 0u, 0u, (uint32_t)p);
  if (lane == 0) used[p] = u + 1;
}

// After generation `gen` (0: the initial population): record each active
// run's best energy, then decide whether it takes generation gen + 1 --
// not beyond max_gens, not if the most the next generation can cost would
// pass max_evals, and with autostop not once ten recorded best energies
// have a standard deviation below stop_std.  One wavefront per run.
__global__ __launch_bounds__(64) void k_run_status(DockArgs D, int gen) {
  const int lane = threadIdx.x;
  const int R = blockIdx.x;
  if (!D.active[R]) return;
  const float *E = D.energy + pop_off(D, gen & 1, R);
  const int b = wave_argmin(E, D.pop, lane);
  if (lane != 0) return;
  float *h = D.hist + (size_t)R * 10;
  h[gen % 10] = E[b];
  D.last_gen[R] = gen;
  bool go = gen + 1 <= D.max_gens && (long long)D.evals[R] + D.max_gen_cost <= D.max_evals;
  if (go && D.autostop && gen + 1 >= 10) {
    double m = 0.0, v = 0.0;
    for (int k = 0; k < 10; ++k) m += (double)h[k];
    m /= 10.0;
    for (int k = 0; k < 10; ++k) v += ((double)h[k] - m) * ((double)h[k] - m);
    if (sqrt(v / 10.0) < D.stop_std) go = false;
  }
  if (go) atomicAdd(&D.n_active[gen], 1);
  else D.active[R] = 0u;
}

// Best individual of every run after the last generation (with per-run
// stopping: after the run's own last generation).
__global__ __launch_bounds__(64) void k_finalize(DockArgs D, int buf_all, float *best_E, float *best_G) {
  const int lane = threadIdx.x;
  const int R = blockIdx.x;
  const int buf = D.last_gen ? (D.last_gen[R] & 1) : buf_all;
  const float *E = D.energy + pop_off(D, buf, R);
  const int b = wave_argmin(E, D.pop, lane);
  if (lane < kStride) best_G[(size_t)R * kStride + lane] = D.geno[(pop_off(D, buf, R) + b) * kStride + lane];
  if (lane == 0) best_E[R] = E[b];
}

// Generation-0 genotypes only (diagnostics).
__global__ __launch_bounds__(64) void k_init_genotypes(GridArgs G, int n_tor, uint32_t k0, uint32_t k1,
                                                       uint32_t lig_id, int run, float *out) {
  const int lane = threadIdx.x, i = blockIdx.x;
  const Rng rng{k0, k1, lig_id, (uint32_t)run, 0u};
  const float g = (float)init_gene(G, rng, i, lane, n_tor);
  if (lane < kStride) out[(size_t)i * kStride + lane] = g;
}

// ---------------------------------------------------------------------------
// Grid maps: one thread per node, receptor atoms staged through LDS.  FP64.
// Writes the float4 resident layout and, optionally, the SoA layout.
// ---------------------------------------------------------------------------
constexpr int kMapTile = 256;

__global__ __launch_bounds__(256) void k_build_maps(const MapBuildArgs *__restrict__ Ap) {
  const MapBuildArgs &A = *Ap;
  __shared__ double sx[kMapTile], sy[kMapTile], sz[kMapTile], sq[kMapTile];
  __shared__ int st[kMapTile];
  const size_t nn = (size_t)A.nx * A.ny * A.nz;
  const size_t node = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = node < nn;
  const int i = active ? (int)(node % A.nx) : 0;
  const int j = active ? (int)((node / A.nx) % A.ny) : 0;
  const int k = active ? (int)(node / ((size_t)A.nx * A.ny)) : 0;
  const double px = A.ox + A.h * i, py = A.oy + A.h * j, pz = A.oz + A.h * k;
  double aff[kMaxTypes];
  for (int m = 0; m < kMaxTypes; ++m) aff[m] = 0.0;
  double elec = 0.0, desolv = 0.0;
  for (int base = 0; base < A.n_rec; base += kMapTile) {
    __syncthreads();
    const int a = base + threadIdx.x;
    if (a < A.n_rec) {
      sx[threadIdx.x] = A.rec_xyz[3 * a];
      sy[threadIdx.x] = A.rec_xyz[3 * a + 1];
      sz[threadIdx.x] = A.rec_xyz[3 * a + 2];
      sq[threadIdx.x] = A.rec_q[a];
      st[threadIdx.x] = A.rec_type[a];
    }
    __syncthreads();
    const int cnt = min(kMapTile, A.n_rec - base);
    for (int b = 0; b < cnt; ++b) {
      const double dx = px - sx[b], dy = py - sy[b], dz = pz - sz[b];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double r = sqrt(r2);
      const double rf = r < A.r_floor ? A.r_floor : r;
      const int ta = st[b];
      const double qa = sq[b];
      // electrostatics over all atoms
      const double e = exp(-A.diel_lB * rf);
      const double den = 1.0 + A.diel_k * e;
      const double eps = A.diel_A + A.diel_B / den;
      elec += A.w_el_ke * qa / (eps * rf);
      if (r2 < A.cutoff2) {
        const double gds = exp(-rf * rf / A.two_s2);
        const double Sa = A.solpar[ta] + A.qasp * fabs(qa);
        desolv += A.w_sol * A.qasp * A.vol[ta] * gds;
        for (int m = 0; m < A.n_maps; ++m) {
          const int t = A.map_type[m];
          const double r0 = A.r0[t][ta];
          double rr;
          if (rf > r0 + A.half_smooth) rr = rf - A.half_smooth;
          else if (rf < r0 - A.half_smooth) rr = rf + A.half_smooth;
          else rr = r0;
          const double inv = 1.0 / rr, i2 = inv * inv, i6 = i2 * i2 * i2;
          const double im = A.hb[t][ta] ? i6 * i2 * i2 : i6;
          aff[m] += A.A[t][ta] * i6 * i6 - A.B[t][ta] * im + A.w_sol * (A.solpar[t] * A.vol[ta] + Sa * A.vol[t]) * gds;
        }
      }
    }
  }
  if (!active) return;
  for (int m = 0; m < A.n_maps; ++m) {
    const float v = (float)fmin(aff[m], A.cap);
    float4 rec = make_float4(v, (float)elec, (float)desolv, 0.0f);
    reinterpret_cast<float4 *>(A.out4)[(size_t)m * nn + node] = rec;
    if (A.soa) A.soa[(size_t)m * nn + node] = v;
  }
  if (A.soa) {
    A.soa[(size_t)A.n_maps * nn + node] = (float)elec;
    A.soa[(size_t)(A.n_maps + 1) * nn + node] = (float)desolv;
  }
}

// SoA [n_maps+2][nodes] -> float4 per (map, node).
__global__ void k_relayout(const float *__restrict__ soa, float *__restrict__ out4, size_t nn, int n_maps) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * n_maps) return;
  const size_t m = idx / nn, node = idx % nn;
  float4 r = make_float4(soa[m * nn + node], soa[(size_t)n_maps * nn + node], soa[(size_t)(n_maps + 1) * nn + node],
                         0.0f);
  reinterpret_cast<float4 *>(out4)[idx] = r;
}

// ---------------------------------------------------------------------------
// launch wrappers (called by the C-ABI layer)
// ---------------------------------------------------------------------------
hipError_t launch_score(const EvalConst &C, int cap, int n, const int *lig_idx, const float *geno, float *E, float *G,
                        float *T, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(n), block(64);
  if (cap <= 32) {   // packed: two poses per wavefront
    const dim3 g2((n + 1) / 2);
    if (G) hipLaunchKernelGGL((k_score_dual<true>), g2, block, 0, s, C, n, lig_idx, geno, E, G, T);
    else hipLaunchKernelGGL((k_score_dual<false>), g2, block, 0, s, C, n, lig_idx, geno, E, G, T);
  } else if (cap <= 64) {
    if (G) hipLaunchKernelGGL((k_score<64, true>), grid, block, 0, s, C, n, lig_idx, geno, E, G, T);
    else hipLaunchKernelGGL((k_score<64, false>), grid, block, 0, s, C, n, lig_idx, geno, E, G, T);
  } else {
    if (G) hipLaunchKernelGGL((k_score<128, true>), grid, block, 0, s, C, n, lig_idx, geno, E, G, T);
    else hipLaunchKernelGGL((k_score<128, false>), grid, block, 0, s, C, n, lig_idx, geno, E, G, T);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static staging block of ad_score_poses_noalloc: index, genotype, energy,
// gradient and terms sections for up to kNoAllocPoses poses at fixed
// offsets.  Each device that loads the library holds its own copy until the
// process ends.  Host code never uses the array's name as an address: its
// device address is taken once per device (noalloc_scratch_init, called by
// ad_create with that device current) and every copy or kernel argument
// uses that address.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kNoAllocDevices];

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void *noalloc_scratch(int device) {
  if (device < 0 || device >= kNoAllocDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_local_search(const EvalConst &C, int cap, int n, const int *lig_idx, float *geno, float *E,
                               int iters, double rho, double eps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(n), block(64);
  if (cap <= 32) {
    hipLaunchKernelGGL(k_local_search_dual, dim3((n + 1) / 2), block, 0, s, C, n, lig_idx, geno, E, iters, rho, eps);
  } else if (cap <= 64) {
    hipLaunchKernelGGL((k_local_search<64>), grid, block, 0, s, C, n, lig_idx, geno, E, iters, rho, eps);
  } else {
    hipLaunchKernelGGL((k_local_search<128>), grid, block, 0, s, C, n, lig_idx, geno, E, iters, rho, eps);
  }
  return hipGetLastError();
}

hipError_t launch_build_maps(const MapBuildArgs *dev_args, size_t nn, hipStream_t s) {
  dim3 grid((unsigned)((nn + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_build_maps, grid, block, 0, s, dev_args);
  return hipGetLastError();
}

hipError_t launch_relayout(const float *soa, float *out4, size_t nn, int n_maps, hipStream_t s) {
  size_t total = nn * n_maps;
  dim3 grid((unsigned)((total + 255) / 256)), block(256);
  hipLaunchKernelGGL(k_relayout, grid, block, 0, s, soa, out4, nn, n_maps);
  return hipGetLastError();
}


// A 1-D grid holds fewer than 2^31 work-items: very large batches are
// launched in chunks of runs (the kernels find their run through run_order).
template <typename F>
hipError_t for_run_chunks(const DockArgs &D, int blocks_per_run, F launch) {
  const long long max_blocks = ((1LL << 31) - 64) / 64;
  const int step = (int)std::max(1LL, max_blocks / std::max(1, blocks_per_run));
  for (int r0 = 0; r0 < D.n_launch; r0 += step) {
    DockArgs Dc = D;
    Dc.run_order = D.run_order + r0;
    Dc.n_launch = std::min(step, D.n_launch - r0);
    launch(Dc, dim3((unsigned)((long long)Dc.n_launch * blocks_per_run)));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_dock_init(const EvalConst &C, int cap, const DockArgs &D, hipStream_t s) {
  if (D.n_launch <= 0) return hipSuccess;
  return for_run_chunks(D, D.pop, [&](const DockArgs &Dc, dim3 grid) {
    if (cap <= 64) hipLaunchKernelGGL((k_init_pop<64>), grid, dim3(64), 0, s, C, Dc);
    else hipLaunchKernelGGL((k_init_pop<128>), grid, dim3(64), 0, s, C, Dc);
  });
}

hipError_t launch_ga_generation(const EvalConst &C, int cap, const DockArgs &D, int gen, hipStream_t s) {
  if (D.n_launch <= 0) return hipSuccess;
  if (D.q_ga) {
    const long long chunks = ((long long)D.n_launch * D.pop + kGaChunk - 1) / kGaChunk;
    const dim3 grid((unsigned)std::max(1LL, std::min(chunks, (long long)D.q_grid_ga)));
    if (cap <= 64) hipLaunchKernelGGL((k_ga_generation<64, true>), grid, dim3(64), 0, s, C, D, gen);
    else hipLaunchKernelGGL((k_ga_generation<128, true>), grid, dim3(64), 0, s, C, D, gen);
    return hipGetLastError();
  }
  return for_run_chunks(D, D.pop, [&](const DockArgs &Dc, dim3 grid) {
    if (cap <= 64) hipLaunchKernelGGL((k_ga_generation<64, false>), grid, dim3(64), 0, s, C, Dc, gen);
    else hipLaunchKernelGGL((k_ga_generation<128, false>), grid, dim3(64), 0, s, C, Dc, gen);
  });
}

size_t ls_dynamic_lds(const EvalConst &C, const DockArgs &D) {
  if (D.stage_pairs <= 0) return perm_aliased(D.pop, 0) ? 0 : (size_t)D.pop * sizeof(int);
  return (size_t)stage_offset(D.pop) + (size_t)C.ff.n_types * C.ff.n_types * 16 + (size_t)D.stage_pairs * 16;
}

size_t ls_workgroup_lds(const EvalConst &C, int cap, const DockArgs &D) {
  if (cap <= 64) {
    const size_t one = sizeof(EvalLds<64>), two = 2 * sizeof(EvalLds<kDualAtoms, kDualTor>);
    const bool packed = D.ls_method == 0 && D.n_dual > 0 && D.stage_pairs <= 0;
    return (D.stage_pairs > 0 ? one : std::max(one, two)) +
           (packed ? (perm_aliased(D.pop, 0) ? 0 : 2 * (size_t)D.pop * sizeof(int)) : ls_dynamic_lds(C, D));
  }
  return sizeof(EvalLds<128>) + ls_dynamic_lds(C, D);
}

// the local-search kernel of a bucket with the launch shape's pair-loop
// unroll, queued (D.q_ls set) or one work-group per item
template <int CAP, bool STAGE, bool QUEUE>
const void *ls_kernel_ptr(int unroll) {
  if constexpr (!STAGE)   // staged pair records keep the plain loop
    if (unroll == 2) return reinterpret_cast<const void *>(&k_ls_generation<CAP, false, 2, QUEUE>);
  return reinterpret_cast<const void *>(&k_ls_generation<CAP, STAGE, 1, QUEUE>);
}

template <int CAP, bool STAGE, bool QUEUE>
void launch_ls_variant(int unroll, dim3 grid, size_t dyn, hipStream_t s, const EvalConst &C, const DockArgs &D,
                       int gen) {
  if constexpr (!STAGE) {
    if (unroll == 2) {
      hipLaunchKernelGGL((k_ls_generation<CAP, false, 2, QUEUE>), grid, dim3(64), dyn, s, C, D, gen);
      return;
    }
  }
  hipLaunchKernelGGL((k_ls_generation<CAP, STAGE, 1, QUEUE>), grid, dim3(64), dyn, s, C, D, gen);
}

template <int CAP, bool STAGE>
void launch_ls_kernel(int unroll, dim3 grid, size_t dyn, hipStream_t s, const EvalConst &C, const DockArgs &D,
                      int gen) {
  if (D.q_ls) launch_ls_variant<CAP, STAGE, true>(unroll, grid, dyn, s, C, D, gen);
  else launch_ls_variant<CAP, STAGE, false>(unroll, grid, dyn, s, C, D, gen);
}

// the bucket's ADADELTA local-search launch: packed work-groups in it, its
// dynamic LDS (with the occupancy pad) and its item count
struct LsLaunch {
  bool packed, stage;
  size_t dyn;
  long long n_items;
};
LsLaunch ls_launch_of(const EvalConst &C, int cap, const DockArgs &D) {
  LsLaunch L;
  const size_t pad = (size_t)std::max(0, D.ls_pad);
  L.packed = cap <= 64 && D.n_dual > 0 && D.stage_pairs <= 0;
  L.stage = D.stage_pairs > 0;
  if (L.packed) {
    L.dyn = (perm_aliased(D.pop, 0) ? 0 : 2 * (size_t)D.pop * sizeof(int)) + pad;
    L.n_items = (long long)(D.n_launch - D.n_dual) * D.n_ls + (long long)(D.n_dual / D.nrun) * ((D.nrun * D.n_ls + 1) / 2);
  } else {
    DockArgs t = D;
    t.n_dual = 0;
    L.dyn = ls_dynamic_lds(C, t) + pad;
    L.n_items = (long long)D.n_launch * D.n_ls;
  }
  return L;
}

int queue_grid(const EvalConst &C, int cap, const DockArgs &D, int kind) {
  int dev = 0, n_cu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const void *k;
  size_t dyn = 0;
  if (kind == 0) {
    k = cap <= 64 ? reinterpret_cast<const void *>(&k_ga_generation<64, true>)
                  : reinterpret_cast<const void *>(&k_ga_generation<128, true>);
  } else {
    const LsLaunch L = ls_launch_of(C, cap, D);
    dyn = L.dyn;
    if (cap <= 64)
      k = L.stage ? ls_kernel_ptr<64, true, true>(D.ls_unroll) : ls_kernel_ptr<64, false, true>(D.ls_unroll);
    else
      k = L.stage ? ls_kernel_ptr<128, true, true>(D.ls_unroll) : ls_kernel_ptr<128, false, true>(D.ls_unroll);
  }
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64, dyn) != hipSuccess) return 0;
  return std::max(1, n_cu) * std::max(1, per_cu);
}

hipError_t launch_ls_generation(const EvalConst &C, int cap, const DockArgs &D0, int gen, hipStream_t s) {
  if (D0.n_launch <= 0 || D0.n_ls <= 0) return hipSuccess;
  const dim3 block(64);
  DockArgs D = D0;
  const size_t pad = D0.ls_method == 0 ? (size_t)std::max(0, D0.ls_pad) : 0;
  const int ur = D0.ls_unroll;
  if (D0.q_ls && D0.ls_method == 0) {
    // persistent work-groups over every item of the bucket (queue)
    const LsLaunch L = ls_launch_of(C, cap, D0);
    const dim3 grid((unsigned)std::max(1LL, std::min(L.n_items, (long long)D0.q_grid_ls)));
    DockArgs Dq = D0;
    if (!L.packed) Dq.n_dual = 0;
    if (cap <= 64) {
      if (L.stage) launch_ls_kernel<64, true>(ur, grid, L.dyn, s, C, Dq, gen);
      else launch_ls_kernel<64, false>(ur, grid, L.dyn, s, C, Dq, gen);
    } else {
      if (L.stage) launch_ls_kernel<128, true>(ur, grid, L.dyn, s, C, Dq, gen);
      else launch_ls_kernel<128, false>(ur, grid, L.dyn, s, C, Dq, gen);
    }
    return hipGetLastError();
  }
  D.q_ls = nullptr;
  if (cap <= 64 && D0.ls_method == 0 && D0.n_dual > 0 && D0.stage_pairs <= 0) {
    // packed ligands: ceil(nrun * n_ls / 2) work-groups per ligand, after the
    // single-individual ones in the same launch when the grid allows
    const long long max_blocks = ((1LL << 31) - 64) / 64;
    const long long wpl = (D0.nrun * D0.n_ls + 1) / 2;
    const long long n_chunks = D0.n_dual / D0.nrun;
    const long long n_single = (long long)(D0.n_launch - D0.n_dual) * D0.n_ls;
    const size_t dyn = (perm_aliased(D0.pop, 0) ? 0 : 2 * (size_t)D0.pop * sizeof(int)) + pad;
    if (n_single + n_chunks * wpl <= max_blocks) {
      launch_ls_kernel<64, false>(ur, dim3((unsigned)(n_single + n_chunks * wpl)), dyn, s, C, D0, gen);
      return hipGetLastError();
    }
    DockArgs Ds = D0;
    Ds.run_order = D0.run_order + D0.n_dual;
    Ds.n_launch = D0.n_launch - D0.n_dual;
    Ds.n_dual = 0;
    hipError_t e = Ds.n_launch > 0 ? for_run_chunks(Ds, D0.n_ls, [&](const DockArgs &Dc, dim3 g) {
      launch_ls_kernel<64, false>(ur, g, dyn, s, C, Dc, gen);
    }) : hipSuccess;
    const long long step = std::max(1LL, max_blocks / wpl);
    for (long long c0 = 0; c0 < n_chunks && e == hipSuccess; c0 += step) {
      DockArgs Dc = D0;   // packed work-groups only: n_launch == n_dual
      Dc.run_order = D0.run_order + c0 * D0.nrun;
      Dc.n_dual = Dc.n_launch = (int)(std::min(step, n_chunks - c0) * D0.nrun);
      launch_ls_kernel<64, false>(ur, dim3((unsigned)(Dc.n_dual / D0.nrun * wpl)), dyn, s, C, Dc, gen);
      e = hipGetLastError();
    }
    return e;
  }
  D.n_dual = 0;   // every run takes one wavefront per individual
  const size_t dyn = ls_dynamic_lds(C, D) + pad;
  const bool st = D.stage_pairs > 0;
  return for_run_chunks(D, D.n_ls, [&](const DockArgs &Dc, dim3 lgrid) {
    if (D.ls_method == 1) {
      if (cap <= 64) hipLaunchKernelGGL((k_sw_generation<64>), lgrid, block, (size_t)D.pop * sizeof(int), s, C, Dc, gen);
      else hipLaunchKernelGGL((k_sw_generation<128>), lgrid, block, (size_t)D.pop * sizeof(int), s, C, Dc, gen);
    } else if (cap <= 64) {
      if (st) launch_ls_kernel<64, true>(ur, lgrid, dyn, s, C, Dc, gen);
      else launch_ls_kernel<64, false>(ur, lgrid, dyn, s, C, Dc, gen);
    } else {
      if (st) launch_ls_kernel<128, true>(ur, lgrid, dyn, s, C, Dc, gen);
      else launch_ls_kernel<128, false>(ur, lgrid, dyn, s, C, Dc, gen);
    }
  });
}

hipError_t launch_solis_wets(const EvalConst &C, int cap, const DockArgs &D, int n, const int *lig_idx, float *geno,
                             float *E, int *used, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (cap <= 64) hipLaunchKernelGGL((k_solis_wets<64>), dim3(n), dim3(64), 0, s, C, D, n, lig_idx, geno, E, used);
  else hipLaunchKernelGGL((k_solis_wets<128>), dim3(n), dim3(64), 0, s, C, D, n, lig_idx, geno, E, used);
  return hipGetLastError();
}

hipError_t launch_run_status(const DockArgs &D, int gen, hipStream_t s) {
  hipLaunchKernelGGL(k_run_status, dim3(D.n_runs), dim3(64), 0, s, D, gen);
  return hipGetLastError();
}

hipError_t launch_dock_finalize(const DockArgs &D, int buf, float *best_E, float *best_G, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(D.n_runs), dim3(64), 0, s, D, buf, best_E, best_G);
  return hipGetLastError();
}

hipError_t launch_init_genotypes(const GridArgs &G, int n_tor, uint32_t k0, uint32_t k1, uint32_t lig_id, int run,
                                 int pop, float *out, hipStream_t s) {
  hipLaunchKernelGGL(k_init_genotypes, dim3(pop), dim3(64), 0, s, G, n_tor, k0, k1, lig_id, run, out);
  return hipGetLastError();
}

}  // namespace ad
