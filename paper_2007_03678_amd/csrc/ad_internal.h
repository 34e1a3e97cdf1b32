// Internal data layout of the addock library (host and device).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/addock.h"

namespace ad {

constexpr int kWave = 64;
constexpr int kMaxAtoms = AD_MAX_ATOMS;
constexpr int kMaxTor = AD_MAX_TORSIONS;
constexpr int kStride = AD_GENO_STRIDE;
constexpr int kMaxTypes = AD_MAX_TYPES;
constexpr int kFeat = 32;     // pre-screen atom features
constexpr int kMaxDeg = 8;    // pre-screen neighbour slots per atom

// Per-ligand descriptor in device memory.
struct LigDesc {
  int n_atoms, n_tor, n_pairs, n_frag;
  int atom_off;   // into the AtomGeo / AtomInfo arrays
  int pair_off;   // into the PairRec array
  int tor_off;    // into the TorRec array
  int max_depth;  // longest chain of nested torsions
};

// Reference coordinates relative to the rotation centre (reference
// centroid), in the internal atom order: depth first from the root atom, so
// that every torsion's moving set is one contiguous index range.
struct alignas(32) AtomGeo {
  double y[3];
  double pad;
};

struct alignas(16) AtomInfo {
  int map;        // affinity map index of the atom's type
  float q;        // partial charge
  int owner;      // deepest torsion whose moving set holds the atom (-1: root fragment)
  int16_t type;   // force-field type
  int16_t slot;   // prefix-sum slot of the atom (-1: no torsion range ends at it), see TorRec
};

// Intramolecular pair (16 bytes): i, j (internal order) and the type-pair
// index packed in one word, with the two pair-specific coefficients
// precomputed in double and rounded: qq = w_el k_e q_i q_j,
// dsv = w_sol (S_i V_j + S_j V_i).  A ligand's list stays L1-resident.
struct alignas(16) PairRec {
  uint32_t ijt;   // i | j << 8 | (ti * n_types + tj) << 16
  float qq;
  float dsv;
  float pad;
};

// Torsion: axis through o (reference frame, relative to the centre) with
// unit direction u; parent torsion (-1: hangs off the root fragment);
// moving set = internal atoms [s, e); root-side atom a and leaf-side atom b
// (internal indices); 1/|y_b - y_a| (bond length is pose invariant).
// The gradient needs the prefix sums over the internal order only where a
// moving set ends (atoms e - 1 and s - 1) and at the last atom (the totals):
// those atoms own the ligand's prefix-sum slots, slot 0 for the last atom and
// the others in increasing atom order, at most min(2T + 1, N) of them.
// s_slot / e_slot are the slots of atoms s - 1 (-1 when s = 0) and e - 1.
struct alignas(16) TorRec {
  double o[3];
  double u[3];
  double inv_len;
  int parent, s, e, a, b;
  int depth;      // torsions on the path from the root, this one included
  int s_slot, e_slot;
};

// 12-6 / 12-10 coefficients of a type pair (weights folded in).
struct alignas(16) LJRec {
  float A, B, r0, hb;   // hb = 1 for the 12-10 form
};

// Scalars of the functional form used inside the kernels.
struct FFConst {
  float diel_A, diel_B, diel_k, diel_lB_log2e;   // exp(-lambda B r) = exp2(-diel_lB_log2e r)
  float ds_log2e;                                // exp(-r^2/(2 s^2)) = exp2(-ds_log2e r^2)
  float inv_s2;                                  // 1/sigma^2
  float diel_c1;                                 // k * B * (lambda B): elec derivative factor
  float half_smooth, r_floor2;
  float w_tor;
  int n_types;
  double k_out;
};

// Resident grid as seen by the kernels: per affinity map m one float4 per
// node {map_m, elec, desolv, 0}, node-major [m][nz][ny][nx].
struct GridArgs {
  const float *maps;   // float4 records
  int nx, ny, nz, n_maps;
  double ox, oy, oz;
  double h, inv_h;
};

// Device view of a ligand batch.
struct BatchArgs {
  const LigDesc *lig;
  const AtomGeo *geo;
  const AtomInfo *info;
  const PairRec *pairs;
  const TorRec *tors;
  const LJRec *lj;       // [n_types * n_types]
  const double *trig;    // [kTrigN][2]: sin, cos of j * pi / (kTrigN / 2), j = 0..kTrigN-1
  int n_lig;
  int n_types;
};

constexpr int kTrigN = 128;   // table of torsion sin/cos at multiples of pi/64

// Host-side prepared ligand (before upload).
struct PreparedLigand {
  int n_atoms = 0, n_tor = 0, n_frag = 0, max_depth = 0, depth_sum = 0;
  std::vector<AtomGeo> geo;
  std::vector<AtomInfo> info;
  std::vector<PairRec> pairs;
  std::vector<TorRec> tors;
  std::vector<int> perm;   // internal index -> input atom index
};

// Host preprocessing (prep.cpp).  type_to_map may be null (validation only).
int prepare_ligand(const ad_ligand &L, const ad_forcefield &ff, const int *type_to_map, PreparedLigand *out,
                   std::string *err);
void build_lj_table(const ad_forcefield &ff, std::vector<LJRec> *out);
FFConst make_ffconst(const ad_forcefield &ff);
uint16_t f32_to_bf16(float f);
bool featurize(const ad_ligand &L, const std::vector<int> &perm, std::vector<uint16_t> *X,
               std::vector<uint8_t> *nbr);

}  // namespace ad
