// Host-side geometry and work decomposition of the bispectrum-multipole
// estimator (arXiv:2405.14513, Sec. II).  Pure C++ (no HIP): built with
// -ffp-contract=off so every float64 decision that picks an integer (a bin,
// a kept combination) is taken in plain IEEE operations in a fixed order.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace bk {

// Shape of the contraction's work items (chosen per plan).  A work item is
// pairs_per_item ring pairs x kTileN slot-B rings; a wave contracts
// items_per_wave items (pairs_per_item / 16 row tiles each); a workgroup of
// kWavesPerGroup waves stages at most max_group_sides sides for its items.
struct K3Shape {
  int pairs_per_item = 16;   // 16, 32 or 64
  int items_per_wave = 1;    // 1 or 2 (2 only with 16 pairs)
  int max_group_sides = 104;
  bool coarse_grids = true;  // evaluate each combination on the smallest alias-free x_perp grid
};

struct Binning {
  int ng = 0;
  double box_len = 0.0;  // L
  int n_k1 = 0;
  double k1_min = 0.0, k1_max = 0.0;
  int n_mu = 0, n_t = 0;
  int l_max = 6, m_max = 6;
  bool even_l_only = true;  // false: odd l too, as the imaginary part (see build_tables)
};

// Sizes of the K3 work decomposition.
constexpr int kTileN = 16;           // third-slot rings per work item (MFMA N)
constexpr int kMaxPairsPerItem = 64;  // ring pairs per work item: 16 per MFMA row tile, 1, 2 or 4 tiles
constexpr int kWavesPerGroup = 8;     // waves per workgroup (items on neighbouring plane triples)
constexpr int kChunkMax = 64;      // x_perp points staged in LDS per step (32 or 64)
constexpr int kMaxGroupSidesLimit = 254;  // LDS slots are bytes, the zero slot included
constexpr int kKeyShift = 24;       // group_sides entries: grid side in the low 24 bits, key above
constexpr int kKeys = 16;           // LDS swizzle keys (16-byte units are permuted within groups of 16)  // sides a workgroup gathering several items may stage

// One workgroup of the contraction kernel: up to kWavesPerGroup * items_per_wave work items on
// one grid (from one or a few neighbouring plane triples) that share the
// sides staged in LDS.
struct GroupDesc {
  int32_t side_begin;  // into group_sides
  int32_t n_sides;     // sides staged (the last LDS slot, n_sides, is all zeros)
  int32_t item_begin;  // first work item
  int32_t n_items;
  int32_t conj_mask;   // bit s set: slot s (0 = A, 1 = B, 2 = C) is a negative plane -> conjugate D
  int32_t grid;        // x_perp grid size m of every combination in the group (sum over m^2 points)
  int32_t zero_key;    // LDS swizzle key of the zero slot
  int32_t pad;
};

// One work item: up to kMaxPairsPerItem pairs of (slot A ring, slot C ring)
// and kTileN slot-B rings.  Indices are LDS slots of the owning group.
struct ItemDesc {
  uint8_t a_slot[kMaxPairsPerItem];
  uint8_t c_slot[kMaxPairsPerItem];
  uint8_t b_slot[kTileN];
};

constexpr int kMaxResolutions = 8;

// One second-level binning of the kept combinations (Eq. 13): the same k1
// range, (l, m) outputs and combinations, with its own numbers of bins.
struct Resolution {
  int n_k1 = 0, n_mu = 0, n_t = 0;
  std::vector<int64_t> combo_slot;       // per combination in bin order: index into the K3 output (item * cells + pair * 16 + col)
  std::vector<double> combo_coef;        // [combo][n_lm]: final coefficient on Re S (Im S for odd l)
  std::vector<int64_t> bin_ptr;          // combinations sorted by bin: CSR offsets [n_bins + 1]
  std::vector<int64_t> bin_count;        // sum of mult * N_tri per bin
  std::vector<double> bin_den;           // [n_lm][n_bins]
  std::vector<double> bin_mean;          // [n_bins][3]
  std::vector<uint8_t> bin_empty_lm;     // [n_lm][n_bins] 1 if NaN
  std::vector<double> model_pred;        // [n_lm][n_bins] discrete prediction (with a model), NaN if empty
  int n_bins() const { return n_k1 * n_mu * n_t; }
};

struct Tables {
  Binning bin;
  K3Shape k3;
  int ng = 0, nr = 0, nmax = 0;
  std::vector<int64_t> edge3;              // 3 * R_r (R_r rational with denominator 3), r = 0..nr
  std::vector<double> mean_radius;         // K_r, r = 1..nr (index r-1)
  std::vector<int64_t> ring_count;         // modes per ring
  std::vector<int64_t> ntri;               // N_tri[r1][r2][r3], nr^3
  std::vector<int32_t> mode_ring;          // ring (1-based, 0 = none) of every (ux, uy) in [-lim, lim]^2
  int lim = 0;

  // sides with n >= 0 (the stored ones); side (r, n) -> index or -1
  std::vector<int32_t> side_of;  // [(nmax+1) * (nr+1)]
  std::vector<int32_t> side_ring, side_plane;

  // (l, m) outputs
  std::vector<int> lm_l, lm_m;

  // kept canonical combinations
  int64_t n_combos = 0;
  int64_t n_self_partner = 0;             // combinations equal to their n -> -n partner
  int64_t n_canonical_planes = 0;
  // the second-level binnings: res[0] is the binning's own (n_k1, n_mu, n_t),
  // further ones share everything but the bin counts
  std::vector<Resolution> res;

  // x_perp grids.  A combination of rings whose modes reach |u_x|, |u_y| <= U
  // is summed exactly on any m x m grid with m > U_A + U_B + U_C (no closure
  // u_A + u_B + u_C = 0 mod m other than 0 fits) and m > 2 max U (every
  // side's modes keep distinct positions mod m); it takes the smallest grid
  // size of the list that qualifies, and its S is rescaled by (N_g / m)^2.
  std::vector<int32_t> ring_u;           // U per ring (index r-1): largest |u_x| with |u_x| < R_r
  std::vector<int32_t> grid_sizes;       // ascending; the last is N_g
  // grid sides: (side, grid level) pairs that some combination uses, in
  // (level, side) order; D holds m^2 points for each, at gside_off
  std::vector<int32_t> gside_side, gside_level;
  std::vector<int64_t> gside_off;        // complex elements from the start of a field's D
  std::vector<int32_t> level_gside_begin;  // [levels + 1]
  int64_t d_elems = 0;                   // complex elements of D per field

  // K3 decomposition
  std::vector<GroupDesc> groups;
  std::vector<ItemDesc> items;
  std::vector<int32_t> group_sides;      // per LDS slot: grid-side index | swizzle key << kKeyShift
  int max_group_sides = 0;
  double dense_terms = 0.0, useful_terms = 0.0;
  // float64 outputs of the contraction per work item: Re S of every (pair,
  // column) cell, followed by Im S when odd l are requested
  int64_t s_per_item = 0;
};

// The paper's model field (Eqs. 14-17): P(k) = amp k^n_s with k in units of
// k_f, B = 2 f_NG (P1 P2 + P2 P3 + P3 P1) prod_i (1 + beta mu_i^2).
struct Model {
  double amp = 0.0, n_s = 0.0, f_ng = 0.0, beta = 0.0;
};

// Builds everything; returns "" on success or an error message.  With a
// model, also the discrete prediction [B]_d per bin (model_pred).  With
// geometry_only, stops after the per-bin geometry (no contraction tables).
// extra_bins lists further (n_k1, n_mu, n_t) binnings of the same
// combinations (res[1], res[2], ...).
std::string build_tables(const Binning& b, const K3Shape& k3, int n_threads, Tables* out,
                         const Model* model = nullptr, bool geometry_only = false,
                         const std::vector<std::array<int, 3>>& extra_bins = {});

// [B_l^m]_c / B_r for the model's redshift-space factor (Eq. 4 with Eqs. 3
// and 17), by Gauss-Legendre x uniform-phase quadrature, exact for the
// polynomial integrand; outputs in (l, m) order as count_lm.  The imaginary
// parts vanish for this model (mirror symmetry in p_y).
std::vector<double> continuum_multipoles(int l_max, int m_max, double mu, double t, double beta);

// Number of (l, m) outputs for l_max, m_max (even l only, or every l).
int count_lm(int l_max, int m_max, bool even_only = true);

}  // namespace bk
