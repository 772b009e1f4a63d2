// Host-side check of the contraction's work decomposition: for every kept
// combination the cell it is summed in must stage three real sides on planes
// (a, b, a + b) of one canonical plane triple, on a grid m that no closure
// other than the exact one can alias (m > U_A + U_B + U_C and m > 2 max U,
// with U the largest |u_x| of the ring's lattice modes), each combination in
// its own cell; and every group must respect its LDS slot and item limits
// and stage sides laid out without overlap in D.  Prints one line per case
// and returns nonzero on the first violation.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "bk_tables.hpp"

#define CHECK(cond, ...)                         \
  do {                                           \
    if (!(cond)) {                               \
      std::printf("FAIL %s: ", #cond);           \
      std::printf(__VA_ARGS__);                  \
      std::printf("\n");                         \
      return false;                              \
    }                                            \
  } while (0)

static bool check(const bk::Binning& b, const bk::K3Shape& sh) {
  bk::Tables T;
  const std::string err = bk::build_tables(b, sh, 4, &T);
  CHECK(err.empty(), "%s", err.c_str());
  // U per ring from the lattice modes themselves
  std::vector<int> umax(T.nr + 1, -1);
  const int w = 2 * T.lim + 1;
  for (int ux = -T.lim; ux <= T.lim; ++ux)
    for (int uy = -T.lim; uy <= T.lim; ++uy) {
      const int r = T.mode_ring[size_t(ux + T.lim) * w + (uy + T.lim)];
      if (r > 0) umax[r] = std::max(umax[r], std::abs(ux));
    }
  const int ppi = sh.pairs_per_item;
  const int cells = ppi * bk::kTileN;
  // D layout: sides of one level back to back, m^2 points each
  int64_t off = 0;
  for (size_t g = 0; g < T.gside_off.size(); ++g) {
    const int m = T.grid_sizes[T.gside_level[g]];
    CHECK(T.gside_off[g] == off, "grid side %zu at %lld, expected %lld", g, (long long)T.gside_off[g], (long long)off);
    off += int64_t(m) * m;
  }
  CHECK(off == T.d_elems, "D holds %lld points, sides need %lld", (long long)T.d_elems, (long long)off);
  // group limits, and the owner group of every item
  std::vector<int> owner(T.items.size(), -1);
  for (size_t g = 0; g < T.groups.size(); ++g) {
    const bk::GroupDesc& gd = T.groups[g];
    CHECK(gd.n_sides >= 1 && gd.n_sides <= sh.max_group_sides, "group %zu stages %d sides", g, gd.n_sides);
    CHECK(gd.n_items >= 1 && gd.n_items <= bk::kWavesPerGroup * sh.items_per_wave, "group %zu holds %d items", g,
          gd.n_items);
    CHECK(gd.zero_key >= 0 && gd.zero_key < bk::kKeys, "group %zu zero key %d", g, gd.zero_key);
    for (int k = 0; k < gd.n_sides; ++k) {
      const int32_t e = T.group_sides[gd.side_begin + k];
      const int gs = e & ((1 << bk::kKeyShift) - 1);
      CHECK((e >> bk::kKeyShift) < bk::kKeys, "group %zu key", g);
      CHECK(T.grid_sizes[T.gside_level[gs]] == gd.grid, "group %zu stages a side of another grid", g);
    }
    for (int i = 0; i < gd.n_items; ++i) {
      const bk::ItemDesc& it = T.items[gd.item_begin + i];
      owner[gd.item_begin + i] = int(g);
      for (int p = 0; p < ppi; ++p)
        CHECK(it.a_slot[p] <= gd.n_sides && it.c_slot[p] <= gd.n_sides, "item slot out of the group");
      for (int j = 0; j < bk::kTileN; ++j) CHECK(it.b_slot[j] <= gd.n_sides, "item slot out of the group");
    }
  }
  for (size_t i = 0; i < owner.size(); ++i) CHECK(owner[i] >= 0, "item %zu in no group", i);
  // every kept combination: one cell of its own, three real sides, an alias-free grid
  const bk::Resolution& R = T.res[0];
  CHECK(int64_t(R.combo_slot.size()) == T.n_combos, "%zu cells for %lld combinations", R.combo_slot.size(),
        (long long)T.n_combos);
  std::vector<int64_t> slots(R.combo_slot);
  std::sort(slots.begin(), slots.end());
  CHECK(std::adjacent_find(slots.begin(), slots.end()) == slots.end(), "two combinations share a cell");
  for (int64_t s : slots) {
    CHECK(s >= 0 && s / T.s_per_item < int64_t(T.items.size()), "cell %lld out of range", (long long)s);
    const int64_t item = s / T.s_per_item, rem = s % T.s_per_item;
    CHECK(rem < cells, "combination in the Im S half");
    const int pair = int(rem / bk::kTileN), col = int(rem % bk::kTileN);
    const bk::GroupDesc& gd = T.groups[owner[item]];
    const bk::ItemDesc& it = T.items[item];
    const int sa = it.a_slot[pair], sb = it.b_slot[col], sc = it.c_slot[pair];
    CHECK(sa < gd.n_sides && sb < gd.n_sides && sc < gd.n_sides, "a kept combination reads the zero slot");
    auto side_of = [&](int slot) {
      return T.gside_side[T.group_sides[gd.side_begin + slot] & ((1 << bk::kKeyShift) - 1)];
    };
    const int A = side_of(sa), B = side_of(sb), C = side_of(sc);
    const int pa = T.side_plane[A], pb = T.side_plane[B], pc = T.side_plane[C];
    CHECK(pa >= pb && pb >= 0 && pc == pa + pb, "planes (%d, %d, %d) are not a canonical triple", pa, pb, pc);
    const int ua = umax[T.side_ring[A]], ub = umax[T.side_ring[B]], uc = umax[T.side_ring[C]];
    CHECK(ua >= 0 && ub >= 0 && uc >= 0, "ring without modes");
    const int m = gd.grid;
    CHECK(m == b.ng || (m > ua + ub + uc && m > 2 * std::max(ua, std::max(ub, uc))),
          "grid %d aliases rings with U = %d, %d, %d", m, ua, ub, uc);
  }
  std::printf("ng=%d pairs=%d ipw=%d sides<=%d ok: %lld combinations in %zu items, %zu groups, %zu grid sides\n", b.ng,
              ppi, sh.items_per_wave, sh.max_group_sides, (long long)T.n_combos, T.items.size(), T.groups.size(),
              T.gside_off.size());
  return true;
}

int main() {
  struct Case {
    int ng, n_k1;
    double k1_min, k1_max;
    int n_mu, n_t;
    bool even;
    int pairs, ipw, sides;
  };
  const std::vector<Case> cases = {
      {16, 3, 2.0, 5.0, 5, 3, true, 16, 2, 159},
      {48, 3, 3.0, 16.0, 4, 4, true, 16, 2, 159},
      {48, 3, 3.0, 16.0, 4, 4, true, 16, 1, 104},
      {48, 3, 3.0, 16.0, 4, 4, true, 32, 1, 104},
      {48, 3, 3.0, 16.0, 4, 4, true, 64, 1, 104},
      {64, 3, 4.0, 21.0, 6, 5, true, 16, 2, 48},
      {96, 20, 1.0, 32.0, 10, 10, true, 16, 2, 159},
      {128, 20, 1.0, 128 / 3.0, 10, 10, false, 16, 2, 159},
  };
  for (const Case& c : cases) {
    bk::Binning b;
    b.ng = c.ng;
    b.box_len = c.ng;
    b.n_k1 = c.n_k1;
    b.k1_min = c.k1_min;
    b.k1_max = c.k1_max;
    b.n_mu = c.n_mu;
    b.n_t = c.n_t;
    b.even_l_only = c.even;
    bk::K3Shape sh;
    sh.pairs_per_item = c.pairs;
    sh.items_per_wave = c.ipw;
    sh.max_group_sides = c.sides;
    if (!check(b, sh)) return 1;
  }
  return 0;
}
