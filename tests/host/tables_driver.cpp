// Host-side driver of the table builder for the sanitizer test: builds the
// full tables (with the model prediction and two extra second-level
// binnings) and the geometry-only tables for a spread of grids, binnings,
// multipole sets and work-item shapes, and prints one line per case.
#include <array>
#include <cstdio>
#include <string>
#include <vector>

#include "bk_tables.hpp"

int main() {
  struct Case {
    int ng, n_k1;
    double k1_min, k1_max;
    int n_mu, n_t, l_max;
    bool even;
    int pairs, ipw, sides;
  };
  const std::vector<Case> cases = {
      {8, 2, 1.0, 8 / 3.0, 3, 2, 6, true, 16, 2, 159},   // smallest grid
      {16, 3, 2.0, 5.0, 5, 3, 6, true, 16, 2, 159},
      {24, 2, 3.0, 8.0, 3, 3, 12, true, 16, 2, 159},     // 49 outputs
      {24, 2, 3.0, 8.0, 3, 3, 7, false, 16, 2, 159},     // every l (64 outputs)
      {48, 2, 3.0, 16.0, 4, 4, 4, false, 16, 1, 104},    // one item per wave
      {48, 3, 3.0, 16.0, 4, 4, 6, true, 32, 1, 104},     // two row tiles per item
      {48, 3, 3.0, 16.0, 4, 4, 6, true, 64, 1, 104},     // four row tiles per item
      {64, 3, 4.0, 21.0, 6, 5, 6, true, 16, 2, 48},      // small side cap
      {96, 20, 1.0, 32.0, 10, 10, 6, true, 16, 2, 159},  // radix-3 and radix-5 grids
  };
  int failures = 0;
  for (const Case& c : cases) {
    bk::Binning b;
    b.ng = c.ng;
    b.box_len = c.ng;
    b.n_k1 = c.n_k1;
    b.k1_min = c.k1_min;
    b.k1_max = c.k1_max;
    b.n_mu = c.n_mu;
    b.n_t = c.n_t;
    b.l_max = c.l_max;
    b.m_max = c.l_max;
    b.even_l_only = c.even;
    bk::K3Shape sh;
    sh.pairs_per_item = c.pairs;
    sh.items_per_wave = c.ipw;
    sh.max_group_sides = c.sides;
    bk::Model model;
    model.amp = 1.0;
    model.n_s = -2.0;
    model.f_ng = 0.5;
    model.beta = 0.5;
    const std::vector<std::array<int, 3>> extra = {{1, 2, 2}, {c.n_k1, 2 * c.n_mu, c.n_t}};
    bk::Tables full, geo;
    const std::string e1 = bk::build_tables(b, sh, 4, &full, &model, false, extra);
    const std::string e2 = bk::build_tables(b, sh, 2, &geo, nullptr, true);
    const bool ok = e1.empty() && e2.empty() && full.n_combos == geo.n_combos && full.res.size() == 3;
    failures += ok ? 0 : 1;
    std::printf("ng=%d pairs=%d ipw=%d %s combinations=%lld items=%zu groups=%zu\n", c.ng, c.pairs, c.ipw,
                ok ? "ok" : (e1 + e2).c_str(), static_cast<long long>(full.n_combos), full.items.size(),
                full.groups.size());
  }
  const std::vector<double> cm = bk::continuum_multipoles(6, 6, 0.7, 0.8, 0.5);
  std::printf("continuum outputs=%zu\n", cm.size());
  return failures == 0 && cm.size() == 16 ? 0 : 1;
}
