// Host-side geometry and work decomposition (see bk_tables.hpp).
//
// Paper references: rings and the N_g/3 cap (Sec. II, implementation
// paragraph), N_tri (Eq. 10), the shape parameters (Eq. 2), the orientation
// (Eq. 3), and the second-level binning (Eq. 13).  The readings fixed here
// are listed in include/bk.h.
#include "bk_tables.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <map>
#include <numeric>
#include <thread>
#include <tuple>

namespace bk {

namespace {

constexpr double kDegenerateS = 1e-12;

// |u|^2 = q lies below edge e (given as 3 * edge): 9 q < e3^2.
inline bool below(int64_t q, int64_t e3) { return 9 * q < e3 * e3; }

// Associated Legendre P_l^m(x) with the Condon-Shortley phase, by the
// standard upward recurrence in l at fixed m.
void legendre_table(int l_max, double x, std::vector<double>* p /* [(l_max+1)^2], p[l*(l_max+1)+m] */) {
  const int L = l_max + 1;
  p->assign(L * L, 0.0);
  const double s = std::sqrt(std::max(0.0, 1.0 - x * x));
  double pmm = 1.0;
  for (int m = 0; m <= l_max; ++m) {
    if (m > 0) pmm *= -(2.0 * m - 1.0) * s;
    (*p)[m * L + m] = pmm;
    if (m + 1 <= l_max) (*p)[(m + 1) * L + m] = x * (2.0 * m + 1.0) * pmm;
    for (int l = m + 2; l <= l_max; ++l) {
      (*p)[l * L + m] = ((2.0 * l - 1.0) * x * (*p)[(l - 1) * L + m] - (l + m - 1.0) * (*p)[(l - 2) * L + m]) /
                        double(l - m);
    }
  }
}

double norm_lm(int l, int m) {
  double r = 1.0;  // (l-m)!/(l+m)!
  for (int i = l - m + 1; i <= l + m; ++i) r /= double(i);
  return std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * r);
}

struct Candidate {
  int32_t ra, rb, rc;  // rings of slots A (plane a), B (plane b), C (plane -(a+b))
};

// Bin of a kept shape (k1, mu, t) among dims = (n_k1, n_mu, n_t) equal bins
// of [k1_min, k1_max) x [1/2, 1] x [1/2, 1]; the upper edges fall in the last bin.
int bin_index(double k1_min, double k1_max, const std::array<int, 3>& dims, double k1, double mu, double tt) {
  const double dk = (k1_max - k1_min) / double(dims[0]);
  const double dmu = 0.5 / double(dims[1]);
  const double dt = 0.5 / double(dims[2]);
  const int ik = std::min(int(std::floor((k1 - k1_min) / dk)), dims[0] - 1);
  const int imu = std::min(int(std::floor((mu - 0.5) / dmu)), dims[1] - 1);
  const int it = std::min(int(std::floor((tt - 0.5) / dt)), dims[2] - 1);
  return (ik * dims[1] + imu) * dims[2] + it;
}

}  // namespace

int count_lm(int l_max, int m_max, bool even_only) {
  int n = 0;
  for (int l = 0; l <= l_max; l += even_only ? 2 : 1) n += std::min(l, m_max) + 1;
  return n;
}

std::string build_tables(const Binning& b, const K3Shape& k3, int n_threads, Tables* out, const Model* model,
                         bool geometry_only, const std::vector<std::array<int, 3>>& extra_bins) {
  Tables& T = *out;
  T = Tables();
  T.bin = b;
  T.k3 = k3;
  const int ppi = k3.pairs_per_item;
  if (ppi != 16 && ppi != 32 && ppi != 64) return "pairs per work item must be 16, 32 or 64";
  const int ipw = k3.items_per_wave;
  if (ipw != 1 && !(ipw == 2 && ppi == 16)) return "items per wave must be 1, or 2 with 16 pairs per item";
  if (k3.max_group_sides < 1 || k3.max_group_sides > kMaxGroupSidesLimit) return "staged sides per workgroup out of range";
  T.s_per_item = int64_t(ppi) * kTileN * (b.even_l_only ? 1 : 2);
  const int ng = b.ng;
  T.ng = ng;
  if (n_threads < 1) n_threads = 1;

  // ---- rings: edges 3*R_r, widths 2^floor((r-1)/10), last edge clipped to N_g/3
  T.edge3.push_back(0);
  for (int r = 1;; ++r) {
    int64_t nxt = T.edge3.back() + 3 * (int64_t(1) << ((r - 1) / 10));
    if (nxt >= ng) {
      T.edge3.push_back(ng);
      break;
    }
    T.edge3.push_back(nxt);
  }
  const int nr = int(T.edge3.size()) - 1;
  T.nr = nr;
  T.ring_u.assign(nr, 0);
  for (int r = 1; r <= nr; ++r) {
    int U = 0;
    while (9 * int64_t(U + 1) * (U + 1) < T.edge3[r] * T.edge3[r]) ++U;
    T.ring_u[r - 1] = U;
  }
  // grid sizes: 2^a, 3 * 2^a and 5 * 2^a from 16 up, multiples of 8 (the sizes
  // the FFT stages take), then N_g
  if (k3.coarse_grids)
    for (int base : {2, 3, 5})
      for (int m = base; m < ng; m *= 2)
        if (m >= 16 && m % 8 == 0) T.grid_sizes.push_back(m);
  std::sort(T.grid_sizes.begin(), T.grid_sizes.end());
  T.grid_sizes.push_back(ng);
  auto level_of = [&](int ra, int rb, int rc) {
    const int ua = T.ring_u[ra - 1], ub = T.ring_u[rb - 1], uc = T.ring_u[rc - 1];
    const int need = std::max(ua + ub + uc + 1, 2 * std::max(ua, std::max(ub, uc)) + 1);
    for (size_t L = 0; L < T.grid_sizes.size(); ++L)
      if (T.grid_sizes[L] >= need) return int32_t(L);
    return int32_t(T.grid_sizes.size() - 1);  // N_g: exact for every combination
  };
  const int lim = ng / 3 + 1;
  T.lim = lim;
  const int side_len = 2 * lim + 1;
  T.mode_ring.assign(size_t(side_len) * side_len, 0);
  std::vector<std::map<int64_t, int64_t>> shells(nr);
  T.ring_count.assign(nr, 0);
  for (int ux = -lim; ux <= lim; ++ux) {
    for (int uy = -lim; uy <= lim; ++uy) {
      const int64_t q = int64_t(ux) * ux + int64_t(uy) * uy;
      for (int r = 1; r <= nr; ++r) {
        if (!below(q, T.edge3[r - 1]) && below(q, T.edge3[r])) {
          T.mode_ring[size_t(ux + lim) * side_len + (uy + lim)] = r;
          shells[r - 1][q] += 1;
          T.ring_count[r - 1] += 1;
          break;
        }
      }
    }
  }
  T.mean_radius.assign(nr, 0.0);
  for (int r = 0; r < nr; ++r) {
    if (T.ring_count[r] == 0) return "ring " + std::to_string(r + 1) + " holds no lattice mode";
    double acc = 0.0;
    for (const auto& kv : shells[r]) acc += double(kv.second) * std::sqrt(double(kv.first));
    T.mean_radius[r] = acc / double(T.ring_count[r]);
  }

  // ---- N_tri(r1, r2, r3) (Eq. 10) by counting every (u, v) with w = -u - v in a ring
  {
    std::vector<int32_t> mx, my, mr;
    for (int ux = -lim; ux <= lim; ++ux)
      for (int uy = -lim; uy <= lim; ++uy) {
        int r = T.mode_ring[size_t(ux + lim) * side_len + (uy + lim)];
        if (r) {
          mx.push_back(ux);
          my.push_back(uy);
          mr.push_back(r);
        }
      }
    const size_t nm = mx.size();
    const int W = 2 * lim;  // |w_x| <= 2 lim
    const int wlen = 2 * W + 1;
    std::vector<int32_t> wring(size_t(wlen) * wlen, 0);
    for (int wx = -W; wx <= W; ++wx)
      for (int wy = -W; wy <= W; ++wy)
        if (std::abs(wx) <= lim && std::abs(wy) <= lim)
          wring[size_t(wx + W) * wlen + (wy + W)] = T.mode_ring[size_t(wx + lim) * side_len + (wy + lim)];
    const size_t nr1 = nr + 1;
    std::vector<std::vector<int64_t>> partial(n_threads, std::vector<int64_t>(nr1 * nr1 * nr1, 0));
    std::vector<std::thread> th;
    for (int t = 0; t < n_threads; ++t) {
      th.emplace_back([&, t]() {
        auto& cnt = partial[t];
        for (size_t i = t; i < nm; i += n_threads) {
          const int ux = mx[i], uy = my[i];
          const size_t base1 = size_t(mr[i]) * nr1 * nr1;
          for (size_t j = 0; j < nm; ++j) {
            const int wx = -ux - mx[j], wy = -uy - my[j];
            const int r3 = wring[size_t(wx + W) * wlen + (wy + W)];
            if (r3) cnt[base1 + size_t(mr[j]) * nr1 + r3] += 1;
          }
        }
      });
    }
    for (auto& x : th) x.join();
    T.ntri.assign(size_t(nr) * nr * nr, 0);
    for (int r1 = 1; r1 <= nr; ++r1)
      for (int r2 = 1; r2 <= nr; ++r2)
        for (int r3 = 1; r3 <= nr; ++r3) {
          int64_t s = 0;
          for (int t = 0; t < n_threads; ++t) s += partial[t][(size_t(r1) * nr1 + r2) * nr1 + r3];
          T.ntri[(size_t(r1 - 1) * nr + (r2 - 1)) * nr + (r3 - 1)] = s;
        }
  }

  // ---- sides n >= 0 with mean-value k < k1_max; the k = 0 side is excluded
  const int nmax = int(std::ceil(b.k1_max));
  T.nmax = nmax;
  T.side_of.assign(size_t(nmax + 1) * (nr + 1), -1);
  for (int n = 0; n <= nmax; ++n)
    for (int r = 1; r <= nr; ++r) {
      if (r == 1 && n == 0) continue;
      const double kk = T.mean_radius[r - 1];
      const double q = kk * kk + double(n) * double(n);
      if (std::sqrt(q) < b.k1_max) {
        T.side_of[size_t(n) * (nr + 1) + r] = int32_t(T.side_ring.size());
        T.side_ring.push_back(r);
        T.side_plane.push_back(n);
      }
    }
  auto side = [&](int r, int n_abs) -> int32_t {
    if (n_abs > nmax || r < 1 || r > nr) return -1;
    return T.side_of[size_t(n_abs) * (nr + 1) + r];
  };

  // ---- outputs.  For odd l a combination and its n -> -n partner carry
  // conjugate S and weights of opposite sign, so their sum is 2 i w Im S: odd
  // l are reported as the imaginary part of Eq. 13 (real part zero), and the
  // same coefficient multiplies Im S instead of Re S.
  for (int l = 0; l <= b.l_max; l += b.even_l_only ? 2 : 1)
    for (int m = 0; m <= std::min(l, b.m_max); ++m) {
      T.lm_l.push_back(l);
      T.lm_m.push_back(m);
    }
  const int nlm = int(T.lm_l.size());
  if (nlm > 64) return "at most 64 multipoles per plan";
  std::vector<double> nlm_norm(nlm), pref(nlm);
  for (int j = 0; j < nlm; ++j) {
    nlm_norm[j] = norm_lm(T.lm_l[j], T.lm_m[j]);
    pref[j] = std::sqrt((2.0 * T.lm_l[j] + 1.0) / (4.0 * M_PI));
  }
  // the resolutions: the binning's own, then the extra ones
  std::vector<std::array<int, 3>> rdims{{b.n_k1, b.n_mu, b.n_t}};
  rdims.insert(rdims.end(), extra_bins.begin(), extra_bins.end());
  const int n_res = int(rdims.size());
  const int n_extra = n_res - 1;
  if (n_res > kMaxResolutions) return "too many resolutions";
  for (const auto& d : rdims)
    if (d[0] < 1 || d[1] < 1 || d[2] < 1) return "bin counts must be >= 1";
  T.res.assign(n_res, Resolution());
  for (int r = 0; r < n_res; ++r) {
    T.res[r].n_k1 = rdims[r][0];
    T.res[r].n_mu = rdims[r][1];
    T.res[r].n_t = rdims[r][2];
  }

  // ---- canonical plane triples (a, b, -(a+b)), a >= b >= 0, and their kept combinations.
  // The partner with every n negated has conjugate S and, for even l, the same
  // weight and bin; it is folded in through mult = 2 (1 when self-partnered).
  struct PT {
    int a, b;
  };
  std::vector<PT> pts;
  for (int a = 0; a <= nmax; ++a)
    for (int bb = 0; bb <= a; ++bb)
      if (a + bb <= nmax) pts.push_back({a, bb});

  struct ComboRec {
    int32_t pt;  // index into pts
    int32_t ra, rb, rc;
    int32_t bin;
    int32_t mult;
    int32_t level;  // x_perp grid
    int64_t ntri;
  };
  std::vector<std::vector<ComboRec>> per_pt(pts.size());
  std::vector<std::vector<int32_t>> per_pt_xbin(pts.size());  // bins in the extra resolutions
  std::vector<std::vector<double>> per_pt_w(pts.size()), per_pt_d(pts.size()), per_pt_kmt(pts.size());
  std::vector<std::vector<double>> per_pt_model(model ? pts.size() : 0);

  std::atomic<size_t> next_pt{0};
  std::vector<std::thread> th;
  for (int t = 0; t < n_threads; ++t) {
    th.emplace_back([&]() {
      std::vector<double> P;
      for (;;) {
        const size_t ip = next_pt.fetch_add(1);
        if (ip >= pts.size()) break;
        const int a = pts[ip].a, bb = pts[ip].b, c = a + bb;
        const int n_s[3] = {a, bb, -c};
        for (int ra = 1; ra <= nr; ++ra) {
          if (side(ra, a) < 0) continue;
          for (int rb = 1; rb <= nr; ++rb) {
            if (side(rb, bb) < 0) continue;
            if (a == bb && rb < ra) continue;  // slots A and B share plane a: unordered
            for (int rc = 1; rc <= nr; ++rc) {
              if (side(rc, c) < 0) continue;
              if (a == 0 && rc < rb) continue;        // (0,0,0): ra <= rb <= rc
              if (bb == 0 && a > 0 && rc < ra) continue;  // (a,0,-a): partner is (rc, rb, ra)
              const int64_t nt = T.ntri[(size_t(ra - 1) * nr + (rb - 1)) * nr + (rc - 1)];
              if (nt <= 0) continue;
              const int rs[3] = {ra, rb, rc};
              double q[3];
              for (int s = 0; s < 3; ++s) {
                const double kk = T.mean_radius[rs[s] - 1];
                q[s] = kk * kk + double(n_s[s]) * double(n_s[s]);
              }
              double qs[3] = {q[0], q[1], q[2]};
              std::sort(qs, qs + 3, [](double x, double y) { return x > y; });
              const double k1 = std::sqrt(qs[0]);
              const double k2 = std::sqrt(qs[1]);
              const double tt = k2 / k1;
              double mu = ((qs[0] + qs[1]) - qs[2]) / ((2.0 * k1) * k2);
              mu = std::min(std::max(mu, -1.0), 1.0);
              if (!(k1 >= b.k1_min && k1 < b.k1_max && tt >= 0.5 && tt <= 1.0 && mu >= 0.5 && mu <= 1.0)) continue;
              const int bin = bin_index(b.k1_min, b.k1_max, rdims[0], k1, mu, tt);
              for (int r = 1; r < n_res; ++r) per_pt_xbin[ip].push_back(bin_index(b.k1_min, b.k1_max, rdims[r], k1, mu, tt));

              // orientation weights, averaged over labellings consistent with k1 >= k2 >= k3
              static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
              double wsum[64], dsum[64];
              std::fill(wsum, wsum + nlm, 0.0);
              std::fill(dsum, dsum + nlm, 0.0);
              int nlab = 0;
              const double s = std::sqrt(1.0 - mu * mu);
              const bool degenerate = s < kDegenerateS;
              for (const auto& p : perms) {
                if (!(q[p[0]] >= q[p[1]] && q[p[1]] >= q[p[2]])) continue;
                ++nlab;
                const double mu1 = double(n_s[p[0]]) / k1;
                const double mu2 = double(n_s[p[1]]) / k2;
                double phi = 0.0;
                if (!degenerate) {
                  const double px = (mu2 + mu * mu1) / s;
                  const double py = std::sqrt(std::max((1.0 - mu1 * mu1) - px * px, 0.0));
                  phi = std::atan2(py, px);
                }
                legendre_table(b.l_max, mu1, &P);
                for (int j = 0; j < nlm; ++j) {
                  const int l = T.lm_l[j], m = T.lm_m[j];
                  const double y = nlm_norm[j] * P[l * (b.l_max + 1) + m];
                  const double w = degenerate ? (m == 0 ? y : 0.0) : y * std::cos(double(m) * phi);
                  wsum[j] += w;
                  dsum[j] += y * y;
                }
              }
              ComboRec cr;
              cr.pt = int32_t(ip);
              cr.ra = ra;
              cr.rb = rb;
              cr.rc = rc;
              cr.bin = bin;
              cr.level = level_of(ra, rb, rc);
              cr.ntri = nt;
              const bool self_partner = (a == 0) || (bb == 0 && ra == rc);
              cr.mult = self_partner ? 1 : 2;
              per_pt[ip].push_back(cr);
              for (int j = 0; j < nlm; ++j) {
                per_pt_w[ip].push_back(wsum[j] / double(nlab));
                per_pt_d[ip].push_back(dsum[j] / double(nlab));
              }
              per_pt_kmt[ip].push_back(k1);
              per_pt_kmt[ip].push_back(mu);
              per_pt_kmt[ip].push_back(tt);
              if (model) {
                // Eqs. 15 and 17 at the combination's mean sides, mu_i = n_i / k_i
                double pk[3], kai = 1.0;
                for (int s3 = 0; s3 < 3; ++s3) {
                  const double ks = std::sqrt(q[s3]);
                  const double mui = double(n_s[s3]) / ks;
                  pk[s3] = model->amp * std::pow(ks, model->n_s);
                  kai *= 1.0 + model->beta * (mui * mui);
                }
                per_pt_model[ip].push_back(2.0 * model->f_ng * (pk[0] * pk[1] + pk[1] * pk[2] + pk[2] * pk[0]) * kai);
              }
            }
          }
        }
      }
    });
  }
  for (auto& x : th) x.join();

  // ---- per-bin geometry sums (den, counts, means) of every resolution, each in the same fixed order
  int64_t total = 0;
  for (size_t ip = 0; ip < pts.size(); ++ip) {
    if (!per_pt[ip].empty()) T.n_canonical_planes += 1;
    for (const ComboRec& cr : per_pt[ip]) {
      if (cr.mult == 1) T.n_self_partner += 1;
      ++total;
    }
  }
  T.n_combos = total;
  auto bin_of = [&](int r, size_t ip, size_t i) -> int {
    return r == 0 ? per_pt[ip][i].bin : per_pt_xbin[ip][i * n_extra + (r - 1)];
  };
  for (int r = 0; r < n_res; ++r) {
    Resolution& R = T.res[r];
    const int n_bins = R.n_bins();
    R.bin_count.assign(n_bins, 0);
    R.bin_den.assign(size_t(nlm) * n_bins, 0.0);
    std::vector<double> mean_acc(size_t(n_bins) * 3, 0.0), mean_w(n_bins, 0.0);
    std::vector<double> model_num(model ? size_t(nlm) * n_bins : 0, 0.0);
    for (size_t ip = 0; ip < pts.size(); ++ip) {
      for (size_t i = 0; i < per_pt[ip].size(); ++i) {
        const ComboRec& cr = per_pt[ip][i];
        const int bin = bin_of(r, ip, i);
        const double wgt = double(cr.mult) * double(cr.ntri);
        R.bin_count[bin] += int64_t(cr.mult) * cr.ntri;
        for (int j = 0; j < nlm; ++j) R.bin_den[size_t(j) * n_bins + bin] += wgt * per_pt_d[ip][i * nlm + j];
        for (int k = 0; k < 3; ++k) mean_acc[size_t(bin) * 3 + k] += wgt * per_pt_kmt[ip][i * 3 + k];
        mean_w[bin] += wgt;
        if (model)
          for (int j = 0; j < nlm; ++j)
            // the model is the same on both partners, whose odd-l weights cancel
            if (T.lm_l[j] % 2 == 0)
              model_num[size_t(j) * n_bins + bin] += wgt * per_pt_w[ip][i * nlm + j] * per_pt_model[ip][i];
      }
    }
    R.bin_mean.assign(size_t(n_bins) * 3, std::nan(""));
    for (int i = 0; i < n_bins; ++i)
      if (mean_w[i] > 0)
        for (int k = 0; k < 3; ++k) R.bin_mean[size_t(i) * 3 + k] = mean_acc[size_t(i) * 3 + k] / mean_w[i];
    R.bin_empty_lm.assign(size_t(nlm) * n_bins, 0);
    for (int j = 0; j < nlm; ++j)
      for (int i = 0; i < n_bins; ++i)
        R.bin_empty_lm[size_t(j) * n_bins + i] = (R.bin_count[i] == 0 || R.bin_den[size_t(j) * n_bins + i] == 0.0);
    if (model) {
      // [B]_d = sqrt((2l+1)/4pi) sum w N_tri B / sum |Y|^2 N_tri (Eq. 13 with B in place of the estimate)
      R.model_pred.assign(size_t(nlm) * n_bins, std::nan(""));
      for (int j = 0; j < nlm; ++j)
        for (int i = 0; i < n_bins; ++i)
          if (!R.bin_empty_lm[size_t(j) * n_bins + i])
            R.model_pred[size_t(j) * n_bins + i] = pref[j] * model_num[size_t(j) * n_bins + i] / R.bin_den[size_t(j) * n_bins + i];
    }
  }
  for (size_t ip = 0; ip < pts.size(); ++ip) {
    std::vector<double>().swap(per_pt_d[ip]);
    std::vector<double>().swap(per_pt_kmt[ip]);
  }
  if (geometry_only) return "";

  // ---- K3 work items.  Pairs are (slot A ring, slot C ring); the MFMA N
  // dimension is the slot-B ring.  Per plane triple, the kept slot-B rings of
  // every pair are cut into windows of kTileN consecutive rings (segments); a
  // segment is summed on the largest grid its combinations need.  Segments
  // are packed into items of up to ppi pairs sharing one window, grid by grid
  // from the largest down; the free rows of an item are then filled with
  // segments of smaller grids that fit its window (a larger grid is still
  // exact).  Items of one grid are finally gathered into workgroups of up to
  // kWavesPerGroup * items_per_wave items that share as many staged sides as
  // a greedy clustering finds, within max_group_sides sides.
  const int n_levels = int(T.grid_sizes.size());
  struct Seg {
    int level, ra, rc, lo, hi;
    std::vector<int> idx;
  };
  struct PItem {
    int32_t pt;
    int lo;
    std::vector<int> segs;
  };
  std::vector<std::vector<Seg>> pt_segs(pts.size());
  std::vector<std::vector<PItem>> level_items(n_levels);
  double useful = 0.0;
  for (size_t ip = 0; ip < pts.size(); ++ip) {
    auto& recs = per_pt[ip];
    if (recs.empty()) continue;
    auto& segs = pt_segs[ip];
    for (const ComboRec& cr : recs) {
      const double m = double(T.grid_sizes[cr.level]);
      useful += m * m;  // on the combination's own grid: the work the method needs
    }
    std::map<std::pair<int, int>, std::vector<int>> by_pair;  // (ra, rc) -> combos
    for (int i = 0; i < int(recs.size()); ++i) by_pair[{recs[i].ra, recs[i].rc}].push_back(i);
    std::vector<double> best;
    std::vector<int> cut;
    for (auto& kv : by_pair) {
      auto& v = kv.second;
      std::sort(v.begin(), v.end(), [&](int x, int y) { return recs[x].rb < recs[y].rb; });
      // Cut the pair's slot-B rings into windows spanning < kTileN rings, each
      // summed on its largest grid, minimising the total sum of m^2 (one row
      // of kTileN columns per window): best[i] covers the first i rings.
      const int nv = int(v.size());
      best.assign(nv + 1, 0.0);
      cut.assign(nv + 1, 0);
      for (int i = 1; i <= nv; ++i) {
        best[i] = 1e300;
        int lev = 0;
        for (int j = i - 1; j >= 0 && recs[v[i - 1]].rb - recs[v[j]].rb < kTileN; --j) {
          lev = std::max(lev, int(recs[v[j]].level));
          const double m = double(T.grid_sizes[lev]);
          if (best[j] + m * m < best[i]) {
            best[i] = best[j] + m * m;
            cut[i] = j;
          }
        }
      }
      std::vector<std::pair<int, int>> spans;
      for (int i = nv; i > 0; i = cut[i]) spans.push_back({cut[i], i});
      for (auto it = spans.rbegin(); it != spans.rend(); ++it) {
        Seg sg;
        sg.ra = kv.first.first;
        sg.rc = kv.first.second;
        sg.lo = recs[v[it->first]].rb;
        sg.level = 0;
        for (int q = it->first; q < it->second; ++q) {
          sg.level = std::max(sg.level, int(recs[v[q]].level));
          sg.idx.push_back(v[q]);
        }
        sg.hi = recs[sg.idx.back()].rb;
        segs.push_back(std::move(sg));
      }
    }
    // per level: segments sorted by (lo, hi, ra, rc)
    std::vector<std::vector<int>> by_level(n_levels);
    for (int sidx = 0; sidx < int(segs.size()); ++sidx) by_level[segs[sidx].level].push_back(sidx);
    for (auto& v : by_level)
      std::sort(v.begin(), v.end(), [&](int x, int y) {
        const Seg &sx = segs[x], &sy = segs[y];
        return sx.lo != sy.lo ? sx.lo < sy.lo : (sx.hi != sy.hi ? sx.hi < sy.hi : (sx.ra != sy.ra ? sx.ra < sy.ra : sx.rc < sy.rc));
      });
    std::vector<char> used(segs.size(), 0);
    for (int L = n_levels - 1; L >= 0; --L) {
      std::vector<PItem> its;
      for (int sidx : by_level[L]) {
        if (used[sidx]) continue;
        const Seg& sg = segs[sidx];
        if (its.empty() || int(its.back().segs.size()) == ppi || sg.hi >= its.back().lo + kTileN)
          its.push_back({int32_t(ip), sg.lo, {}});
        its.back().segs.push_back(sidx);
        used[sidx] = 1;
      }
      for (auto& it : its) {
        for (int l2 = L - 1; l2 >= 0 && int(it.segs.size()) < ppi; --l2) {
          const auto& v = by_level[l2];
          auto first = std::lower_bound(v.begin(), v.end(), it.lo, [&](int x, int lo) { return segs[x].lo < lo; });
          for (auto q = first; q != v.end() && segs[*q].lo < it.lo + kTileN && int(it.segs.size()) < ppi; ++q) {
            if (used[*q] || segs[*q].hi >= it.lo + kTileN) continue;
            it.segs.push_back(*q);
            used[*q] = 1;
          }
        }
        for (int sidx : it.segs) {
          segs[sidx].level = L;
          for (int ci : segs[sidx].idx) recs[ci].level = L;  // the grid the combination is summed on
        }
        level_items[L].push_back(std::move(it));
      }
    }
  }
  T.useful_terms = useful;

  std::vector<std::vector<int64_t>> pt_combo_slot(pts.size());
  for (size_t ip = 0; ip < pts.size(); ++ip) pt_combo_slot[ip].assign(per_pt[ip].size(), -1);
  std::map<std::pair<int32_t, int32_t>, int32_t> gside_tmp;  // (level, side) -> id in first-use order
  std::vector<std::pair<int32_t, int32_t>> gside_key;
  auto gside_id = [&](int32_t level, int32_t sidx) {
    auto it = gside_tmp.find({level, sidx});
    if (it != gside_tmp.end()) return it->second;
    const int32_t id = int32_t(gside_key.size());
    gside_tmp[{level, sidx}] = id;
    gside_key.push_back({level, sidx});
    return id;
  };
  // sides an item stages, and its slot-B rings kept by some pair (bit j: ring lo + j)
  auto item_sides = [&](const PItem& it, std::vector<int32_t>* out, uint32_t* b_used) {
    const int a = pts[it.pt].a, bb = pts[it.pt].b, c = a + bb;
    const auto& segs = pt_segs[it.pt];
    const auto& recs = per_pt[it.pt];
    uint32_t bu = 0;
    for (int sidx : it.segs) {
      out->push_back(side(segs[sidx].ra, a));
      out->push_back(side(segs[sidx].rc, c));
      for (int ci : segs[sidx].idx) bu |= 1u << (recs[ci].rb - it.lo);
    }
    for (int j = 0; j < kTileN; ++j)
      if (bu >> j & 1u) out->push_back(side(it.lo + j, bb));
    *b_used = bu;
  };
  // Items of one grid are ordered into workgroups: a group starts at the
  // first item not yet placed and repeatedly takes, among the next
  // kGroupLook unplaced items of the packing order, the one that adds the
  // fewest sides to the group (the earliest on ties), up to
  // kWavesPerGroup * ipw items and max_group_sides sides.  Fewer staged sides
  // per item means less staging traffic per term.  Each candidate's overlap
  // with the group is kept up to date through per-side lists of the items
  // that stage the side.
  constexpr size_t kGroupLook = 16384;
  auto cluster = [&](const std::vector<PItem>& in, std::vector<PItem>* out, std::vector<size_t>* ends) {
    const size_t n = in.size();
    std::vector<std::vector<int32_t>> isides(n);
    std::map<int32_t, std::vector<int32_t>> holders;  // side -> items staging it, ascending
    for (size_t i = 0; i < n; ++i) {
      uint32_t bu = 0;
      item_sides(in[i], &isides[i], &bu);
      std::sort(isides[i].begin(), isides[i].end());
      isides[i].erase(std::unique(isides[i].begin(), isides[i].end()), isides[i].end());
      for (int32_t x : isides[i]) holders[x].push_back(int32_t(i));
    }
    std::vector<char> placed(n, 0);
    std::vector<int32_t> overlap(n, 0);  // sides an item shares with the current group
    std::vector<int32_t> members;        // sides of the current group
    size_t first = 0;
    while (first < n) {
      members.clear();
      size_t nitems = 0;
      auto take = [&](size_t i) {
        for (int32_t x : isides[i]) {
          if (std::find(members.begin(), members.end(), x) != members.end()) continue;
          members.push_back(x);
          for (int32_t j : holders[x]) overlap[j] += 1;
        }
        placed[i] = 1;
        out->push_back(in[i]);
        ++nitems;
      };
      take(first);
      while (nitems < size_t(kWavesPerGroup * ipw)) {
        size_t best = n, seen = 0;
        int best_new = 1 << 30;
        for (size_t j = first + 1; j < n && seen < kGroupLook; ++j) {
          if (placed[j]) continue;
          ++seen;
          const int add = int(isides[j].size()) - overlap[j];
          if (add >= best_new || int(members.size()) + add > k3.max_group_sides) continue;
          best_new = add;
          best = j;
          if (add == 0) break;
        }
        if (best == n) break;
        take(best);
      }
      for (int32_t x : members)
        for (int32_t j : holders[x]) overlap[j] -= 1;
      ends->push_back(out->size());
      while (first < n && placed[first]) ++first;
    }
  };
  // levels are clustered independently, on the host threads
  std::vector<std::vector<PItem>> level_order(n_levels);
  std::vector<std::vector<size_t>> level_ends(n_levels);
  {
    std::atomic<int> next_level{0};
    std::vector<std::thread> workers;
    for (int t = 0; t < std::min(n_threads, n_levels); ++t)
      workers.emplace_back([&]() {
        for (int L = next_level.fetch_add(1); L < n_levels; L = next_level.fetch_add(1))
          cluster(level_items[L], &level_order[L], &level_ends[L]);
      });
    for (auto& w : workers) w.join();
  }
  for (int L = n_levels - 1; L >= 0; --L) {
    const std::vector<PItem>& its = level_order[L];
    const std::vector<size_t>& ends = level_ends[L];
    const int m = T.grid_sizes[L];
    size_t g0 = 0, gi = 0;
    while (g0 < its.size()) {
      std::vector<int32_t> gs;  // sorted, unique
      std::vector<uint32_t> b_used;
      size_t g1 = g0;
      const size_t gend = ends[gi];
      while (g1 < gend && g1 - g0 < size_t(kWavesPerGroup * ipw)) {
        std::vector<int32_t> add;
        uint32_t bu = 0;
        item_sides(its[g1], &add, &bu);
        std::vector<int32_t> merged(gs);
        merged.insert(merged.end(), add.begin(), add.end());
        std::sort(merged.begin(), merged.end());
        merged.erase(std::unique(merged.begin(), merged.end()), merged.end());
        if (g1 > g0 && int(merged.size()) > k3.max_group_sides) break;
        gs.swap(merged);
        b_used.push_back(bu);
        ++g1;
      }
      GroupDesc gd{};
      gd.side_begin = int32_t(T.group_sides.size());
      gd.item_begin = int32_t(T.items.size());
      gd.n_items = int32_t(g1 - g0);
      gd.conj_mask = 4;  // slot C is plane -(a+b); D(r, 0) is real, so conj is harmless on (0,0,0)
      gd.grid = m;
      // LDS slots: the group's sides numbered in (plane, ring) order, so rows
      // of a tile that read different rings of one plane read different banks.
      std::sort(gs.begin(), gs.end(), [&](int32_t x, int32_t y) {
        return T.side_plane[x] != T.side_plane[y] ? T.side_plane[x] < T.side_plane[y] : T.side_ring[x] < T.side_ring[y];
      });
      std::map<int32_t, int> lds;  // side index -> slot
      for (size_t k = 0; k < gs.size(); ++k) {
        lds[gs[k]] = int(k);
        T.group_sides.push_back(gside_id(L, gs[k]));
      }
      const int zero_slot = int(gs.size());
      if (zero_slot > 255) return "too many sides in one workgroup";
      gd.n_sides = zero_slot;
      auto slot = [&](int32_t sidx) -> uint8_t { return uint8_t(lds.at(sidx)); };
      for (size_t ii = g0; ii < g1; ++ii) {
        const PItem& it = its[ii];
        const int a = pts[it.pt].a, bb = pts[it.pt].b, c = a + bb;
        const auto& segs = pt_segs[it.pt];
        const auto& recs = per_pt[it.pt];
        ItemDesc d;
        for (int p = 0; p < ppi; ++p) {
          if (p < int(it.segs.size())) {
            d.a_slot[p] = slot(side(segs[it.segs[p]].ra, a));
            d.c_slot[p] = slot(side(segs[it.segs[p]].rc, c));
          } else {
            d.a_slot[p] = d.c_slot[p] = uint8_t(zero_slot);
          }
        }
        for (int p = ppi; p < kMaxPairsPerItem; ++p) d.a_slot[p] = d.c_slot[p] = uint8_t(zero_slot);
        const uint32_t bu = b_used[ii - g0];
        for (int j = 0; j < kTileN; ++j) d.b_slot[j] = (bu >> j & 1u) ? slot(side(it.lo + j, bb)) : uint8_t(zero_slot);
        const int64_t item_index = int64_t(T.items.size());
        auto& slot_of = pt_combo_slot[it.pt];
        for (int p = 0; p < int(it.segs.size()); ++p)
          for (int ci : segs[it.segs[p]].idx)
            slot_of[ci] = item_index * T.s_per_item + int64_t(p) * kTileN + (recs[ci].rb - it.lo);
        T.items.push_back(d);
        T.dense_terms += double(ppi) * kTileN * double(m) * double(m);
      }
      // LDS swizzle keys: unit u of slot s sits at u ^ key(s), and one 16-byte
      // read serves the 16 rows (or columns) of a tile together, so slots read
      // by the same tile should carry different keys.  Greedy colouring of the
      // slots (zero slot included) with kKeys keys by how often two of them
      // share a tile.
      {
        const int nv = zero_slot + 1;
        std::vector<int32_t> w(size_t(nv) * nv, 0);
        int phase[kTileN];
        auto add_phase = [&](int n) {
          std::sort(phase, phase + n);
          n = int(std::unique(phase, phase + n) - phase);
          for (int x = 0; x < n; ++x)
            for (int y = 0; y < n; ++y)
              if (x != y) w[size_t(phase[x]) * nv + phase[y]] += 1;
        };
        for (int64_t ii = T.items.size() - (g1 - g0); ii < int64_t(T.items.size()); ++ii) {
          const ItemDesc& d = T.items[ii];
          for (int h = 0; h < ppi / kTileN; ++h) {
            for (int r = 0; r < kTileN; ++r) phase[r] = d.a_slot[kTileN * h + r];
            add_phase(kTileN);
            for (int r = 0; r < kTileN; ++r) phase[r] = d.c_slot[kTileN * h + r];
            add_phase(kTileN);
          }
          for (int r = 0; r < kTileN; ++r) phase[r] = d.b_slot[r];
          add_phase(kTileN);
        }
        std::vector<int64_t> deg(nv, 0);
        for (int x = 0; x < nv; ++x)
          for (int y = 0; y < nv; ++y) deg[x] += w[size_t(x) * nv + y];
        std::vector<int> order(nv);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return deg[x] > deg[y]; });
        std::vector<int> key(nv, -1);
        auto best_key = [&](int x) {
          int64_t best = -1;
          int bk = 0;
          for (int k = 0; k < kKeys; ++k) {
            int64_t c = 0;
            for (int y = 0; y < nv; ++y)
              if (y != x && key[y] == k) c += w[size_t(x) * nv + y];
            if (best < 0 || c < best) {
              best = c;
              bk = k;
            }
          }
          return bk;
        };
        for (int x : order) key[x] = best_key(x);
        for (int sweep = 0; sweep < 3; ++sweep)
          for (int x : order) key[x] = best_key(x);
        for (int k = 0; k < zero_slot; ++k) T.group_sides[gd.side_begin + k] |= key[k] << kKeyShift;
        gd.zero_key = key[zero_slot];
      }
      T.max_group_sides = std::max(T.max_group_sides, zero_slot + 1);
      T.groups.push_back(gd);
      if (g1 == gend) ++gi;
      g0 = g1;
    }
  }
  std::vector<std::vector<Seg>>().swap(pt_segs);
  std::vector<std::vector<PItem>>().swap(level_items);

  // ---- grid sides in (level, side) order and their offsets in D
  {
    std::vector<int32_t> order(gside_key.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return gside_key[x] < gside_key[y]; });
    std::vector<int32_t> remap(order.size());
    const int n_levels = int(T.grid_sizes.size());
    T.level_gside_begin.assign(n_levels + 1, 0);
    int64_t off = 0;
    for (size_t k = 0; k < order.size(); ++k) {
      const auto& key = gside_key[order[k]];
      remap[order[k]] = int32_t(k);
      T.gside_level.push_back(key.first);
      T.gside_side.push_back(key.second);
      T.gside_off.push_back(off);
      const int64_t m = T.grid_sizes[key.first];
      off += m * m;
      T.level_gside_begin[key.first + 1] += 1;
    }
    for (int L = 0; L < n_levels; ++L) T.level_gside_begin[L + 1] += T.level_gside_begin[L];
    T.d_elems = off;
    if (order.size() >= (size_t(1) << kKeyShift)) return "too many grid sides";
    const int32_t low = (int32_t(1) << kKeyShift) - 1;
    for (auto& g : T.group_sides) g = remap[g & low] | (g & ~low);
  }

  // ---- per-combination coefficients of every resolution in its bin order
  // (counting sort, stable in pt order)
  std::vector<std::vector<int64_t>> fill(n_res);
  for (int r = 0; r < n_res; ++r) {
    Resolution& R = T.res[r];
    const int n_bins = R.n_bins();
    R.bin_ptr.assign(n_bins + 1, 0);
    for (size_t ip = 0; ip < pts.size(); ++ip)
      for (size_t i = 0; i < per_pt[ip].size(); ++i) R.bin_ptr[bin_of(r, ip, i) + 1] += 1;
    for (int i = 0; i < n_bins; ++i) R.bin_ptr[i + 1] += R.bin_ptr[i];
    fill[r].assign(R.bin_ptr.begin(), R.bin_ptr.end() - 1);
    R.combo_slot.resize(total);
    R.combo_coef.resize(size_t(total) * nlm);
  }
  for (size_t ip = 0; ip < pts.size(); ++ip) {
    for (int r = 0; r < n_res; ++r) {
      Resolution& R = T.res[r];
      const int n_bins = R.n_bins();
      for (size_t i = 0; i < per_pt[ip].size(); ++i) {
        const ComboRec& cr = per_pt[ip][i];
        const int bin = bin_of(r, ip, i);
        const int64_t pos = fill[r][bin]++;
        const double mg = double(T.grid_sizes[cr.level]);
        const double grid_scale = (double(ng) * double(ng)) / (mg * mg);  // S on the m-grid is (m/N_g)^2 S
        R.combo_slot[pos] = pt_combo_slot[ip][i];
        for (int j = 0; j < nlm; ++j) {
          const double den = R.bin_den[size_t(j) * n_bins + bin];
          R.combo_coef[size_t(pos) * nlm + j] =
              den > 0 ? pref[j] * double(cr.mult) * per_pt_w[ip][i * nlm + j] / den * grid_scale : 0.0;
        }
      }
    }
    std::vector<ComboRec>().swap(per_pt[ip]);
    std::vector<int32_t>().swap(per_pt_xbin[ip]);
    std::vector<double>().swap(per_pt_w[ip]);
    std::vector<int64_t>().swap(pt_combo_slot[ip]);
  }
  // within each bin, order the combinations by output slot (locality of the S gather)
  std::vector<int64_t> idx;
  std::vector<int64_t> tmp_slot;
  std::vector<double> tmp_coef;
  for (int r = 0; r < n_res; ++r) {
    Resolution& R = T.res[r];
    for (int bin = 0; bin < R.n_bins(); ++bin) {
      const int64_t c0 = R.bin_ptr[bin], c1 = R.bin_ptr[bin + 1];
      if (c1 - c0 < 2) continue;
      idx.resize(c1 - c0);
      for (int64_t i = 0; i < c1 - c0; ++i) idx[i] = c0 + i;
      std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return R.combo_slot[x] < R.combo_slot[y]; });
      tmp_slot.resize(c1 - c0);
      for (int64_t i = 0; i < c1 - c0; ++i) tmp_slot[i] = R.combo_slot[idx[i]];
      std::copy(tmp_slot.begin(), tmp_slot.end(), R.combo_slot.begin() + c0);
      tmp_coef.resize(size_t(c1 - c0) * nlm);
      for (int64_t i = 0; i < c1 - c0; ++i)
        for (int j = 0; j < nlm; ++j) tmp_coef[size_t(i) * nlm + j] = R.combo_coef[size_t(idx[i]) * nlm + j];
      std::copy(tmp_coef.begin(), tmp_coef.end(), R.combo_coef.begin() + size_t(c0) * nlm);
    }
  }
  return "";
}

// Gauss-Legendre nodes and weights on [-1, 1]: Newton iterations on P_n
// started from the asymptotic estimate of each root.
static void gauss_legendre(int n, std::vector<double>* x, std::vector<double>* w) {
  x->assign(n, 0.0);
  w->assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    (*x)[i] = -z;
    (*x)[n - 1 - i] = z;
    (*w)[i] = (*w)[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

std::vector<double> continuum_multipoles(int l_max, int m_max, double mu, double t, double beta) {
  // integrand: Y*_lm(p) prod_i (1 + beta mu_i^2), a polynomial of degree
  // l + 6 in p; 24 cos(theta) nodes and 48 phases integrate it exactly
  const int n_theta = 24, n_phi = 48;
  std::vector<double> x, wx;
  gauss_legendre(n_theta, &x, &wx);
  std::vector<int> ls, ms;
  for (int l = 0; l <= l_max; l += 2)
    for (int m = 0; m <= std::min(l, m_max); ++m) {
      ls.push_back(l);
      ms.push_back(m);
    }
  std::vector<double> out(ls.size(), 0.0);
  // Eq. 3: orientation cosines of the three sides
  const double s = std::sqrt(std::max(0.0, 1.0 - mu * mu));
  const double r3 = std::sqrt(1.0 - 2.0 * t * mu + t * t);
  std::vector<double> P;
  for (int it = 0; it < n_theta; ++it) {
    const double pz = x[it];
    const double st = std::sqrt(std::max(0.0, 1.0 - pz * pz));
    legendre_table(l_max, pz, &P);
    for (int ip = 0; ip < n_phi; ++ip) {
      const double phi = 2.0 * M_PI * ip / n_phi;
      const double px = st * std::cos(phi);
      const double mu1 = pz;
      const double mu2 = -mu * pz + s * px;
      const double mu3 = -((1.0 - t * mu) * pz + t * s * px) / r3;
      const double ang = (1.0 + beta * mu1 * mu1) * (1.0 + beta * mu2 * mu2) * (1.0 + beta * mu3 * mu3);
      for (size_t j = 0; j < ls.size(); ++j) {
        const double y = norm_lm(ls[j], ms[j]) * P[ls[j] * (l_max + 1) + ms[j]];
        out[j] += wx[it] * (2.0 * M_PI / n_phi) * y * std::cos(ms[j] * phi) * ang;
      }
    }
  }
  for (size_t j = 0; j < ls.size(); ++j) out[j] *= std::sqrt((2.0 * ls[j] + 1.0) / (4.0 * M_PI));
  return out;
}

}  // namespace bk
