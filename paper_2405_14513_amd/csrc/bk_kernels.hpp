// Device kernels of the estimator (gfx950).
//
//  K1  forward 3-D DFT of the field, three batched 1-D passes (z, then y, then x),
//      keeping only the k_parallel planes n = 0..nkeep-1 (Sec. II; negative
//      planes follow from Delta(u, -n) = conj Delta(-u, n)).
//  K2  ring sums D(r, n, x) of Eq. 9, per (side, column block): the row
//      transform restricted to the block's columns as a pruned DFT over the
//      ring's modes, then the column FFT over u_x in LDS.
//  K3  triple-product sums S(c) = sum_x D D D of Eq. 8 for every kept
//      combination, as MFMA 16x16x4 tiles: rows = (slot A, slot C) ring pairs,
//      columns = slot-B rings, K = x_perp points staged through LDS.
//  K4  second-level binning of Eq. 13: per bin, a fixed-order float64 sum of
//      coefficient x Re S over the bin's combinations.
#pragma once

#include <hip/hip_runtime.h>

#include "bk_fft.hpp"
#include "bk_tables.hpp"

namespace bk {

// ---------------------------------------------------------------- K1
// z pass: real input lines delta[b][x][y][:] (contiguous), `tb` consecutive y
// per block; writes F[b][n][x][y] for n < nkeep, scaled by `scale`.
template <typename T, typename Tin>
__global__ __launch_bounds__(256) void k1_z_kernel(const Tin* __restrict__ delta, cplx<T>* __restrict__ F,
                                                   const cplx<T>* __restrict__ tw, FftShape sh, int tb, int nkeep,
                                                   T scale) {
  extern __shared__ char smem_raw[];
  const int n = sh.n;
  const int ls = n + 1;  // padded line stride: transposed accesses hit different banks
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + n;
  cplx<T>* b1 = b0 + tb * ls;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw_l[i] = tw[i];
  const int ytiles = n / tb;
  const int x = blockIdx.x / ytiles;
  const int y0 = (blockIdx.x % ytiles) * tb;
  const int b = blockIdx.y;
  const size_t n3 = size_t(n) * n * n;
  const Tin* src = delta + size_t(b) * n3 + (size_t(x) * n + y0) * n;
  for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
    const int l = q / n, i = q - l * n;
    b0[l * ls + i] = {T(src[q]) * scale, T(0)};
  }
  __syncthreads();
  cplx<T>* res = lds_fft(b0, b1, tw_l, sh, tb, ls);
  cplx<T>* dst = F + size_t(b) * nkeep * n * n + size_t(x) * n + y0;
  for (int q = threadIdx.x; q < tb * nkeep; q += blockDim.x) {
    const int kz = q / tb, l = q - kz * tb;
    dst[size_t(kz) * n * n + l] = res[l * ls + kz];
  }
}

// In-place transform of contiguous lines: line i of `lines` at base + i * n.
template <typename T>
__global__ __launch_bounds__(256) void k_rows_kernel(cplx<T>* __restrict__ data, const cplx<T>* __restrict__ tw,
                                                     FftShape sh, int tb, long lines_total) {
  extern __shared__ char smem_raw[];
  const int n = sh.n;
  const int ls = n + 1;  // padded line stride: transposed accesses hit different banks
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + n;
  cplx<T>* b1 = b0 + tb * ls;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw_l[i] = tw[i];
  const long line0 = long(blockIdx.x) * tb;
  const int lines = int(min(long(tb), lines_total - line0));
  cplx<T>* base = data + line0 * n;
  for (int q = threadIdx.x; q < lines * n; q += blockDim.x) {
    const int l = q / n, i = q - l * n;
    b0[l * ls + i] = base[q];
  }
  __syncthreads();
  cplx<T>* res = lds_fft(b0, b1, tw_l, sh, lines, ls);
  for (int q = threadIdx.x; q < lines * n; q += blockDim.x) {
    const int l = q / n, i = q - l * n;
    base[q] = res[l * ls + i];
  }
}

// In-place transform of strided lines: for each plane p (grid.y), the lines are
// the columns c of an n x n array (element i at i * n + c); `tb` columns per block.
template <typename T>
__global__ __launch_bounds__(256) void k_cols_kernel(cplx<T>* __restrict__ data, const cplx<T>* __restrict__ tw,
                                                     FftShape sh, int tb) {
  extern __shared__ char smem_raw[];
  const int n = sh.n;
  const int ls = n + 1;  // padded line stride: transposed accesses hit different banks
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + n;
  cplx<T>* b1 = b0 + tb * ls;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw_l[i] = tw[i];
  const int c0 = blockIdx.x * tb;
  cplx<T>* base = data + size_t(blockIdx.y) * n * n + c0;
  for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
    const int i = q / tb, l = q - i * tb;
    b0[l * ls + i] = base[size_t(i) * n + l];
  }
  __syncthreads();
  cplx<T>* res = lds_fft(b0, b1, tw_l, sh, tb, ls);
  for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
    const int i = q / tb, l = q - i * tb;
    base[size_t(i) * n + l] = res[l * ls + i];
  }
}

// ---------------------------------------------------------------- K2
// Fused ring sums on one grid level of size m (sh.n): block = (grid side gs,
// tb consecutive columns y0..y0+tb-1).  Row transform restricted to the
// block's columns, straight from the ring's modes (pruned DFT):
// G(u_x, y) = sum_{u_y : (u_x,u_y) in ring} Delta(u, n) e^{-2 pi i u_y y / m},
// then the column FFT over u_x (placed at u_x mod m) in LDS, then D at
// gside_off[gs] + x m + y.  Delta is read from the N_g-point planes.  Every
// ring reaching this level has 2 U < m, so no two modes share a position.
// ring_mode_uy holds each ring's modes sorted by (u_x, u_y); ring_seg gives,
// per ring, the start of every row u_x = -U..U (2U + 2 offsets from ring_seg_off[r]).
template <typename T>
__global__ __launch_bounds__(256) void k2_fused_kernel(const cplx<T>* __restrict__ F, cplx<T>* __restrict__ D,
                                                       const int32_t* __restrict__ gside_side,
                                                       const int64_t* __restrict__ gside_off, int gs_begin,
                                                       long d_elems, const int32_t* __restrict__ side_ring,
                                                       const int32_t* __restrict__ side_plane,
                                                       const int32_t* __restrict__ side_u,
                                                       const int32_t* __restrict__ ring_seg_off,
                                                       const int32_t* __restrict__ ring_seg,
                                                       const int16_t* __restrict__ ring_mode_uy, int ng, int nkeep,
                                                       const cplx<T>* __restrict__ tw, FftShape sh, int tb) {
  extern __shared__ char smem_raw[];
  const int m = sh.n;
  const int ls = m + 1;
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + m;
  cplx<T>* b1 = b0 + tb * ls;
  for (int i = threadIdx.x; i < m; i += blockDim.x) tw_l[i] = tw[i];
  const int ytiles = m / tb;
  const int gs = gs_begin + int(blockIdx.x) / ytiles;
  const int y0 = (blockIdx.x % ytiles) * tb;
  const int b = blockIdx.y;
  const int s = gside_side[gs];
  const int r = side_ring[s];
  const int U = side_u[s];
  const cplx<T>* Fp = F + (size_t(b) * nkeep + side_plane[s]) * size_t(ng) * ng;
  const int32_t* seg = ring_seg + ring_seg_off[r - 1];
  for (int q = threadIdx.x; q < tb * m; q += blockDim.x) b0[(q / m) * ls + (q % m)] = {T(0), T(0)};
  __syncthreads();
  const int nrow = 2 * U + 1;
  const float inv_m = 1.0f / float(m);
  for (int q = threadIdx.x; q < nrow * tb; q += blockDim.x) {
    const int row = q / tb, l = q - row * tb;
    const int ux = row - U;
    const int y = y0 + l;
    const cplx<T>* Frow = Fp + size_t(ux < 0 ? ux + ng : ux) * ng;
    cplx<T> acc0 = {T(0), T(0)}, acc1 = {T(0), T(0)};
    const int m0 = seg[row], m1 = seg[row + 1];
    int k = m0;
    // (u_y y) mod m without an integer division: u_y y < 2^18, exact in float32 after correction
    auto term = [&](int kk) {
      const int uy = ring_mode_uy[kk];
      const int uyf = uy < 0 ? uy + ng : uy;
      const int t = (uy < 0 ? uy + m : uy) * y;
      int e = t - int(float(t) * inv_m) * m;
      e += e < 0 ? m : 0;
      e -= e >= m ? m : 0;
      return cmul(Frow[uyf], tw_l[e]);
    };
    for (; k + 1 < m1; k += 2) {
      acc0 = cadd(acc0, term(k));
      acc1 = cadd(acc1, term(k + 1));
    }
    if (k < m1) acc0 = cadd(acc0, term(k));
    b0[l * ls + (ux < 0 ? ux + m : ux)] = cadd(acc0, acc1);
  }
  __syncthreads();
  cplx<T>* res = lds_fft(b0, b1, tw_l, sh, tb, ls);
  cplx<T>* Ds = D + size_t(b) * d_elems + gside_off[gs];
  for (int q = threadIdx.x; q < tb * m; q += blockDim.x) {
    const int x = q / tb, l = q - x * tb;
    Ds[size_t(x) * m + y0 + l] = res[l * ls + x];
  }
}

// ---------------------------------------------------------------- K3
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

// Operands: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].  Result
// register k of lane l holds column l % 16 and row out_row(l / 16, k); the two
// instructions place rows differently (measured with mfma_probe_kernel).
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int kq, int k) { return 4 * kq + k; }
};

template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int kq, int k) { return 4 * k + kq; }
};

// LDS slot stride in complex elements: an odd number of 8-byte words between
// slots so the 16 rows of an MFMA tile, reading 16 different slots at one
// point, fall in different banks.
//
// float32: slot = CH interleaved complex values (8-byte reads), stride CH + 1.
// float64: slot = CH real parts then CH imaginary parts (two 8-byte reads per
// value instead of one 16-byte read), stride 2 CH + 1 doubles.
template <typename T, int CH>
struct K3Lds {
  static constexpr bool split = sizeof(T) == 8;
  static constexpr int stride = split ? 2 * CH + 1 : CH + 1;     // in units of T (split) or complex
  static constexpr int vec = 16 / int(sizeof(cplx<T>));          // complex per 16-byte global load
  static constexpr int per_side = CH / vec;                      // 16-byte loads per side per chunk
  static constexpr size_t slot_bytes = split ? size_t(stride) * sizeof(T) : size_t(stride) * sizeof(cplx<T>);
};
constexpr int kK3Threads = 64 * kItemsPerGroup;
constexpr int kK3MaxLoads = 8;  // 16-byte global loads per thread per chunk

// One block = one GroupDesc (all on one canonical plane triple and one grid
// of m x m points), one wave per work item of 16 * TILES ring pairs x 16
// slot-B rings.  Every CH points of x_perp the block stages the group's sides into LDS (16-byte loads, the next
// chunk prefetched into registers while the current one is consumed); each
// wave then forms the pair products P = D_A conj(D_C) (4 points per lane
// group) and feeds Re P, -Im P against Re D_B, Im D_B into 16x16x4 MFMAs
// (K = 4 points), one accumulator per row tile.  The chunk's partial sums are
// added to float64 registers.  Groups come largest grid first and, within a
// grid, in plane-triple order: the dispatcher deals consecutive blocks to the
// eight XCDs in turn, so every XCD gets an even share of each grid size, and
// groups that read the same sides run at about the same time.
template <typename T, int CH, int TILES>
__global__ __launch_bounds__(kK3Threads) void k3_contract_kernel(const cplx<T>* __restrict__ D, long d_elems,
                                                                 const int64_t* __restrict__ gside_off,
                                                                 const GroupDesc* __restrict__ groups,
                                                                 const ItemDesc* __restrict__ items,
                                                                 const int32_t* __restrict__ group_sides,
                                                                 double* __restrict__ S_out, long n_items_total) {
  using L = K3Lds<T, CH>;
  constexpr int kOut = 16 * TILES * kTileN;
  typedef uint4 v16;
  extern __shared__ char smem_raw[];
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem_raw);
  T* ldsr = reinterpret_cast<T*>(smem_raw);  // split layout view
  const GroupDesc gd = groups[blockIdx.x];
  const int b = blockIdx.y;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int row = lane & 15;
  const int kq = lane >> 4;
  const cplx<T>* Db = D + size_t(b) * d_elems;
  const long X = long(gd.grid) * gd.grid;  // the group's grid points (a multiple of CH)

  // zero slot
  if constexpr (L::split) {
    for (int i = threadIdx.x; i < L::stride; i += blockDim.x) ldsr[gd.n_sides * L::stride + i] = T(0);
  } else {
    for (int i = threadIdx.x; i < L::stride; i += blockDim.x) lds[gd.n_sides * L::stride + i] = {T(0), T(0)};
  }

  // this thread's staging loads: global source and LDS destination per chunk
  const v16* src[kK3MaxLoads];
  int dst[kK3MaxLoads];
  const int n_loads = gd.n_sides * L::per_side;
#pragma unroll
  for (int i = 0; i < kK3MaxLoads; ++i) {
    const int q = threadIdx.x + i * kK3Threads;
    const int qq = q < n_loads ? q : 0;
    const int sl = qq / L::per_side, v = qq - sl * L::per_side;
    src[i] = reinterpret_cast<const v16*>(Db + gside_off[group_sides[gd.side_begin + sl]] + v * L::vec);
    dst[i] = sl * L::stride + v * L::vec;
  }
  v16 stage[kK3MaxLoads];
#pragma unroll
  for (int i = 0; i < kK3MaxLoads; ++i)
    if (threadIdx.x + i * kK3Threads < n_loads) stage[i] = src[i][0];

  // Slot C always lies on plane -(a+b) <= 0 and is read as conj D(r, a+b); on
  // the (0,0,0) triple D(r, 0) is real, so the conjugate changes nothing.
  const bool active = wave < gd.n_items;
  int sa[TILES], sc[TILES], sb = 0;
#pragma unroll
  for (int t = 0; t < TILES; ++t) sa[t] = sc[t] = 0;
  if (active) {
    const ItemDesc& it = items[gd.item_begin + wave];
#pragma unroll
    for (int t = 0; t < TILES; ++t) {
      sa[t] = it.a_slot[16 * t + row] * L::stride;
      sc[t] = it.c_slot[16 * t + row] * L::stride;
    }
    sb = it.b_slot[row] * L::stride;
  }

  typedef typename Mfma<T>::acc_t acc_t;
  double out[TILES][4];
#pragma unroll
  for (int t = 0; t < TILES; ++t)
#pragma unroll
    for (int k = 0; k < 4; ++k) out[t][k] = 0.0;
  const long step = long(CH) / L::vec;  // 16-byte units per chunk
  for (long x0 = 0; x0 < X; x0 += CH) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int i = 0; i < kK3MaxLoads; ++i) {
      if (threadIdx.x + i * kK3Threads < n_loads) {
        // slots are 8-byte aligned only (odd stride): store 8 bytes at a time
        const cplx<T>* v = reinterpret_cast<const cplx<T>*>(&stage[i]);
        if constexpr (L::split) {
          ldsr[dst[i]] = v[0].x;
          ldsr[dst[i] + CH] = v[0].y;
        } else {
#pragma unroll
          for (int e = 0; e < L::vec; ++e) lds[dst[i] + e] = v[e];
        }
      }
    }
    __syncthreads();
    if (x0 + CH < X) {
#pragma unroll
      for (int i = 0; i < kK3MaxLoads; ++i) {
        if (threadIdx.x + i * kK3Threads < n_loads) {
          src[i] += step;
          stage[i] = src[i][0];
        }
      }
    }
    if (active) {
      // Software pipeline over the CH/4 k-steps: the LDS operands of step
      // ks+1 are read before the MFMAs of step ks are issued, and the pair
      // products of a step are formed into their own registers.
      acc_t acc[TILES];
#pragma unroll
      for (int t = 0; t < TILES; ++t) acc[t] = acc_t{0, 0, 0, 0};
      cplx<T> a_n[TILES], c_n[TILES], b_n;
      auto load_step = [&](int ks, cplx<T>* a, cplx<T>* c, cplx<T>& bvv) {
        const int xi = ks * 4 + kq;
        if constexpr (L::split) {
          bvv = {ldsr[sb + xi], ldsr[sb + CH + xi]};
#pragma unroll
          for (int t = 0; t < TILES; ++t) {
            a[t] = {ldsr[sa[t] + xi], ldsr[sa[t] + CH + xi]};
            c[t] = {ldsr[sc[t] + xi], ldsr[sc[t] + CH + xi]};
          }
        } else {
          bvv = lds[sb + xi];
#pragma unroll
          for (int t = 0; t < TILES; ++t) {
            a[t] = lds[sa[t] + xi];
            c[t] = lds[sc[t] + xi];
          }
        }
      };
      load_step(0, a_n, c_n, b_n);
#pragma unroll
      for (int ks = 0; ks < CH / 4; ++ks) {
        // P = D_A conj(D_C); Re(P D_B) = Re P Re D_B + (-Im P) Im D_B
        T pr[TILES], pn[TILES];
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
          pr[t] = a_n[t].x * c_n[t].x + a_n[t].y * c_n[t].y;
          pn[t] = a_n[t].x * c_n[t].y - a_n[t].y * c_n[t].x;
        }
        const T br = b_n.x, bi = b_n.y;
        if (ks + 1 < CH / 4) load_step(ks + 1, a_n, c_n, b_n);
#pragma unroll
        for (int t = 0; t < TILES; ++t) acc[t] = Mfma<T>::step(pr[t], br, acc[t]);
#pragma unroll
        for (int t = 0; t < TILES; ++t) acc[t] = Mfma<T>::step(pn[t], bi, acc[t]);
      }
#pragma unroll
      for (int t = 0; t < TILES; ++t)
#pragma unroll
        for (int k = 0; k < 4; ++k) out[t][k] += double(acc[t][k]);
    }
  }
  if (active) {
    double* o = S_out + (size_t(b) * n_items_total + gd.item_begin + wave) * kOut;
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) o[(16 * t + Mfma<T>::out_row(kq, k)) * kTileN + row] = out[t][k];
  }
}

// Layout probe: one wave, A[i][k] = i + 16 k, B[k][j] = (j == k).
template <typename T>
__global__ __launch_bounds__(64) void mfma_probe_kernel(double* out) {
  const int lane = threadIdx.x;
  const int row = lane & 15, kq = lane >> 4;
  const T a = T(row + 16 * kq);
  const T bv = T(row == kq ? 1 : 0);
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
  acc = Mfma<T>::step(a, bv, acc);
  for (int k = 0; k < 4; ++k) out[lane * 4 + k] = double(acc[k]);
}

// ---------------------------------------------------------------- K4
// Second-level binning in two passes.  The combinations of a bin are
// contiguous (sorted by output slot) and cut into chunks of at most
// kK4Chunk.  Pass 1: one wave per (chunk, field); lane l handles multipole
// j = l % G of combination first + l / G (G = 16, 32 or 64 >= n_lm), so one
// load reads 64 consecutive coefficients; lanes of one j are summed in a
// fixed butterfly order into part[field][chunk][j].  Pass 2: per (bin, field)
// the chunk partials are added in chunk order and scaled; empty bins are NaN.
constexpr int kK4Chunk = 1024;

template <int G>
__global__ __launch_bounds__(64) void k4_partial_kernel(const double* __restrict__ S, long s_per_batch,
                                                        const long* __restrict__ chunk_begin,
                                                        const int32_t* __restrict__ combo_slot,
                                                        const double* __restrict__ coef, int n_lm, long n_chunks,
                                                        double* __restrict__ part) {
  constexpr int per_iter = 64 / G;
  const long ch = blockIdx.x;
  const int b = blockIdx.y;
  const int lane = threadIdx.x;
  const int j = lane % G, cc = lane / G;
  const long c0 = chunk_begin[ch], c1 = chunk_begin[ch + 1];
  const double* Sb = S + size_t(b) * s_per_batch;
  double acc = 0.0;
  if (j < n_lm) {
#pragma unroll 4
    for (long c = c0 + cc; c < c1; c += per_iter) acc += coef[size_t(c) * n_lm + j] * Sb[combo_slot[c]];
  }
#pragma unroll
  for (int off = G; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  if (lane < n_lm) part[(size_t(b) * n_chunks + ch) * n_lm + lane] = acc;
}

__global__ __launch_bounds__(64) void k4_finish_kernel(const double* __restrict__ part, long n_chunks,
                                                       const long* __restrict__ bin_chunk,
                                                       const unsigned char* __restrict__ empty, int n_lm, int n_bins,
                                                       double norm, double* __restrict__ B) {
  const int bin = blockIdx.x;
  const int b = blockIdx.y;
  for (int j = threadIdx.x; j < n_lm; j += blockDim.x) {
    double acc = 0.0;
    for (long ch = bin_chunk[bin]; ch < bin_chunk[bin + 1]; ++ch) acc += part[(size_t(b) * n_chunks + ch) * n_lm + j];
    B[(size_t(b) * n_lm + j) * n_bins + bin] = empty[size_t(j) * n_bins + bin] ? __builtin_nan("") : norm * acc;
  }
}

}  // namespace bk
