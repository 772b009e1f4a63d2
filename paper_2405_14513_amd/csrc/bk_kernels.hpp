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

#include <type_traits>

#include "bk_fft.hpp"
#include "bk_tables.hpp"

namespace bk {

// ---------------------------------------------------------------- K1
// z pass: real input lines delta[b][x][y][:] (contiguous), `tb` consecutive y
// per block; writes F[b][n][x][y] for n < nkeep, scaled by `scale`.  The K1
// kernels take the length N at compile time (N = sh.n) or at run time (N = 0).
template <typename T, typename Tin, int N>
__global__ __launch_bounds__(256) void k1_z_kernel(const Tin* __restrict__ delta, cplx<T>* __restrict__ F,
                                                   const cplx<T>* __restrict__ tw, FftShape sh, int tb, int nkeep,
                                                   T scale) {
  extern __shared__ char smem_raw[];
  const int n = N > 0 ? N : sh.n;
  const int tb_shift = __builtin_ctz(unsigned(tb));  // tb is a power of two
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
  cplx<T>* res;
  if constexpr (N > 0)
    res = lds_fft_c<T, N>(b0, b1, tw_l, tb, ls);
  else
    res = lds_fft(b0, b1, tw_l, sh, tb, ls);
  cplx<T>* dst = F + size_t(b) * nkeep * n * n + size_t(x) * n + y0;
  for (int q = threadIdx.x; q < tb * nkeep; q += blockDim.x) {
    const int kz = q >> tb_shift, l = q & (tb - 1);
    dst[size_t(kz) * n * n + l] = res[l * ls + kz];
  }
}

// In-place transform of contiguous lines: line i of `lines` at base + i * n.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_rows_kernel(cplx<T>* __restrict__ data, const cplx<T>* __restrict__ tw,
                                                     FftShape sh, int tb, long lines_total) {
  extern __shared__ char smem_raw[];
  const int n = N > 0 ? N : sh.n;
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
  cplx<T>* res;
  if constexpr (N > 0)
    res = lds_fft_c<T, N>(b0, b1, tw_l, lines, ls);
  else
    res = lds_fft(b0, b1, tw_l, sh, lines, ls);
  for (int q = threadIdx.x; q < lines * n; q += blockDim.x) {
    const int l = q / n, i = q - l * n;
    base[q] = res[l * ls + i];
  }
}

// In-place transform of strided lines: for each plane p (grid.y), the lines are
// the columns c of an n x n array (element i at i * n + c); `tb` columns per block.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_cols_kernel(cplx<T>* __restrict__ data, const cplx<T>* __restrict__ tw,
                                                     FftShape sh, int tb) {
  extern __shared__ char smem_raw[];
  const int n = N > 0 ? N : sh.n;
  const int tb_shift = __builtin_ctz(unsigned(tb));  // tb is a power of two
  const int ls = n + 1;  // padded line stride: transposed accesses hit different banks
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + n;
  cplx<T>* b1 = b0 + tb * ls;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tw_l[i] = tw[i];
  const int c0 = blockIdx.x * tb;
  cplx<T>* base = data + size_t(blockIdx.y) * n * n + c0;
  for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
    const int i = q >> tb_shift, l = q & (tb - 1);
    b0[l * ls + i] = base[size_t(i) * n + l];
  }
  __syncthreads();
  cplx<T>* res;
  if constexpr (N > 0)
    res = lds_fft_c<T, N>(b0, b1, tw_l, tb, ls);
  else
    res = lds_fft(b0, b1, tw_l, sh, tb, ls);
  for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
    const int i = q >> tb_shift, l = q & (tb - 1);
    base[size_t(i) * n + l] = res[l * ls + i];
  }
}

// ---------------------------------------------------------------- K2
// Ring sums on one grid level of size M: block = (grid side gs, TB
// consecutive columns y0..y0+TB-1).  The row transform restricted to the
// block's columns is a pruned DFT straight from the ring's modes,
// G(u_x, y) = sum_{u_y : (u_x,u_y) in ring} Delta(u, n) e^{-2 pi i u_y y / M},
// then the column FFT over u_x (placed at u_x mod M) runs in place in one LDS
// buffer, and D is written at gside_off[gs] + x M + y.  Delta is read from the N_g-point
// planes.  Every ring reaching this level has 2 U < M, so no two modes share
// a position.  ring_mode_uy holds each ring's modes sorted by (u_x, u_y);
// ring_seg gives, per ring, the start of every row u_x = -U..U (2U + 2
// offsets from ring_seg_off[r]).
//
// One work item of the row transform = the two rows +u_x and -u_x (the ring is
// symmetric, so both hold the same u_y) and kK2Cols columns.  A row's u_y are
// symmetric, [-b, b] or [-b, -b + h - 1] and [b - h + 1, b] with h = cnt / 2
// (checked when the plan is built), so they follow from its first mode, and
// the four modes (+-u_x, +-v) share one twiddle w^{v y} = c - i s:
// F(v) w^{v y} + F(-v) w^{-v y} = c S - i s A with S = F(v) + F(-v),
// A = F(v) - F(-v).  The twiddle index advances by y per v.
constexpr int kK2Cols = 4;      // columns per work item of the row transform
constexpr int kK2Threads = 256;  // threads per block

template <typename T, int M, int TB>
__global__ __launch_bounds__(kK2Threads) void k2_ring_kernel(const cplx<T>* __restrict__ F, cplx<T>* __restrict__ D,
                                                      const int32_t* __restrict__ gside_side,
                                                      const int64_t* __restrict__ gside_off, int gs_begin,
                                                      long d_elems, const int32_t* __restrict__ side_ring,
                                                      const int32_t* __restrict__ side_plane,
                                                      const int32_t* __restrict__ side_u,
                                                      const int32_t* __restrict__ ring_seg_off,
                                                      const int32_t* __restrict__ ring_seg,
                                                      const int16_t* __restrict__ ring_mode_uy, int ng, int nkeep,
                                                      const cplx<T>* __restrict__ tw) {
  static_assert(M % TB == 0 && TB % kK2Cols == 0, "the slab must divide the grid and hold whole column groups");
  constexpr unsigned LS = M + 1;  // padded line stride: transposed accesses hit different banks
  constexpr unsigned CG = TB / kK2Cols;  // column groups per slab
  constexpr unsigned YT = M / TB;        // slabs per grid side
  extern __shared__ char smem_raw[];
  cplx<T>* tw_l = reinterpret_cast<cplx<T>*>(smem_raw);
  cplx<T>* b0 = tw_l + M;  // TB lines of LS: the row transform's output, then the column FFT in place
  for (unsigned i = threadIdx.x; i < unsigned(M); i += blockDim.x) tw_l[i] = tw[i];
  const unsigned gs_rel = blockIdx.x / YT;
  const int gs = gs_begin + int(gs_rel);
  const unsigned y0 = (blockIdx.x - gs_rel * YT) * TB;
  const int b = blockIdx.y;
  const int s = gside_side[gs];
  const int r = side_ring[s];
  const int U = side_u[s];
  const cplx<T>* Fp = F + (size_t(b) * nkeep + side_plane[s]) * size_t(ng) * ng;
  const int32_t* seg = ring_seg + ring_seg_off[r - 1];
  // positions no row reaches: u_x in (U, M - U)
  for (unsigned q = threadIdx.x; q < unsigned(TB * M); q += blockDim.x) {
    const unsigned l = q / M, i = q - l * M;
    if (int(i) > U && int(i) < M - U) b0[l * LS + i] = {T(0), T(0)};
  }
  __syncthreads();
  const unsigned items = unsigned(U + 1) * CG;
  for (unsigned q = threadIdx.x; q < items; q += blockDim.x) {
    const int ux = int(q / CG);
    const unsigned cg = q - unsigned(ux) * CG;
    // columns y0 + cg + CG c, c < kK2Cols (interleaved: neighbouring threads write neighbouring lines)
    cplx<T> ap[kK2Cols], am[kK2Cols];
#pragma unroll
    for (int c = 0; c < kK2Cols; ++c) ap[c] = am[c] = {T(0), T(0)};
    const int m0 = seg[ux + U], cnt = seg[ux + U + 1] - m0;
    const cplx<T>* rp = Fp + size_t(ux) * ng;
    const cplx<T>* rm = Fp + size_t(ux > 0 ? ng - ux : 0) * ng;
    if (cnt > 0) {
      const int bmax = -int(ring_mode_uy[m0]);
      const bool one = cnt == 2 * bmax + 1;
      const int vlo = one ? 1 : bmax - cnt / 2 + 1;
      if (one) {
        const cplx<T> f0p = rp[0], f0m = rm[0];
#pragma unroll
        for (int c = 0; c < kK2Cols; ++c) {
          ap[c] = f0p;
          am[c] = f0m;
        }
      }
      unsigned yc[kK2Cols], e[kK2Cols];
#pragma unroll
      for (int c = 0; c < kK2Cols; ++c) {
        yc[c] = y0 + cg + CG * c;
        e[c] = (unsigned(vlo) * yc[c]) % unsigned(M);
      }
      // the loads of v + 1 are issued before the sums of v
      cplx<T> fpp = rp[vlo], fpm = rp[ng - vlo], fmp = rm[vlo], fmm = rm[ng - vlo];
      for (int v = vlo; v <= bmax; ++v) {
        const cplx<T> sp = cadd(fpp, fpm), dp = csub(fpp, fpm);
        const cplx<T> sm = cadd(fmp, fmm), dm = csub(fmp, fmm);
        const int vn = v < bmax ? v + 1 : v;
        fpp = rp[vn];
        fpm = rp[ng - vn];
        fmp = rm[vn];
        fmm = rm[ng - vn];
#pragma unroll
        for (int c = 0; c < kK2Cols; ++c) {
          const cplx<T> w = tw_l[e[c]];  // (c, -s)
          ap[c].x = fma(w.x, sp.x, ap[c].x);
          ap[c].x = fma(-w.y, dp.y, ap[c].x);
          ap[c].y = fma(w.x, sp.y, ap[c].y);
          ap[c].y = fma(w.y, dp.x, ap[c].y);
          am[c].x = fma(w.x, sm.x, am[c].x);
          am[c].x = fma(-w.y, dm.y, am[c].x);
          am[c].y = fma(w.x, sm.y, am[c].y);
          am[c].y = fma(w.y, dm.x, am[c].y);
          e[c] += yc[c];
          e[c] -= e[c] >= unsigned(M) ? unsigned(M) : 0u;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kK2Cols; ++c) {
      cplx<T>* line = b0 + (cg + CG * c) * LS;
      line[ux] = ap[c];
      if (ux > 0) line[M - ux] = am[c];
    }
  }
  __syncthreads();
  lds_fft_ip<T, M, TB, kK2Threads, LS>(b0, tw_l);
  cplx<T>* Ds = D + size_t(b) * d_elems + gside_off[gs] + y0;
  for (unsigned q = threadIdx.x; q < unsigned(TB * M); q += blockDim.x) {
    const unsigned x = q / TB, l = q - x * TB;
    Ds[size_t(x) * M + l] = b0[l * LS + x];
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

// LDS staging of the contraction.  A slot holds CH consecutive x_perp points
// of one side's D as 16-byte units (2 float32 or 1 float64 complex points),
// slot after slot with no padding, so whole 1 KiB lines are filled by direct
// global-to-LDS loads (64 lanes x 16 bytes, lane i to byte 16 i).  Unit u of
// slot s is stored at position u ^ key(s), with a 4-bit key per slot chosen on
// the host: the 16 rows of an MFMA tile that one 16-byte LDS read serves
// together fall in different banks whenever their slots' keys differ.
template <typename T, int CH>
struct K3Stage {
  static constexpr int cs = int(sizeof(cplx<T>));
  static constexpr int ppu = 16 / cs;           // points per 16-byte unit
  static constexpr int units = CH / ppu;        // units per slot
  static constexpr int slot_bytes = CH * cs;
  static constexpr int steps = units / 4;       // 16-byte reads per operand per chunk
  static constexpr bool valid = units >= 16 && units % 16 == 0;  // the swizzle needs 16 units per slot
};
constexpr int kK3Threads = 64 * kWavesPerGroup;
constexpr int kK3MaxLines = 8;  // 1 KiB staging lines per wave per chunk
// slots per staging buffer at a fixed buffer stride (159 sides and the zero slot)
constexpr int kK3FixedSlots = 160;

typedef double f64x2v __attribute__((ext_vector_type(2)));

template <typename T>
struct Unit;
template <>
struct Unit<float> {
  typedef f32x4 type;  // two complex points
};
template <>
struct Unit<double> {
  typedef f64x2v type;  // one complex point
};

// One block = one GroupDesc (items on one grid of m x m points that share
// the sides staged in LDS); wave w contracts items IPW w .. IPW w + IPW - 1,
// each 16 TPI ring pairs x 16 slot-B rings (TPI row tiles sharing the slot-B
// reads), TILES = TPI IPW row tiles in all.  The m^2 points are visited in
// chunks of CH: while the waves contract chunk c from one LDS buffer, the
// direct loads of chunk c+1 fill the other.  Per 16-byte unit step, lane
// (row, kq) reads unit 4 q + kq of its pair's A and C slots and of its
// column's B slot, forms the pair products P = D_A conj(D_C) and feeds
// Re P, -Im P against Re D_B, Im D_B into 16x16x4 MFMAs (K = the 4 points of
// the lanes' kq), one accumulator per row tile (Re S; with IMS a second one
// takes Re P Im D_B + Im P Re D_B = Im S); float32 units carry two points,
// i.e. two k-steps.  Float32 partial sums are added to float64 registers
// every 128 points; float64 accumulates in the MFMA registers.
//
// With two items per wave the Im S accumulators would take the kernel past
// 128 VGPRs, leaving room for one block per CU; that instance is held to four
// waves per SIMD (two blocks per CU) at the price of a few spilled registers.
template <typename T, int CH, int TPI, int IPW, bool IMS>
__global__ __launch_bounds__(kK3Threads) __attribute__((amdgpu_waves_per_eu(IMS && IPW == 2 && CH * 2 * sizeof(T) == 256 ? 4 : 1)))
void k3_contract_kernel(const cplx<T>* __restrict__ D, long d_elems,
                                                                 const int64_t* __restrict__ gside_off,
                                                                 const GroupDesc* __restrict__ groups,
                                                                 const ItemDesc* __restrict__ items,
                                                                 const int32_t* __restrict__ group_sides,
                                                                 double* __restrict__ S_out, long n_items_total) {
  using G = K3Stage<T, CH>;
  static_assert(G::valid, "the swizzle needs a multiple of 16 units per slot");
  typedef typename Unit<T>::type unit_t;
  constexpr int TILES = TPI * IPW;
  constexpr int kRe = 16 * TPI * kTileN;           // Re S outputs per item
  constexpr int kOut = kRe * (IMS ? 2 : 1);         // then Im S (odd l requested)
  extern __shared__ char smem_raw[];  // starts at LDS address 0 (no static LDS): 16-byte aligned
  const GroupDesc gd = groups[blockIdx.x];
  const int b = blockIdx.y;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int row = lane & 15;
  const int kq = lane >> 4;
  const char* Db = reinterpret_cast<const char*>(D + size_t(b) * d_elems);
  const int nchunks = int((long(gd.grid) * gd.grid) / CH);  // m^2 is a multiple of CH
  // With two items per wave and 256-byte slots the second buffer starts at a
  // fixed offset (kK3FixedSlots slots), so that every operand read is a
  // register plus an immediate offset; otherwise right after the first.
  constexpr int kFixedStride = (IPW == 2 && G::slot_bytes == 256) ? kK3FixedSlots * 256 : 0;
  const int buf_bytes = kFixedStride ? kFixedStride : (gd.n_sides + 1) * G::slot_bytes;
  const int data_bytes = gd.n_sides * G::slot_bytes;

  // the zero slot (last) of both buffers
  for (int i = threadIdx.x; i < G::slot_bytes / 16; i += kK3Threads) {
    reinterpret_cast<uint4*>(smem_raw + data_bytes)[i] = make_uint4(0u, 0u, 0u, 0u);
    reinterpret_cast<uint4*>(smem_raw + buf_bytes + data_bytes)[i] = make_uint4(0u, 0u, 0u, 0u);
  }

  // this wave's staging lines (wave, wave + waves, ...): per lane, the global
  // source of the 16 bytes it moves; null for lanes past the last slot
  const int n_lines = (data_bytes + 1023) >> 10;
  const char* src[kK3MaxLines];
#pragma unroll
  for (int i = 0; i < kK3MaxLines; ++i) {
    const int o = (wave + kWavesPerGroup * i) * 1024 + lane * 16;
    src[i] = nullptr;
    if (o < data_bytes) {
      const int sl = o / G::slot_bytes;
      const int32_t e = group_sides[gd.side_begin + sl];
      const int u = ((o - sl * G::slot_bytes) >> 4) ^ (e >> kKeyShift);  // key < 16 <= units
      src[i] = Db + (gside_off[e & ((1 << kKeyShift) - 1)] * G::cs + u * 16);
    }
  }
  auto issue = [&](int chunk, int sel) {
    char* dst = smem_raw + sel * buf_bytes;
#pragma unroll
    for (int i = 0; i < kK3MaxLines; ++i) {
      const int line = wave + kWavesPerGroup * i;
      if (line < n_lines && src[i])
        __builtin_amdgcn_global_load_lds(reinterpret_cast<const uint4*>(src[i] + long(chunk) * G::slot_bytes),
                                         reinterpret_cast<uint4*>(dst + line * 1024), 16, 0, 0);
    }
  };
  issue(0, 0);

  // Slot C always lies on plane -(a+b) <= 0 and is read as conj D(r, a+b); on
  // the (0,0,0) triple D(r, 0) is real, so the conjugate changes nothing.
  const int item0 = wave * IPW;  // this wave's first item in the group
  const bool active = item0 < gd.n_items;
  // per operand: the byte offset of its read at unit step q is o[q & 3] + 64 q
  // (unit 4 q + kq sits at position (4 q + kq) ^ key: the key's low two bits
  // permute kq, its high two bits permute q within each group of four steps)
  int ao[TILES][4], co[TILES][4], bo[IPW][4];
  auto offsets = [&](int slot, int (&o)[4]) {
    const int key = slot < gd.n_sides ? group_sides[gd.side_begin + slot] >> kKeyShift : gd.zero_key;
    const int base = slot * G::slot_bytes + 16 * (kq ^ (key & 3));
    const int k2 = key >> 2;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = base + 64 * ((j ^ k2) - j);
  };
  // an item past the group's last reads the zero slot and is not written
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    const bool live = item0 + i < gd.n_items;
    const ItemDesc* it = live ? &items[gd.item_begin + item0 + i] : nullptr;
#pragma unroll
    for (int u = 0; u < TPI; ++u) {
      offsets(live ? it->a_slot[16 * u + row] : gd.n_sides, ao[TPI * i + u]);
      offsets(live ? it->c_slot[16 * u + row] : gd.n_sides, co[TPI * i + u]);
    }
    offsets(live ? it->b_slot[row] : gd.n_sides, bo[i]);
  }

  typedef typename Mfma<T>::acc_t acc_t;
  // float64 accumulates in the MFMA registers throughout; float32 adds its
  // partial sums into float64 every kFlushPoints points
  constexpr int kFlushPoints = 128;
  constexpr int kFlush = sizeof(T) == 8 ? 0 : (kFlushPoints / CH > 1 ? kFlushPoints / CH : 1);
  // a float64 wave with one tile keeps the Re and Im products in two
  // accumulators, so consecutive MFMAs do not wait on each other
  constexpr int kChains = sizeof(T) == 8 && TILES == 1 ? 2 : 1;
  // with IMS, Im S = Re P Im D_B + Im P Re D_B in one more accumulator per tile
  constexpr int kImT = IMS ? TILES : 1;
  double out[TILES][4], out_im[kImT][4];
  acc_t acc[TILES][kChains], acc_im[kImT];
#pragma unroll
  for (int t = 0; t < TILES; ++t) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) acc[t][j] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) out[t][k] = 0.0;
  }
#pragma unroll
  for (int t = 0; t < kImT; ++t) {
    acc_im[t] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 4; ++k) out_im[t][k] = 0.0;
  }

  // Chunk c sits in buffer sel; with a fixed buffer stride the loop is unrolled
  // by two so that sel, and with it every LDS address offset, is a constant.
  auto run_chunk = [&](int c, auto sel_c) {
    constexpr int kSel = decltype(sel_c)::value;  // 0 or 1, or -1: c & 1 at run time
    const int sel = kSel >= 0 ? kSel : (c & 1);
    // chunk c has landed (each wave waits for its own loads, the barrier for
    // everyone's) and every wave is done with the buffer chunk c + 1 will fill
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (c + 1 < nchunks) issue(c + 1, 1 - sel);
    if (active) {
      const char* buf = smem_raw + (kSel >= 0 ? kSel * kFixedStride : sel * buf_bytes);
      unit_t a_n[TILES], c_n[TILES], b_n[IPW];
      auto load_step = [&](int q, unit_t* a, unit_t* cc, unit_t* bv) {
        const int shift = 64 * q;
#pragma unroll
        for (int i = 0; i < IPW; ++i) bv[i] = *reinterpret_cast<const unit_t*>(buf + bo[i][q & 3] + shift);
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
          a[t] = *reinterpret_cast<const unit_t*>(buf + ao[t][q & 3] + shift);
          cc[t] = *reinterpret_cast<const unit_t*>(buf + co[t][q & 3] + shift);
        }
      };
      load_step(0, a_n, c_n, b_n);
#pragma unroll
      for (int q = 0; q < G::steps; ++q) {
        unit_t a_c[TILES], c_c[TILES], b_c[IPW];
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
          a_c[t] = a_n[t];
          c_c[t] = c_n[t];
        }
#pragma unroll
        for (int i = 0; i < IPW; ++i) b_c[i] = b_n[i];
        if (q + 1 < G::steps) load_step(q + 1, a_n, c_n, b_n);
#pragma unroll
        for (int h = 0; h < G::ppu; ++h) {
          // P = D_A conj(D_C); Re(P D_B) = Re P Re D_B + (-Im P) Im D_B
          T pr[TILES], pn[TILES];
#pragma unroll
          for (int t = 0; t < TILES; ++t) {
            const T ar = a_c[t][2 * h], ai = a_c[t][2 * h + 1];
            const T cr = c_c[t][2 * h], ci = c_c[t][2 * h + 1];
            pr[t] = ar * cr + ai * ci;
            pn[t] = ar * ci - ai * cr;
          }
#pragma unroll
          for (int t = 0; t < TILES; ++t) acc[t][0] = Mfma<T>::step(pr[t], b_c[t / TPI][2 * h], acc[t][0]);
#pragma unroll
          for (int t = 0; t < TILES; ++t)
            acc[t][kChains - 1] = Mfma<T>::step(pn[t], b_c[t / TPI][2 * h + 1], acc[t][kChains - 1]);
          if constexpr (IMS) {
#pragma unroll
            for (int t = 0; t < TILES; ++t) acc_im[t] = Mfma<T>::step(pr[t], b_c[t / TPI][2 * h + 1], acc_im[t]);
#pragma unroll
            for (int t = 0; t < TILES; ++t) acc_im[t] = Mfma<T>::step(-pn[t], b_c[t / TPI][2 * h], acc_im[t]);
          }
        }
      }
      if constexpr (kFlush > 0) {
        if ((c + 1) % kFlush == 0 || c + 1 == nchunks) {
#pragma unroll
          for (int t = 0; t < TILES; ++t) {
#pragma unroll
            for (int k = 0; k < 4; ++k) out[t][k] += double(acc[t][0][k]);
            acc[t][0] = acc_t{0, 0, 0, 0};
          }
          if constexpr (IMS) {
#pragma unroll
            for (int t = 0; t < TILES; ++t) {
#pragma unroll
              for (int k = 0; k < 4; ++k) out_im[t][k] += double(acc_im[t][k]);
              acc_im[t] = acc_t{0, 0, 0, 0};
            }
          }
        }
      }
    }
  };
  if constexpr (kFixedStride > 0) {
    for (int c = 0; c < nchunks; c += 2) {
      run_chunk(c, std::integral_constant<int, 0>{});
      if (c + 1 < nchunks) run_chunk(c + 1, std::integral_constant<int, 1>{});
    }
  } else {
    for (int c = 0; c < nchunks; ++c) run_chunk(c, std::integral_constant<int, -1>{});
  }
  if constexpr (kFlush == 0) {
#pragma unroll
    for (int t = 0; t < TILES; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        out[t][k] = double(acc[t][0][k]);
        if constexpr (kChains == 2) out[t][k] += double(acc[t][1][k]);
      }
#pragma unroll
    for (int t = 0; t < kImT; ++t)
#pragma unroll
      for (int k = 0; k < 4; ++k) out_im[t][k] = double(acc_im[t][k]);
  }
#pragma unroll
  for (int i = 0; i < IPW; ++i) {
    if (item0 + i >= gd.n_items) break;
    double* o = S_out + (size_t(b) * n_items_total + gd.item_begin + item0 + i) * kOut;
#pragma unroll
    for (int u = 0; u < TPI; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int cell = (16 * u + Mfma<T>::out_row(kq, k)) * kTileN + row;
        o[cell] = out[TPI * i + u][k];
        if constexpr (IMS) o[kRe + cell] = out_im[TPI * i + u][k];
      }
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
// Second-level binning in two passes (Re S for even l, Im S for odd l).  The combinations of a bin are
// contiguous (sorted by output slot) and cut into chunks of at most
// kK4Chunk.  Pass 1: one wave per (chunk, field); lane l handles multipole
// j = l % G of combination first + l / G (G = 16, 32 or 64 >= n_lm), so one
// load reads 64 consecutive coefficients; lanes of one j are summed in a
// fixed butterfly order into part[field][chunk][j].  Pass 2: per (bin, field)
// the chunk partials are added in chunk order and scaled; empty bins are NaN.
constexpr int kK4Chunk = 1024;

template <int G, typename CT>
__global__ __launch_bounds__(64) void k4_partial_kernel(const double* __restrict__ S, long s_per_batch,
                                                        const long* __restrict__ chunk_begin,
                                                        const int32_t* __restrict__ combo_slot,
                                                        const CT* __restrict__ coef, int n_lm, long n_chunks,
                                                        unsigned long long odd_mask, long im_off,
                                                        double* __restrict__ part) {
  constexpr int per_iter = 64 / G;
  const long ch = blockIdx.x;
  const int b = blockIdx.y;
  const int lane = threadIdx.x;
  const int j = lane % G, cc = lane / G;
  const long c0 = chunk_begin[ch], c1 = chunk_begin[ch + 1];
  // odd l (bit j of odd_mask) take Im S, stored im_off after Re S
  const double* Sb = S + size_t(b) * s_per_batch + ((odd_mask >> j) & 1ull ? im_off : 0);
  double acc = 0.0;
  if (j < n_lm) {
#pragma unroll 4
    for (long c = c0 + cc; c < c1; c += per_iter) acc += double(coef[size_t(c) * n_lm + j]) * Sb[combo_slot[c]];
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
