// C ABI of the estimator: plan, device memory, launches (include/bk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bk.h"
#include "bk_kernels.hpp"
#include "bk_tables.hpp"

namespace {

thread_local std::string g_last_error;

bk_status fail(bk_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define BK_HIP(call)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess)                                                                                \
      return fail(e_ == hipErrorOutOfMemory ? BK_ERR_OOM : BK_ERR_HIP,                                   \
                  std::string(#call) + ": " + hipGetErrorString(e_));                                    \
  } while (0)

// Radices of an LDS FFT of length n = 2^a 3^b 5^c (a >= 1, b, c <= 1).
bool fft_shape(int n, bk::FftShape* sh) {
  sh->n = n;
  sh->nstages = 0;
  int m = n;
  if (m % 3 == 0) m /= 3;
  if (m % 5 == 0) m /= 5;
  if (m < 2 || (m & (m - 1)) != 0) return false;
  while (m % 4 == 0) {
    sh->radix[sh->nstages++] = 4;
    m /= 4;
  }
  if (m == 2) sh->radix[sh->nstages++] = 2;
  if (n % 3 == 0) sh->radix[sh->nstages++] = 3;
  if (n % 5 == 0) sh->radix[sh->nstages++] = 5;
  return true;
}

}  // namespace

// Device tables and outputs of the binning (K4) at one resolution.
struct K4Res {
  int n_bins = 0;
  long n_chunks = 0;
  long* d_chunk_begin = nullptr;  // combination index where each chunk starts [n_chunks + 1]
  long* d_bin_chunk = nullptr;    // first chunk of each bin [n_bins + 1]
  int32_t* d_combo_slot = nullptr;
  void* d_coef = nullptr;         // per-combination coefficients, float32 (BK_F32 plans) or float64
  unsigned char* d_empty = nullptr;
  double* d_part = nullptr;       // partial sums [max_batch][n_chunks][n_lm]
  double* d_B = nullptr;          // [max_batch][n_lm][n_bins]
};

struct bk_plan_s {
  bk::Tables tab;
  int prec = BK_F64;
  int device = 0;
  int max_batch = 1;
  int batch = 0;          // fields currently loaded
  int in_dtype = 0;       // dtype of the loaded fields
  int estimated = 0;      // a completed estimate is enqueued for `batch`
  hipStream_t stream = nullptr;
  size_t elem = 8;        // sizeof(complex T) / 2
  bk::FftShape sh{};
  int nkeep = 0;
  long n_sides = 0;
  long n_items = 0;
  double norm = 0.0;
  double delta_scale = 1.0;
  size_t lds_k3 = 0;
  int item_out = 512;     // float64 outputs per work item
  int fft_tb = 0;         // lines per block of the K1 passes (0 = default)
  int k2_tb = 0;          // columns per block of the ring sums (0 = default)
  int tuned = 0;          // tile choices came from bk_plan_autotune
  int k3_chunk = 32;
  size_t bytes = 0;

  void* d_in = nullptr;       // [max_batch][N^3] of the input dtype
  void* d_F = nullptr;        // [max_batch][nkeep][N][N] complex
  void* d_D = nullptr;        // [max_batch][d_elems] complex: every grid side's m x m points
  double* d_S = nullptr;      // [max_batch][n_items][512]
  void* d_tw = nullptr;       // twiddles, N complex
  void* d_tw_lv = nullptr;    // twiddles of every grid level, m complex each, at tw_lv_off
  std::vector<long> tw_lv_off;
  std::vector<bk::FftShape> lv_sh;
  int32_t* d_gs_side = nullptr;  // side of every grid side
  int64_t* d_gs_off = nullptr;   // offset of every grid side in a field's D
  bk::GroupDesc* d_groups = nullptr;
  bk::ItemDesc* d_items = nullptr;
  int32_t* d_group_sides = nullptr;
  int32_t* d_side_ring = nullptr;
  int32_t* d_side_plane = nullptr;
  int32_t* d_side_u = nullptr;
  int32_t* d_ring_seg_off = nullptr;  // per ring: offset of its row table in d_ring_seg
  int32_t* d_ring_seg = nullptr;      // per ring: start of each row u_x = -U..U in the mode list, plus end
  int16_t* d_ring_mode_uy = nullptr;  // every ring's modes sorted by (u_x, u_y): u_y
  // the binning of every resolution (res[0]: the plan's binning)
  std::vector<K4Res> k4;
  // Stage events: launch_all records the five stage boundaries into `ev`,
  // which points at one of kEvSets sets used in turn by consecutive timed
  // estimates; ev_count sets (the latest ones) belong to timed estimates of
  // the current results (0 after a graph replay).
  static constexpr int kEvSets = 32;
  hipEvent_t evs[kEvSets][5] = {};
  hipEvent_t* ev = evs[0];
  int ev_next = 0;
  int ev_count = 0;
  bool have_events = false;
  int d_injected = 0;     // D was set by bk_debug_set_D: the next estimate starts at the contraction
  // bk_estimate replays the plan's kernels from a graph captured on cap_stream
  // for the launch configuration graph_key (recaptured when it changes)
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  std::array<long, 6> graph_key{};
};

namespace {

// Tuned tile choices, cached per (N_g, precision, device, sides, workgroups).
typedef std::tuple<int, int, int, long, long> TuneKey;
std::mutex g_tune_mutex;
std::map<TuneKey, std::array<int, 3>> g_tune_cache;

TuneKey tune_key(bk_plan p) {
  return TuneKey(p->sh.n, p->prec, p->device, p->n_sides, long(p->tab.groups.size()));
}

}  // namespace

namespace {

bk_status dalloc(bk_plan p, void** ptr, size_t bytes) {
  if (bytes == 0) bytes = 256;
  const char* cap = std::getenv("BK_MAX_DEVICE_BYTES");
  if (cap && p->bytes + bytes > size_t(std::strtoull(cap, nullptr, 10)))
    return fail(BK_ERR_OOM, "device allocation exceeds BK_MAX_DEVICE_BYTES");
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(e == hipErrorOutOfMemory ? BK_ERR_OOM : BK_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  p->bytes += bytes;
  return BK_OK;
}

template <typename V>
bk_status put(bk_plan p, V** dptr, const V* host, size_t count) {
  bk_status st = dalloc(p, reinterpret_cast<void**>(dptr), count * sizeof(V));
  if (st != BK_OK) return st;
  if (count) BK_HIP(hipMemcpy(*dptr, host, count * sizeof(V), hipMemcpyHostToDevice));
  return BK_OK;
}

void release(bk_plan p) {
  void* ptrs[] = {p->d_in,         p->d_F,          p->d_D,          p->d_S,
                  p->d_tw,         p->d_groups,     p->d_items,      p->d_group_sides,
                  p->d_side_ring,  p->d_side_plane, p->d_side_u,
                  p->d_ring_seg_off, p->d_ring_seg,
                  p->d_ring_mode_uy, p->d_tw_lv,   p->d_gs_side,  p->d_gs_off};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (K4Res& k : p->k4) {
    void* kp[] = {k.d_chunk_begin, k.d_bin_chunk, k.d_combo_slot, k.d_coef, k.d_empty, k.d_part, k.d_B};
    for (void* q : kp)
      if (q) (void)hipFree(q);
  }
  if (p->have_events)
    for (auto& set : p->evs)
      for (auto& e : set)
        if (e) (void)hipEventDestroy(e);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
}

// Device buffers one estimate reads and writes.  The plan's own (bk_estimate)
// or caller input/output with the library's static scratch
// (bk_estimate_noalloc).
struct Bufs {
  const void* in = nullptr;  // [batch][N^3] fields of in_dtype
  int in_dtype = 0;
  int batch = 0;
  void* F = nullptr;         // [batch][nkeep][N][N] complex
  void* D = nullptr;         // [batch][d_elems] complex
  double* S = nullptr;       // [batch][n_items][item_out]
  double* part = nullptr;    // [batch][n_chunks][n_lm] of the first resolution
  double* B = nullptr;       // [batch][n_lm][n_bins] of the first resolution
  bool first_res_only = false;  // bin at the first resolution only (else every resolution, into the plan's buffers)
  bool skip_fft = false;     // D is already set: run the contraction and the binning only
};

Bufs plan_bufs(bk_plan p) {
  Bufs b;
  b.in = p->d_in;
  b.in_dtype = p->in_dtype;
  b.batch = p->batch;
  b.F = p->d_F;
  b.D = p->d_D;
  b.S = p->d_S;
  b.part = p->k4[0].d_part;
  b.B = p->k4[0].d_B;
  b.skip_fft = p->d_injected != 0;
  return b;
}

template <typename T>
constexpr bool prec_is_f32() {
  return sizeof(T) == 4;
}

// LDS bytes of the contraction for a chunk of ch points (two buffers of every
// staged slot plus the zero slot; kK3FixedSlots slots each when the buffers
// sit at a fixed stride), 0 if the kernel has no instance for the chunk
// (float32: 32 or 64 points, float64: 16 or 32), if it does not divide every grid
// level's m^2 points, gives fewer than 16 16-byte units per slot, needs more
// staging lines than the kernel issues, or exceeds the 160 KiB of a CU.
size_t k3_lds_bytes(const bk::Tables& T, int prec, int ch) {
  // the chunks the contraction kernel is instantiated for
  if (prec == BK_F32 ? (ch != 32 && ch != 64) : (ch != 16 && ch != 32)) return 0;
  const size_t cs = prec == BK_F32 ? 8 : 16;
  const int units = int(size_t(ch) * cs / 16);
  if (units < 16 || units % 16 != 0) return 0;
  for (int m : T.grid_sizes)
    if ((long(m) * m) % ch != 0) return 0;
  const size_t slot = size_t(ch) * cs;
  if (size_t(T.max_group_sides - 1) * slot > size_t(bk::kK3MaxLines) * bk::kWavesPerGroup * 1024) return 0;
  // two items per wave with 256-byte slots: the kernel places its second
  // buffer kK3FixedSlots slots after the first
  if (T.k3.items_per_wave == 2 && slot == 256)
    return T.max_group_sides <= bk::kK3FixedSlots ? 2 * size_t(bk::kK3FixedSlots) * slot : 0;
  const size_t lds = 2 * size_t(T.max_group_sides) * slot;
  return lds <= 163840 ? lds : 0;
}

// LDS of the FFT kernels: n twiddles plus two buffers of tb lines padded to n + 1.
size_t fft_lds_bytes(int n, int tb, size_t elem_bytes) { return (size_t(n) + size_t(2) * tb * (n + 1)) * elem_bytes; }

int pick_tb(int n, size_t elem_bytes) {
  // lines per block: at most 16, dividing n, LDS at most 72 KiB (two blocks per CU)
  int tb = 16;
  while (tb > 1 && (fft_lds_bytes(n, tb, elem_bytes) > 73728 || n % tb != 0)) tb /= 2;
  return tb;
}

#define BK_K3(TT, CHV, TPI, IPW)                                                                                 \
  do {                                                                                                           \
    if (p->tab.bin.even_l_only)                                                                                  \
      hipLaunchKernelGGL((bk::k3_contract_kernel<TT, CHV, TPI, IPW, false>), g3, dim3(bk::kK3Threads), p->lds_k3, \
                         st, D, long(p->tab.d_elems), p->d_gs_off, p->d_groups, p->d_items, p->d_group_sides,      \
                         S, p->n_items);                                                                         \
    else                                                                                                         \
      hipLaunchKernelGGL((bk::k3_contract_kernel<TT, CHV, TPI, IPW, true>), g3, dim3(bk::kK3Threads), p->lds_k3,  \
                         st, D, long(p->tab.d_elems), p->d_gs_off, p->d_groups, p->d_items, p->d_group_sides,      \
                         S, p->n_items);                                                                         \
  } while (0)

// Contraction launch for the plan's item shape (row tiles per item, items per wave).
template <typename T, int CH>
void launch_k3_shape(bk_plan p, const bk::cplx<T>* D, double* S, dim3 g3, hipStream_t st) {
  const int tpi = p->tab.k3.pairs_per_item / bk::kTileN;
  if (p->tab.k3.items_per_wave == 2)
    BK_K3(T, CH, 1, 2);
  else if (tpi == 1)
    BK_K3(T, CH, 1, 1);
  else if (tpi == 2)
    BK_K3(T, CH, 2, 1);
  else
    BK_K3(T, CH, 4, 1);
}

// ... and the plan's chunk (one of the two k3_lds_bytes allows per precision).
bk_status launch_k3(bk_plan p, const bk::cplx<float>* D, double* S, dim3 g3, hipStream_t st) {
  if (p->k3_chunk == 64)
    launch_k3_shape<float, 64>(p, D, S, g3, st);
  else if (p->k3_chunk == 32)
    launch_k3_shape<float, 32>(p, D, S, g3, st);
  else
    return fail(BK_ERR_ARG, "internal: no float32 contraction instance for this chunk");
  return BK_OK;
}

bk_status launch_k3(bk_plan p, const bk::cplx<double>* D, double* S, dim3 g3, hipStream_t st) {
  if (p->k3_chunk == 32)
    launch_k3_shape<double, 32>(p, D, S, g3, st);
  else if (p->k3_chunk == 16)
    launch_k3_shape<double, 16>(p, D, S, g3, st);
  else
    return fail(BK_ERR_ARG, "internal: no float64 contraction instance for this chunk");
  return BK_OK;
}
#undef BK_K3

// The three K1 passes for a transform length N known at compile time (0: any).
template <typename T, int N>
void launch_k1(bk_plan p, const Bufs& bf, bk::cplx<T>* F, const bk::cplx<T>* tw, int tb, size_t lds, hipStream_t st) {
  const int n = p->sh.n;
  const int B = bf.batch;
  dim3 grid(n * (n / tb), B);
  if (bf.in_dtype == BK_F32)
    hipLaunchKernelGGL((bk::k1_z_kernel<T, float, N>), grid, dim3(256), lds, st,
                       reinterpret_cast<const float*>(bf.in), F, tw, p->sh, tb, p->nkeep, T(p->delta_scale));
  else
    hipLaunchKernelGGL((bk::k1_z_kernel<T, double, N>), grid, dim3(256), lds, st,
                       reinterpret_cast<const double*>(bf.in), F, tw, p->sh, tb, p->nkeep, T(p->delta_scale));
  const long lines = long(B) * p->nkeep * n;
  hipLaunchKernelGGL((bk::k_rows_kernel<T, N>), dim3((lines + tb - 1) / tb), dim3(256), lds, st, F, tw, p->sh, tb,
                     lines);
  hipLaunchKernelGGL((bk::k_cols_kernel<T, N>), dim3(n / tb, B * p->nkeep), dim3(256), lds, st, F, tw, p->sh, tb);
}

// LDS of the ring sums: m twiddles plus one buffer of tb lines padded to m + 1.
size_t k2_lds_bytes(int m, int tb, size_t elem_bytes) { return (size_t(m) + size_t(tb) * (m + 1)) * elem_bytes; }

// Columns per block of the ring sums on an m-point grid: the largest of 16,
// 8, 4 not above `want` that divides m and keeps the block's LDS within 40
// KiB (four blocks per compute unit), 4 at least.
int k2_slab(int m, int want, size_t elem_bytes) {
  int tb = want >= 16 ? 16 : want >= 8 ? 8 : 4;
  while (tb > 4 && (m % tb != 0 || k2_lds_bytes(m, tb, elem_bytes) > 40960)) tb /= 2;
  return tb;
}

template <typename T, int M, int TB>
void launch_k2_mt(bk_plan p, const Bufs& bf, const bk::cplx<T>* F, bk::cplx<T>* D, size_t L, int n_gs,
                  const bk::cplx<T>* tw, hipStream_t st) {
  if constexpr (M % TB == 0) {
    dim3 g2(unsigned(n_gs) * (M / TB), bf.batch);
    hipLaunchKernelGGL((bk::k2_ring_kernel<T, M, TB>), g2, dim3(bk::kK2Threads), k2_lds_bytes(M, TB, sizeof(bk::cplx<T>)), st,
                       F, D, p->d_gs_side, p->d_gs_off, p->tab.level_gside_begin[L], long(p->tab.d_elems),
                       p->d_side_ring, p->d_side_plane, p->d_side_u, p->d_ring_seg_off, p->d_ring_seg,
                       p->d_ring_mode_uy, p->sh.n, p->nkeep, tw);
  }
}

template <typename T, int M>
void launch_k2_m(bk_plan p, const Bufs& bf, const bk::cplx<T>* F, bk::cplx<T>* D, size_t L, int tb, int n_gs,
                 const bk::cplx<T>* tw, hipStream_t st) {
  if (tb == 16)
    launch_k2_mt<T, M, 16>(p, bf, F, D, L, n_gs, tw, st);
  else if (tb == 8)
    launch_k2_mt<T, M, 8>(p, bf, F, D, L, n_gs, tw, st);
  else
    launch_k2_mt<T, M, 4>(p, bf, F, D, L, n_gs, tw, st);
}

// The ring sums of grid level L (m points, slabs of tb columns); one kernel
// instance per grid size the tables can produce.
template <typename T>
bk_status launch_k2(bk_plan p, const Bufs& bf, const bk::cplx<T>* F, bk::cplx<T>* D, size_t L, int m, int tb,
                    int n_gs, const bk::cplx<T>* tw, hipStream_t st) {
  if (m % tb != 0) return fail(BK_ERR_ARG, "internal: ring-sum slab does not divide the grid");
  switch (m) {
    case 8: launch_k2_m<T, 8>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 16: launch_k2_m<T, 16>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 24: launch_k2_m<T, 24>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 32: launch_k2_m<T, 32>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 40: launch_k2_m<T, 40>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 48: launch_k2_m<T, 48>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 64: launch_k2_m<T, 64>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 80: launch_k2_m<T, 80>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 96: launch_k2_m<T, 96>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 128: launch_k2_m<T, 128>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 160: launch_k2_m<T, 160>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 192: launch_k2_m<T, 192>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 256: launch_k2_m<T, 256>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 320: launch_k2_m<T, 320>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 384: launch_k2_m<T, 384>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    case 512: launch_k2_m<T, 512>(p, bf, F, D, L, tb, n_gs, tw, st); break;
    default: return fail(BK_ERR_ARG, "internal: no ring-sum kernel for grid size " + std::to_string(m));
  }
  return BK_OK;
}

// K1 and K2: the forward FFT of the fields, then the ring sums D of every
// grid side (ev[1] between them when timing).
template <typename T>
bk_status launch_fft(bk_plan p, const Bufs& bf, hipStream_t st, bool timing) {
  using C = bk::cplx<T>;
  const int n = p->sh.n;
  const int B = bf.batch;
  const size_t cs = sizeof(C);
  const int tb = p->fft_tb > 0 ? p->fft_tb : pick_tb(n, cs);
  const size_t lds_fft = fft_lds_bytes(n, tb, cs);
  const C* tw = reinterpret_cast<const C*>(p->d_tw);
  C* F = reinterpret_cast<C*>(bf.F);
  C* D = reinterpret_cast<C*>(bf.D);
  // K1: z pass (real input), y rows, x columns; one instance per supported N_g
  switch (n) {
    case 8: launch_k1<T, 8>(p, bf, F, tw, tb, lds_fft, st); break;
    case 16: launch_k1<T, 16>(p, bf, F, tw, tb, lds_fft, st); break;
    case 24: launch_k1<T, 24>(p, bf, F, tw, tb, lds_fft, st); break;
    case 32: launch_k1<T, 32>(p, bf, F, tw, tb, lds_fft, st); break;
    case 48: launch_k1<T, 48>(p, bf, F, tw, tb, lds_fft, st); break;
    case 64: launch_k1<T, 64>(p, bf, F, tw, tb, lds_fft, st); break;
    case 96: launch_k1<T, 96>(p, bf, F, tw, tb, lds_fft, st); break;
    case 128: launch_k1<T, 128>(p, bf, F, tw, tb, lds_fft, st); break;
    case 192: launch_k1<T, 192>(p, bf, F, tw, tb, lds_fft, st); break;
    case 256: launch_k1<T, 256>(p, bf, F, tw, tb, lds_fft, st); break;
    case 384: launch_k1<T, 384>(p, bf, F, tw, tb, lds_fft, st); break;
    case 512: launch_k1<T, 512>(p, bf, F, tw, tb, lds_fft, st); break;
    default: launch_k1<T, 0>(p, bf, F, tw, tb, lds_fft, st);
  }
  BK_HIP(hipGetLastError());
  if (timing) BK_HIP(hipEventRecord(p->ev[1], st));
  // K2: ring sums, pruned row DFT + column FFT per (grid side, column slab), one launch per grid level
  {
    const C* twl = reinterpret_cast<const C*>(p->d_tw_lv);
    const auto& lvb = p->tab.level_gside_begin;
    for (size_t L = 0; L + 1 < lvb.size(); ++L) {
      const int n_gs = lvb[L + 1] - lvb[L];
      if (n_gs == 0) continue;
      const int m = p->tab.grid_sizes[L];
      const int tb2 = k2_slab(m, p->k2_tb > 0 ? p->k2_tb : 16, cs);
      bk_status s2 = launch_k2<T>(p, bf, F, D, L, m, tb2, n_gs, twl + p->tw_lv_off[L], st);
      if (s2 != BK_OK) return s2;
      BK_HIP(hipGetLastError());
    }
  }
  return BK_OK;
}

template <typename T>
bk_status launch_all(bk_plan p, const Bufs& bf, hipStream_t st, bool timing) {
  using C = bk::cplx<T>;
  const int B = bf.batch;
  const C* D = reinterpret_cast<const C*>(bf.D);

  if (timing) BK_HIP(hipEventRecord(p->ev[0], st));
  if (!bf.skip_fft) {
    bk_status s12 = launch_fft<T>(p, bf, st, timing);
    if (s12 != BK_OK) return s12;
  } else if (timing) {
    BK_HIP(hipEventRecord(p->ev[1], st));
  }
  if (timing) BK_HIP(hipEventRecord(p->ev[2], st));
  // K3: triple products
  if (!p->tab.groups.empty()) {
    dim3 g3(p->tab.groups.size(), B);
    bk_status s3 = launch_k3(p, D, bf.S, g3, st);
    if (s3 != BK_OK) return s3;
    BK_HIP(hipGetLastError());
  }
  if (timing) BK_HIP(hipEventRecord(p->ev[3], st));
  // K4: binning, at every resolution
  const int nlm = int(p->tab.lm_l.size());
  unsigned long long odd_mask = 0;
  for (int j = 0; j < nlm; ++j)
    if (p->tab.lm_l[j] % 2) odd_mask |= 1ull << j;
  const long s_per = p->n_items * long(p->item_out);
  const long im_off = long(p->tab.k3.pairs_per_item) * bk::kTileN;  // Im S follows Re S in every item
  const size_t n_res = bf.first_res_only ? 1 : p->k4.size();
  for (size_t r = 0; r < n_res; ++r) {
    const K4Res& k = p->k4[r];
    double* part = r == 0 ? bf.part : k.d_part;
    double* Bout = r == 0 ? bf.B : k.d_B;
    const T* coef = reinterpret_cast<const T*>(k.d_coef);
    if (k.n_chunks > 0) {
      dim3 gp(k.n_chunks, B);
      if (nlm <= 16)
        hipLaunchKernelGGL((bk::k4_partial_kernel<16, T>), gp, dim3(64), 0, st, bf.S, s_per, k.d_chunk_begin,
                           k.d_combo_slot, coef, nlm, k.n_chunks, odd_mask, im_off, part);
      else if (nlm <= 32)
        hipLaunchKernelGGL((bk::k4_partial_kernel<32, T>), gp, dim3(64), 0, st, bf.S, s_per, k.d_chunk_begin,
                           k.d_combo_slot, coef, nlm, k.n_chunks, odd_mask, im_off, part);
      else
        hipLaunchKernelGGL((bk::k4_partial_kernel<64, T>), gp, dim3(64), 0, st, bf.S, s_per, k.d_chunk_begin,
                           k.d_combo_slot, coef, nlm, k.n_chunks, odd_mask, im_off, part);
      BK_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(bk::k4_finish_kernel, dim3(k.n_bins, B), dim3(64), 0, st, part, k.n_chunks, k.d_bin_chunk,
                       k.d_empty, nlm, k.n_bins, p->norm, Bout);
    BK_HIP(hipGetLastError());
  }
  if (timing) BK_HIP(hipEventRecord(p->ev[4], st));
  return BK_OK;
}

// Capture the plan's launches (full path, no stage events) into its graph,
// unless the graph already matches the launch configuration.
bk_status plan_graph(bk_plan p) {
  const std::array<long, 6> key = {long(p->batch), long(p->in_dtype), long(p->fft_tb), long(p->k2_tb),
                                   long(p->k3_chunk), long(p->lds_k3)};
  if (p->graph_exec && key == p->graph_key) return BK_OK;
  if (!p->cap_stream) BK_HIP(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
  if (p->graph_exec) {
    BK_HIP(hipGraphExecDestroy(p->graph_exec));
    p->graph_exec = nullptr;
  }
  if (p->graph) {
    BK_HIP(hipGraphDestroy(p->graph));
    p->graph = nullptr;
  }
  BK_HIP(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
  Bufs bf = plan_bufs(p);
  bf.skip_fft = false;
  bk_status st = p->prec == BK_F32 ? launch_all<float>(p, bf, p->cap_stream, false)
                                   : launch_all<double>(p, bf, p->cap_stream, false);
  hipGraph_t graph = nullptr;
  hipError_t he = hipStreamEndCapture(p->cap_stream, &graph);
  if (st != BK_OK || he != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return st != BK_OK ? st : fail(BK_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(he));
  }
  p->graph = graph;
  BK_HIP(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
  p->graph_key = key;
  return BK_OK;
}

}  // namespace

namespace {

// One eager estimate with stage events into the next event set.
bk_status timed_launch(bk_plan p, const Bufs& bf, hipStream_t st) {
  p->ev = p->evs[p->ev_next];
  bk_status s = p->prec == BK_F32 ? launch_all<float>(p, bf, st, true) : launch_all<double>(p, bf, st, true);
  if (s != BK_OK) return s;
  p->ev_next = (p->ev_next + 1) % bk_plan_s::kEvSets;
  p->ev_count = std::min(p->ev_count + 1, bk_plan_s::kEvSets);
  return BK_OK;
}

// Base and size (bytes) of a plan's device buffer for the loaded batch:
// 0 Delta planes, 1 D, 6 contraction outputs S.
void device_buffer(bk_plan p, int which, const void** src, size_t* bytes) {
  const size_t cs = 2 * p->elem;
  const size_t n2 = size_t(p->sh.n) * p->sh.n;
  const size_t b = size_t(std::max(p->batch, 0));
  if (which == 0) {
    *src = p->d_F;
    *bytes = b * p->nkeep * n2 * cs;
  } else if (which == 1) {
    *src = p->d_D;
    *bytes = b * size_t(p->tab.d_elems) * cs;
  } else {
    *src = p->d_S;
    *bytes = b * size_t(p->n_items) * size_t(p->item_out) * sizeof(double);
  }
}

}  // namespace

extern "C" const char* bk_last_error(void) { return g_last_error.c_str(); }

namespace {

bk_status check_binning(const bk_binning* bn, bk::FftShape* sh, bk::Binning* b) {
  if (bn->ng < 8 || bn->ng > 512 || bn->ng % 8 != 0 || bn->ng % 5 == 0 || !fft_shape(bn->ng, sh))
    return fail(BK_ERR_ARG, "ng must be 2^a or 3*2^a, a multiple of 8, with 8 <= ng <= 512");
  if (bn->n_k1 < 1 || bn->n_mu < 1 || bn->n_t < 1) return fail(BK_ERR_ARG, "bin counts must be >= 1");
  if (!(bn->k1_min >= 0.0) || !(bn->k1_max > bn->k1_min)) return fail(BK_ERR_ARG, "need 0 <= k1_min < k1_max");
  if (bn->k1_max > double(bn->ng) / 3.0) return fail(BK_ERR_ARG, "k1_max must not exceed ng/3");
  if (bn->l_max < 0 || bn->l_max > 12 || bn->m_max < 0 || bn->m_max > bn->l_max)
    return fail(BK_ERR_ARG, "need 0 <= m_max <= l_max <= 12");
  if (bn->even_l_only != 0 && bn->even_l_only != 1) return fail(BK_ERR_ARG, "even_l_only must be 0 or 1");
  if (!(bn->box_len >= 0.0) && !(bn->box_len < 0.0)) return fail(BK_ERR_ARG, "box_len is NaN");
  b->ng = bn->ng;
  b->box_len = bn->box_len > 0 ? bn->box_len : double(bn->ng);
  b->n_k1 = bn->n_k1;
  b->k1_min = bn->k1_min;
  b->k1_max = bn->k1_max;
  b->n_mu = bn->n_mu;
  b->n_t = bn->n_t;
  b->l_max = bn->l_max;
  b->m_max = bn->m_max;
  b->even_l_only = bn->even_l_only == 1;
  if (bk::count_lm(b->l_max, b->m_max, b->even_l_only) > 64)
    return fail(BK_ERR_ARG, "at most 64 multipoles per plan (lower l_max or m_max)");
  return BK_OK;
}

int host_threads() { return int(std::max(1u, std::min(16u, std::thread::hardware_concurrency()))); }

}  // namespace

extern "C" bk_status bk_count_triangles(const bk_binning* bn, int64_t* out, size_t cap, int64_t* n_comb) {
  g_last_error.clear();
  if (!bn || !out) return fail(BK_ERR_ARG, "null argument");
  bk::FftShape sh{};
  bk::Binning b;
  bk_status st = check_binning(bn, &sh, &b);
  if (st != BK_OK) return st;
  const size_t n_bins = size_t(b.n_k1) * b.n_mu * b.n_t;
  if (cap < n_bins) return fail(BK_ERR_SIZE, "output buffer too small");
  bk::Tables T;
  std::string err;
  try {
    err = bk::build_tables(b, bk::K3Shape(), host_threads(), &T, nullptr, true);
  } catch (const std::bad_alloc&) {
    return fail(BK_ERR_OOM, "host allocation failed while building tables");
  }
  if (!err.empty()) return fail(BK_ERR_ARG, err);
  std::copy(T.res[0].bin_count.begin(), T.res[0].bin_count.end(), out);
  if (n_comb) *n_comb = T.n_combos;
  return BK_OK;
}

extern "C" bk_status bk_discrete_prediction(const bk_binning* bn, const bk_model* model, double* out, size_t cap) {
  g_last_error.clear();
  if (!bn || !model || !out) return fail(BK_ERR_ARG, "null argument");
  if (!(model->amp >= 0.0) || !std::isfinite(model->n_s) || !std::isfinite(model->f_ng) || !std::isfinite(model->beta))
    return fail(BK_ERR_ARG, "model parameters must be finite, amp >= 0");
  bk::FftShape sh{};
  bk::Binning b;
  bk_status st = check_binning(bn, &sh, &b);
  if (st != BK_OK) return st;
  const size_t n_out = size_t(bk::count_lm(b.l_max, b.m_max, b.even_l_only)) * b.n_k1 * b.n_mu * b.n_t;
  if (cap < n_out) return fail(BK_ERR_SIZE, "output buffer too small");
  bk::Model mdl;
  mdl.amp = model->amp;
  mdl.n_s = model->n_s;
  mdl.f_ng = model->f_ng;
  mdl.beta = model->beta;
  bk::Tables T;
  std::string err;
  try {
    err = bk::build_tables(b, bk::K3Shape(), host_threads(), &T, &mdl, true);
  } catch (const std::bad_alloc&) {
    return fail(BK_ERR_OOM, "host allocation failed while building tables");
  }
  if (!err.empty()) return fail(BK_ERR_ARG, err);
  const std::vector<double>& pred = T.res[0].model_pred;
  if (pred.size() != n_out) return fail(BK_ERR_ARG, "internal: prediction size mismatch");
  std::copy(pred.begin(), pred.end(), out);
  return BK_OK;
}

extern "C" bk_status bk_continuum_multipoles(int l_max, int m_max, double mu, double t, double beta, double* out,
                                             size_t cap) {
  g_last_error.clear();
  if (!out) return fail(BK_ERR_ARG, "null argument");
  if (l_max < 0 || l_max > 12 || m_max < 0 || m_max > l_max) return fail(BK_ERR_ARG, "need 0 <= m_max <= l_max <= 12");
  if (!(mu >= -1.0 && mu <= 1.0) || !(t > 0.0 && t <= 1.0) || !std::isfinite(beta))
    return fail(BK_ERR_ARG, "need -1 <= mu <= 1, 0 < t <= 1 and a finite beta");
  if (!(1.0 - 2.0 * t * mu + t * t > 0.0)) return fail(BK_ERR_ARG, "degenerate shape: k3 = 0");
  const std::vector<double> v = bk::continuum_multipoles(l_max, m_max, mu, t, beta);
  if (cap < v.size()) return fail(BK_ERR_SIZE, "output buffer too small");
  std::copy(v.begin(), v.end(), out);
  return BK_OK;
}

extern "C" bk_status bk_plan_create(const bk_binning* bn, int prec, int device, int max_batch, bk_plan* out) {
  return bk_plan_create_multires(bn, nullptr, 0, prec, device, max_batch, out);
}

extern "C" bk_status bk_plan_create_multires(const bk_binning* bn, const int* extra_bins, int n_extra, int prec,
                                             int device, int max_batch, bk_plan* out) {
  g_last_error.clear();
  if (!bn || !out) return fail(BK_ERR_ARG, "null argument");
  *out = nullptr;
  if (prec != BK_F32 && prec != BK_F64) return fail(BK_ERR_ARG, "prec must be BK_F32 or BK_F64");
  if (max_batch < 1) return fail(BK_ERR_ARG, "max_batch must be >= 1");
  if (n_extra < 0 || n_extra > bk::kMaxResolutions - 1 || (n_extra > 0 && !extra_bins))
    return fail(BK_ERR_ARG, "n_extra must be in [0, " + std::to_string(bk::kMaxResolutions - 1) +
                                "] with extra_bins holding 3 * n_extra counts");
  bk::FftShape sh{};
  bk::Binning b;
  {
    bk_status cst = check_binning(bn, &sh, &b);
    if (cst != BK_OK) return cst;
  }
  std::vector<std::array<int, 3>> extra;
  for (int r = 0; r < n_extra; ++r) {
    const std::array<int, 3> d{extra_bins[3 * r], extra_bins[3 * r + 1], extra_bins[3 * r + 2]};
    if (d[0] < 1 || d[1] < 1 || d[2] < 1) return fail(BK_ERR_ARG, "bin counts must be >= 1");
    if (double(d[0]) * d[1] * d[2] > 1e7) return fail(BK_ERR_ARG, "at most 10^7 bins per resolution");
    extra.push_back(d);
  }
  int ndev = 0;
  BK_HIP(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(BK_ERR_ARG, "no such device");
  BK_HIP(hipSetDevice(device));

  bk_plan p = new (std::nothrow) bk_plan_s();
  if (!p) return fail(BK_ERR_OOM, "host allocation failed");
  p->prec = prec;
  p->device = device;
  p->max_batch = max_batch;
  p->sh = sh;
  // Work-item shape: items of 16 pairs (one row tile) pack the (pair,
  // slot-B window) rows tightly; two per wave make workgroups of 16 items,
  // which share their staged sides: about 0.26 staged bytes per padded term
  // (float32) against 0.33 with eight items, and the contraction is close to
  // bound by that traffic.  Two buffers of 160 slots (159 sides and the zero
  // slot) of 256 bytes take 81 920 bytes of LDS: two workgroups fill the
  // compute unit's 160 KiB.  With one item per wave, 104 sides (53 760 bytes)
  // let three workgroups share a compute unit.
  // BK_K3_PAIRS=32 or 64 selects items of two or four tiles (one per wave),
  // BK_K3_ITEMS=1 one 16-pair item per wave; BK_K3_SIDES overrides the cap.
  bk::K3Shape shape;
  shape.pairs_per_item = 16;
  shape.items_per_wave = 2;
  if (const char* v = std::getenv("BK_K3_PAIRS")) {
    shape.pairs_per_item = std::atoi(v);
    if (shape.pairs_per_item != 16) shape.items_per_wave = 1;
  }
  if (const char* v = std::getenv("BK_K3_ITEMS")) shape.items_per_wave = std::atoi(v);
  shape.max_group_sides = shape.items_per_wave == 2 ? 159 : 104;
  if (const char* v = std::getenv("BK_K3_SIDES")) shape.max_group_sides = std::atoi(v);
  if (const char* v = std::getenv("BK_FULL_GRID")) shape.coarse_grids = std::atoi(v) == 0;
  std::string err;
  try {
    err = bk::build_tables(b, shape, host_threads(), &p->tab, nullptr, false, extra);
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(BK_ERR_OOM, "host allocation failed while building tables");
  }
  if (!err.empty()) {
    delete p;
    return fail(BK_ERR_ARG, err);
  }
  bk::Tables& T = p->tab;
  const int n = bn->ng;
  p->nkeep = T.nmax + 1;
  if (p->nkeep > n / 2 + 1) p->nkeep = n / 2 + 1;
  p->n_sides = long(T.side_ring.size());
  p->n_items = long(T.items.size());
  p->item_out = int(T.s_per_item);
  p->elem = prec == BK_F32 ? 4 : 8;
  const size_t cs = 2 * p->elem;
  // scale so float32 sums stay far from overflow: Delta' = Delta_DFT / N^{3/2}
  p->delta_scale = 1.0 / std::pow(double(n), 1.5);
  const double vol = b.box_len * b.box_len * b.box_len;
  const double n3 = double(n) * n * n;
  // B = sqrt(.) Re sum w S_Delta / (V N^2) / den;  S_Delta = (V/N^3)^3 S_DFT;  S_DFT = S' / scale^3
  p->norm = std::pow(vol / n3, 3) / (vol * double(n) * n) / std::pow(p->delta_scale, 3);

  // row extent U of each side's ring: the largest |u_x| with |u_x| < R_r
  std::vector<int32_t> side_u(p->n_sides);
  for (long s = 0; s < p->n_sides; ++s) {
    const int64_t e3 = T.edge3[T.side_ring[s]];
    int U = 0;
    while (9 * int64_t(U + 1) * (U + 1) < e3 * e3) ++U;
    side_u[s] = U;
  }
  // per ring: modes sorted by (u_x, u_y) and the start of each row u_x = -U_r..U_r
  std::vector<int32_t> ring_seg_off(T.nr + 1, 0), ring_seg;
  std::vector<int16_t> ring_mode_uy;
  {
    const int lim = T.lim, side_len = 2 * lim + 1;
    for (int r = 1; r <= T.nr; ++r) {
      int U = 0;
      while (9 * int64_t(U + 1) * (U + 1) < T.edge3[r] * T.edge3[r]) ++U;
      ring_seg_off[r - 1] = int32_t(ring_seg.size());
      for (int ux = -U; ux <= U; ++ux) {
        ring_seg.push_back(int32_t(ring_mode_uy.size()));
        for (int uy = -lim; uy <= lim; ++uy)
          if (T.mode_ring[size_t(ux + lim) * side_len + (uy + lim)] == r) ring_mode_uy.push_back(int16_t(uy));
      }
      ring_seg.push_back(int32_t(ring_mode_uy.size()));
    }
    ring_seg_off[T.nr] = int32_t(ring_seg.size());
    // K2 rebuilds each row's u_y from its first one: the row must be the
    // symmetric run [-b, b] or the two runs [-b, -b + h - 1], [b - h + 1, b]
    for (int r = 1; r <= T.nr; ++r)
      for (int i = ring_seg_off[r - 1]; i + 1 < ring_seg_off[r]; ++i) {
        const int m0 = ring_seg[i], cnt = ring_seg[i + 1] - m0;
        if (cnt == 0) continue;
        const int bmax = -ring_mode_uy[m0];
        const bool one = cnt == 2 * bmax + 1;
        const int h = one ? cnt : cnt / 2;
        bool ok = bmax >= 0 && (one || cnt % 2 == 0);
        for (int j = 0; ok && j < cnt; ++j)
          ok = ring_mode_uy[m0 + j] == (j < h ? -bmax + j : bmax - (cnt - 1 - j));
        if (!ok) return fail(BK_ERR_ARG, "internal: a ring row is not a pair of symmetric u_y runs");
      }
  }

  std::vector<double> twd(2 * size_t(n));
  for (int t = 0; t < n; ++t) {
    twd[2 * t] = std::cos(2.0 * M_PI * double(t) / double(n));
    twd[2 * t + 1] = -std::sin(2.0 * M_PI * double(t) / double(n));
  }
  std::vector<float> twf(twd.begin(), twd.end());

  bk_status st = BK_OK;
  const int nlm = int(T.lm_l.size());
#define TRY(x)              \
  do {                      \
    st = (x);               \
    if (st != BK_OK) {      \
      release(p);           \
      delete p;             \
      return st;            \
    }                       \
  } while (0)
  TRY(dalloc(p, &p->d_in, size_t(max_batch) * size_t(n3) * 8));
  TRY(dalloc(p, &p->d_F, size_t(max_batch) * p->nkeep * size_t(n) * n * cs));
  TRY(put(p, &p->d_ring_seg_off, ring_seg_off.data(), ring_seg_off.size()));
  TRY(put(p, &p->d_ring_seg, ring_seg.data(), ring_seg.size()));
  TRY(put(p, &p->d_ring_mode_uy, ring_mode_uy.data(), ring_mode_uy.size()));
  TRY(dalloc(p, &p->d_D, size_t(max_batch) * size_t(T.d_elems) * cs));
  {
    // twiddles e^{-2 pi i t / m} of every grid level, concatenated
    std::vector<double> tl;
    for (int m : T.grid_sizes) {
      bk::FftShape lsh{};
      fft_shape(m, &lsh);
      p->lv_sh.push_back(lsh);
      p->tw_lv_off.push_back(long(tl.size() / 2));
      for (int t = 0; t < m; ++t) {
        tl.push_back(std::cos(2.0 * M_PI * double(t) / double(m)));
        tl.push_back(-std::sin(2.0 * M_PI * double(t) / double(m)));
      }
    }
    if (prec == BK_F32) {
      std::vector<float> tf(tl.begin(), tl.end());
      TRY(put(p, reinterpret_cast<float**>(&p->d_tw_lv), tf.data(), tf.size()));
    } else {
      TRY(put(p, reinterpret_cast<double**>(&p->d_tw_lv), tl.data(), tl.size()));
    }
  }
  TRY(put(p, &p->d_gs_side, T.gside_side.data(), T.gside_side.size()));
  TRY(put(p, &p->d_gs_off, T.gside_off.data(), T.gside_off.size()));
  TRY(dalloc(p, reinterpret_cast<void**>(&p->d_S), size_t(max_batch) * size_t(p->n_items) * p->item_out * 8));
  if (prec == BK_F32)
    TRY(put(p, reinterpret_cast<float**>(&p->d_tw), twf.data(), twf.size()));
  else
    TRY(put(p, reinterpret_cast<double**>(&p->d_tw), twd.data(), twd.size()));
  TRY(put(p, &p->d_groups, T.groups.data(), T.groups.size()));
  TRY(put(p, &p->d_items, T.items.data(), T.items.size()));
  TRY(put(p, &p->d_group_sides, T.group_sides.data(), T.group_sides.size()));
  TRY(put(p, &p->d_side_ring, T.side_ring.data(), T.side_ring.size()));
  TRY(put(p, &p->d_side_plane, T.side_plane.data(), T.side_plane.size()));
  TRY(put(p, &p->d_side_u, side_u.data(), side_u.size()));
  if (long(p->n_items) * p->item_out * max_batch >= (1L << 31)) {
    release(p);
    delete p;
    return fail(BK_ERR_ARG, "too many work items for 32-bit output slots");
  }
  p->k4.resize(T.res.size());
  for (size_t r = 0; r < T.res.size(); ++r) {
    bk::Resolution& R = T.res[r];
    K4Res& k = p->k4[r];
    k.n_bins = R.n_bins();
    std::vector<long> chunk_begin, bin_chunk(k.n_bins + 1, 0);
    for (int bin = 0; bin < k.n_bins; ++bin) {
      bin_chunk[bin] = long(chunk_begin.size());
      for (long c = R.bin_ptr[bin]; c < R.bin_ptr[bin + 1]; c += bk::kK4Chunk) chunk_begin.push_back(c);
    }
    bin_chunk[k.n_bins] = long(chunk_begin.size());
    k.n_chunks = long(chunk_begin.size());
    chunk_begin.push_back(R.bin_ptr[k.n_bins]);
    // chunks are consecutive and start at every bin start, so none crosses a bin
    TRY(put(p, &k.d_chunk_begin, chunk_begin.data(), chunk_begin.size()));
    TRY(put(p, &k.d_bin_chunk, bin_chunk.data(), bin_chunk.size()));
    TRY(dalloc(p, reinterpret_cast<void**>(&k.d_part), size_t(max_batch) * std::max(1L, k.n_chunks) * nlm * 8));
    TRY(dalloc(p, reinterpret_cast<void**>(&k.d_B), size_t(max_batch) * nlm * k.n_bins * 8));
    {
      std::vector<int32_t> cslot(R.combo_slot.begin(), R.combo_slot.end());
      TRY(put(p, &k.d_combo_slot, cslot.data(), cslot.size()));
    }
    // Coefficients in the plan's precision: float32 rounding (2^-24 relative)
    // of each coefficient is far below the float32 path's error, and halves
    // the bytes the binning reads; the per-bin sums stay float64.
    if (prec == BK_F32) {
      std::vector<float> c32(R.combo_coef.begin(), R.combo_coef.end());
      TRY(put(p, reinterpret_cast<float**>(&k.d_coef), c32.data(), c32.size()));
    } else {
      TRY(put(p, reinterpret_cast<double**>(&k.d_coef), R.combo_coef.data(), R.combo_coef.size()));
    }
    TRY(put(p, &k.d_empty, R.bin_empty_lm.data(), R.bin_empty_lm.size()));
    // the host copies of the per-combination arrays are no longer needed
    std::vector<double>().swap(R.combo_coef);
    std::vector<int64_t>().swap(R.combo_slot);
  }
#undef TRY

  {
    // largest chunk whose two staging buffers fit 80 KiB (at least two
    // workgroups per CU), else the smallest valid one
    p->k3_chunk = 0;
    for (int ch : {64, 32, 16, 8}) {
      const size_t lds = k3_lds_bytes(T, prec, ch);
      if (lds && (lds <= 81920 || p->k3_chunk == 0)) {
        p->k3_chunk = ch;
        p->lds_k3 = lds;
        if (lds <= 81920) break;
      }
    }
    if (p->k3_chunk == 0) {
      release(p);
      delete p;
      return fail(BK_ERR_ARG, "workgroup staging does not fit the LDS");
    }
  }
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    auto it = g_tune_cache.find(tune_key(p));
    if (it != g_tune_cache.end() && k3_lds_bytes(T, prec, it->second[2])) {
      p->fft_tb = it->second[0];
      p->k2_tb = it->second[1];
      p->k3_chunk = it->second[2];
      p->lds_k3 = k3_lds_bytes(T, prec, p->k3_chunk);
      p->tuned = 1;
    }
  }
  p->have_events = true;
  for (auto& set : p->evs)
    for (auto& e : set) {
      hipError_t he = hipEventCreate(&e);
      if (he != hipSuccess) {
        release(p);
        delete p;
        return fail(BK_ERR_HIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
      }
    }
  *out = p;
  return BK_OK;
}

extern "C" {

bk_status bk_plan_destroy(bk_plan p) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  (void)hipSetDevice(p->device);
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  (void)hipDeviceSynchronize();
  release(p);
  delete p;
  return BK_OK;
}

bk_status bk_load_grid(bk_plan p, const void* delta, int dtype, int batch, int is_device_ptr, void* hip_stream) {
  g_last_error.clear();
  if (!p || !delta) return fail(BK_ERR_ARG, "null argument");
  if (dtype != BK_F32 && dtype != BK_F64) return fail(BK_ERR_ARG, "dtype must be BK_F32 or BK_F64");
  if (batch < 1 || batch > p->max_batch) return fail(BK_ERR_ARG, "batch must be in [1, max_batch]");
  BK_HIP(hipSetDevice(p->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t n3 = size_t(p->sh.n) * p->sh.n * p->sh.n;
  const size_t bytes = size_t(batch) * n3 * (dtype == BK_F32 ? 4 : 8);
  BK_HIP(hipMemcpyAsync(p->d_in, delta, bytes, is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (!is_device_ptr) BK_HIP(hipStreamSynchronize(st));
  p->batch = batch;
  p->in_dtype = dtype;
  p->estimated = 0;
  p->ev_count = 0;
  p->d_injected = 0;
  p->stream = st;
  return BK_OK;
}

bk_status bk_estimate(bk_plan p, void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  if (p->batch < 1) return fail(BK_ERR_STATE, "no grid loaded");
  BK_HIP(hipSetDevice(p->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (p->d_injected) {
    // test support: D was set directly, run the contraction and binning eagerly
    p->ev_count = 0;
    bk_status s = timed_launch(p, plan_bufs(p), st);
    if (s != BK_OK) return s;
    p->d_injected = 0;
  } else {
    bk_status s = plan_graph(p);
    if (s != BK_OK) return s;
    BK_HIP(hipGraphLaunch(p->graph_exec, st));
    p->ev_count = 0;
  }
  p->stream = st;
  p->estimated = 1;
  return BK_OK;
}

bk_status bk_estimate_timed(bk_plan p, void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  if (p->batch < 1) return fail(BK_ERR_STATE, "no grid loaded");
  BK_HIP(hipSetDevice(p->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  if (p->d_injected) p->ev_count = 0;
  bk_status s = timed_launch(p, plan_bufs(p), st);
  if (s != BK_OK) return s;
  p->d_injected = 0;
  p->stream = st;
  p->estimated = 1;
  return BK_OK;
}

bk_status bk_synchronize(bk_plan p) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  BK_HIP(hipSetDevice(p->device));
  BK_HIP(hipStreamSynchronize(p->stream));
  return BK_OK;
}

bk_status bk_query_sizes(bk_plan p, int* n_lm, int* n_k1, int* n_mu, int* n_t) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  if (n_lm) *n_lm = int(p->tab.lm_l.size());
  if (n_k1) *n_k1 = p->tab.res[0].n_k1;
  if (n_mu) *n_mu = p->tab.res[0].n_mu;
  if (n_t) *n_t = p->tab.res[0].n_t;
  return BK_OK;
}

bk_status bk_get_lm_list(bk_plan p, int* lm, size_t cap) {
  g_last_error.clear();
  if (!p || !lm) return fail(BK_ERR_ARG, "null argument");
  const size_t need = 2 * p->tab.lm_l.size();
  if (cap < need) return fail(BK_ERR_SIZE, "lm buffer too small");
  for (size_t j = 0; j < p->tab.lm_l.size(); ++j) {
    lm[2 * j] = p->tab.lm_l[j];
    lm[2 * j + 1] = p->tab.lm_m[j];
  }
  return BK_OK;
}

bk_status bk_query_resolution(bk_plan p, int res, int* n_k1, int* n_mu, int* n_t) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  if (res < 0 || res >= int(p->tab.res.size())) return fail(BK_ERR_ARG, "no such resolution");
  const bk::Resolution& R = p->tab.res[res];
  if (n_k1) *n_k1 = R.n_k1;
  if (n_mu) *n_mu = R.n_mu;
  if (n_t) *n_t = R.n_t;
  return BK_OK;
}

int bk_n_resolutions(bk_plan p) { return p ? int(p->tab.res.size()) : 0; }

bk_status bk_get_multipoles_res(bk_plan p, int res, double* out, size_t cap) {
  g_last_error.clear();
  if (!p || !out) return fail(BK_ERR_ARG, "null argument");
  if (res < 0 || res >= int(p->k4.size())) return fail(BK_ERR_ARG, "no such resolution");
  if (!p->estimated) return fail(BK_ERR_STATE, "no estimate has been run for the loaded grid");
  const size_t need = size_t(p->batch) * p->tab.lm_l.size() * size_t(p->k4[res].n_bins);
  if (cap < need) return fail(BK_ERR_SIZE, "output buffer too small");
  BK_HIP(hipSetDevice(p->device));
  BK_HIP(hipStreamSynchronize(p->stream));
  BK_HIP(hipMemcpy(out, p->k4[res].d_B, need * sizeof(double), hipMemcpyDeviceToHost));
  return BK_OK;
}

bk_status bk_get_multipoles(bk_plan p, double* out, size_t cap) { return bk_get_multipoles_res(p, 0, out, cap); }

bk_status bk_get_triangle_counts_res(bk_plan p, int res, int64_t* out, size_t cap) {
  g_last_error.clear();
  if (!p || !out) return fail(BK_ERR_ARG, "null argument");
  if (res < 0 || res >= int(p->tab.res.size())) return fail(BK_ERR_ARG, "no such resolution");
  const bk::Resolution& R = p->tab.res[res];
  if (cap < R.bin_count.size()) return fail(BK_ERR_SIZE, "output buffer too small");
  std::copy(R.bin_count.begin(), R.bin_count.end(), out);
  return BK_OK;
}

bk_status bk_get_triangle_counts(bk_plan p, int64_t* out, size_t cap) {
  return bk_get_triangle_counts_res(p, 0, out, cap);
}

bk_status bk_get_bin_means_res(bk_plan p, int res, double* out, size_t cap) {
  g_last_error.clear();
  if (!p || !out) return fail(BK_ERR_ARG, "null argument");
  if (res < 0 || res >= int(p->tab.res.size())) return fail(BK_ERR_ARG, "no such resolution");
  const bk::Resolution& R = p->tab.res[res];
  if (cap < R.bin_mean.size()) return fail(BK_ERR_SIZE, "output buffer too small");
  std::copy(R.bin_mean.begin(), R.bin_mean.end(), out);
  return BK_OK;
}

bk_status bk_get_bin_means(bk_plan p, double* out, size_t cap) { return bk_get_bin_means_res(p, 0, out, cap); }

bk_status bk_get_plan_info(bk_plan p, double* info, size_t cap) {
  g_last_error.clear();
  if (!p || !info) return fail(BK_ERR_ARG, "null argument");
  if (cap < 9) return fail(BK_ERR_SIZE, "info buffer needs at least 9 entries");
  info[0] = double(p->tab.n_combos);
  info[1] = double(p->n_items);
  info[2] = double(p->n_sides);
  info[3] = double(p->tab.nr);
  info[4] = p->tab.dense_terms;
  info[5] = p->tab.useful_terms;
  info[6] = double(p->bytes);
  info[7] = double(p->tab.n_canonical_planes);
  info[8] = double(p->tab.n_self_partner);
  if (cap > 9) info[9] = double(p->tab.gside_side.size());
  if (cap > 10) info[10] = double(p->tab.d_elems);
  return BK_OK;
}

bk_status bk_get_stage_times(bk_plan p, double* ms, size_t cap) {
  g_last_error.clear();
  if (!p || !ms) return fail(BK_ERR_ARG, "null argument");
  if (cap < 4) return fail(BK_ERR_SIZE, "need 4 entries");
  if (!p->estimated || p->ev_count == 0) return fail(BK_ERR_STATE, "no timed estimate has been run");
  BK_HIP(hipSetDevice(p->device));
  const int K = bk_plan_s::kEvSets;
  const int last = (p->ev_next + K - 1) % K;
  BK_HIP(hipEventSynchronize(p->evs[last][4]));
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < p->ev_count; ++j) {
    const int set = (last + K - j) % K;
    for (int i = 0; i < 4; ++i) {
      float t = 0.f;
      BK_HIP(hipEventElapsedTime(&t, p->evs[set][i], p->evs[set][i + 1]));
      acc[i] += double(t);
    }
  }
  for (int i = 0; i < 4; ++i) ms[i] = acc[i] / p->ev_count;
  if (cap > 4) ms[4] = double(p->ev_count);
  return BK_OK;
}

bk_status bk_debug_get_buffer(bk_plan p, int which, void* out, size_t cap_bytes, size_t* needed) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  size_t bytes = 0;
  const void* src = nullptr;
  std::vector<int32_t> table;
  if (which == 0 || which == 1 || which == 6) {
    device_buffer(p, which, &src, &bytes);
  } else if (which == 2) {
    for (size_t g = 0; g < p->tab.gside_side.size(); ++g) {
      const int32_t s = p->tab.gside_side[g];
      table.push_back(p->tab.side_ring[s]);
      table.push_back(p->tab.side_plane[s]);
      table.push_back(p->tab.grid_sizes[p->tab.gside_level[g]]);
    }
    bytes = table.size() * sizeof(int32_t);
  } else if (which == 3) {
    bytes = p->tab.items.size() * sizeof(bk::ItemDesc);
  } else if (which == 4) {
    bytes = p->tab.groups.size() * sizeof(bk::GroupDesc);
  } else if (which == 5) {
    bytes = p->tab.group_sides.size() * sizeof(int32_t);
  } else {
    return fail(BK_ERR_ARG, "which must be 0..6");
  }
  if (needed) *needed = bytes;
  if (!out) return BK_OK;
  if (cap_bytes < bytes) return fail(BK_ERR_SIZE, "output buffer too small");
  if (which == 2) {
    std::memcpy(out, table.data(), bytes);
    return BK_OK;
  }
  if (which >= 3 && which <= 5) {
    const void* hs = which == 3 ? static_cast<const void*>(p->tab.items.data())
                     : which == 4 ? static_cast<const void*>(p->tab.groups.data())
                                  : static_cast<const void*>(p->tab.group_sides.data());
    std::memcpy(out, hs, bytes);
    return BK_OK;
  }
  if (!p->estimated) return fail(BK_ERR_STATE, "no estimate has been run");
  BK_HIP(hipSetDevice(p->device));
  BK_HIP(hipStreamSynchronize(p->stream));
  BK_HIP(hipMemcpy(out, src, bytes, hipMemcpyDeviceToHost));
  return BK_OK;
}

bk_status bk_debug_read_range(bk_plan p, int which, size_t offset_bytes, void* out, size_t bytes) {
  g_last_error.clear();
  if (!p || (!out && bytes)) return fail(BK_ERR_ARG, "null argument");
  if (which != 0 && which != 1 && which != 6) return fail(BK_ERR_ARG, "which must be 0, 1 or 6");
  const void* src = nullptr;
  size_t total = 0;
  device_buffer(p, which, &src, &total);
  if (offset_bytes > total || bytes > total - offset_bytes) return fail(BK_ERR_SIZE, "range outside the buffer");
  if (!p->estimated) return fail(BK_ERR_STATE, "no estimate has been run");
  if (bytes == 0) return BK_OK;
  BK_HIP(hipSetDevice(p->device));
  BK_HIP(hipStreamSynchronize(p->stream));
  BK_HIP(hipMemcpy(out, static_cast<const char*>(src) + offset_bytes, bytes, hipMemcpyDeviceToHost));
  return BK_OK;
}

bk_status bk_debug_set_D(bk_plan p, const void* D, int batch, int is_device_ptr, void* hip_stream) {
  g_last_error.clear();
  if (!p || !D) return fail(BK_ERR_ARG, "null argument");
  if (batch < 1 || batch > p->max_batch) return fail(BK_ERR_ARG, "batch must be in [1, max_batch]");
  BK_HIP(hipSetDevice(p->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const size_t bytes = size_t(batch) * size_t(p->tab.d_elems) * 2 * p->elem;
  BK_HIP(hipMemcpyAsync(p->d_D, D, bytes, is_device_ptr ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (!is_device_ptr) BK_HIP(hipStreamSynchronize(st));
  p->batch = batch;
  p->estimated = 0;
  p->d_injected = 1;
  p->stream = st;
  return BK_OK;
}

bk_status bk_debug_mfma_probe(int prec, double* out, size_t cap) {
  g_last_error.clear();
  if (!out) return fail(BK_ERR_ARG, "null argument");
  if (cap < 256) return fail(BK_ERR_SIZE, "need 256 entries");
  if (prec != BK_F32 && prec != BK_F64) return fail(BK_ERR_ARG, "prec must be BK_F32 or BK_F64");
  double* d = nullptr;
  BK_HIP(hipMalloc(&d, 256 * sizeof(double)));
  if (prec == BK_F32)
    hipLaunchKernelGGL(bk::mfma_probe_kernel<float>, dim3(1), dim3(64), 0, 0, d);
  else
    hipLaunchKernelGGL(bk::mfma_probe_kernel<double>, dim3(1), dim3(64), 0, 0, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(out, d, 256 * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(BK_ERR_HIP, std::string("mfma probe: ") + hipGetErrorString(e));
  return BK_OK;
}


}  // extern "C"

struct bk_group_s {
  std::vector<bk_plan> plans;
  std::vector<int> captured_batch;
  int device = 0;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

void group_release(bk_group g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (auto e : g->join)
    if (e) (void)hipEventDestroy(e);
  if (g->fork) (void)hipEventDestroy(g->fork);
  for (auto s : g->side)
    if (s) (void)hipStreamDestroy(s);
  if (g->cap) (void)hipStreamDestroy(g->cap);
}

bk_status group_capture(bk_group g) {
  if (g->exec) {
    BK_HIP(hipGraphExecDestroy(g->exec));
    g->exec = nullptr;
  }
  if (g->graph) {
    BK_HIP(hipGraphDestroy(g->graph));
    g->graph = nullptr;
  }
  BK_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
  bk_status st = BK_OK;
  hipError_t he = hipEventRecord(g->fork, g->cap);
  for (size_t i = 0; i < g->plans.size() && st == BK_OK && he == hipSuccess; ++i) {
    bk_plan p = g->plans[i];
    he = hipStreamWaitEvent(g->side[i], g->fork, 0);
    if (he != hipSuccess) break;
    Bufs bf = plan_bufs(p);
    bf.skip_fft = false;
    st = p->prec == BK_F32 ? launch_all<float>(p, bf, g->side[i], false) : launch_all<double>(p, bf, g->side[i], false);
    if (st != BK_OK) break;
    he = hipEventRecord(g->join[i], g->side[i]);
    if (he == hipSuccess) he = hipStreamWaitEvent(g->cap, g->join[i], 0);
  }
  hipGraph_t graph = nullptr;
  hipError_t he_end = hipStreamEndCapture(g->cap, &graph);
  if (st != BK_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (he != hipSuccess || he_end != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return fail(BK_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(he != hipSuccess ? he : he_end));
  }
  g->graph = graph;
  BK_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  for (size_t i = 0; i < g->plans.size(); ++i) g->captured_batch[i] = g->plans[i]->batch;
  return BK_OK;
}

}  // namespace

extern "C" {

bk_status bk_group_create(const bk_plan* plans, int n, bk_group* out) {
  g_last_error.clear();
  if (!plans || !out || n < 1) return fail(BK_ERR_ARG, "need at least one plan");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(BK_ERR_ARG, "null plan in group");
    if (plans[i]->device != plans[0]->device) return fail(BK_ERR_ARG, "all plans of a group must use one device");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(BK_ERR_ARG, "a plan appears twice in the group");
  }
  BK_HIP(hipSetDevice(plans[0]->device));
  bk_group g = new (std::nothrow) bk_group_s();
  if (!g) return fail(BK_ERR_OOM, "host allocation failed");
  g->plans.assign(plans, plans + n);
  g->captured_batch.assign(n, -1);
  g->device = plans[0]->device;
  g->side.assign(n, nullptr);
  g->join.assign(n, nullptr);
  hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&g->fork, hipEventDisableTiming);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&g->join[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    group_release(g);
    delete g;
    return fail(BK_ERR_HIP, std::string("group streams: ") + hipGetErrorString(e));
  }
  *out = g;
  return BK_OK;
}

bk_status bk_group_estimate(bk_group g, void* hip_stream) {
  g_last_error.clear();
  if (!g) return fail(BK_ERR_ARG, "null group");
  BK_HIP(hipSetDevice(g->device));
  bool recapture = g->exec == nullptr;
  for (size_t i = 0; i < g->plans.size(); ++i) {
    if (g->plans[i]->batch < 1) return fail(BK_ERR_STATE, "a plan of the group has no grid loaded");
    if (g->plans[i]->batch != g->captured_batch[i]) recapture = true;
  }
  if (recapture) {
    // the members' inputs were loaded on other streams: finish those copies first
    for (auto p : g->plans) BK_HIP(hipStreamSynchronize(p->stream));
    bk_status st = group_capture(g);
    if (st != BK_OK) return st;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  BK_HIP(hipGraphLaunch(g->exec, st));
  for (auto p : g->plans) {
    p->stream = st;
    p->estimated = 1;
    p->ev_count = 0;
  }
  return BK_OK;
}

bk_status bk_group_destroy(bk_group g) {
  g_last_error.clear();
  if (!g) return fail(BK_ERR_ARG, "null group");
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  group_release(g);
  delete g;
  return BK_OK;
}

}  // extern "C"


extern "C" bk_status bk_plan_autotune(bk_plan p, void* hip_stream, int* choices) {
  g_last_error.clear();
  if (!p) return fail(BK_ERR_ARG, "null plan");
  if (p->batch < 1) return fail(BK_ERR_STATE, "load a grid before tuning");
  BK_HIP(hipSetDevice(p->device));
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  const int n = p->sh.n;
  const size_t cs = 2 * p->elem;
  std::vector<int> c_fft, c_k2, c_k3;
  for (int tb : {2, 4, 8, 16})
    if (n % tb == 0 && fft_lds_bytes(n, tb, cs) <= 73728) c_fft.push_back(tb);
  for (int tb : {4, 8, 16}) c_k2.push_back(tb);  // the per-level slab is k2_slab(m, tb)
  for (int ch : {8, 16, 32, 64})
    if (k3_lds_bytes(p->tab, p->prec, ch)) c_k3.push_back(ch);
  if (c_fft.empty() || c_k3.empty()) return fail(BK_ERR_ARG, "no valid tile choice to tune");
  const int saved[3] = {p->fft_tb, p->k2_tb, p->k3_chunk};
  const size_t saved_lds = p->lds_k3;
  const size_t rounds = std::max({c_fft.size(), c_k2.size(), c_k3.size()});
  std::vector<double> t_fft(c_fft.size(), 1e30), t_k2(c_k2.size(), 1e30), t_k3(c_k3.size(), 1e30);
  // Stage times are independent of the other stages' tiles, so round i times
  // candidate i of every stage at once; each configuration runs twice, the
  // second run is kept.
  for (size_t i = 0; i < rounds; ++i) {
    p->fft_tb = c_fft[std::min(i, c_fft.size() - 1)];
    p->k2_tb = c_k2[std::min(i, c_k2.size() - 1)];
    p->k3_chunk = c_k3[std::min(i, c_k3.size() - 1)];
    p->lds_k3 = k3_lds_bytes(p->tab, p->prec, p->k3_chunk);
    for (int rep = 0; rep < 2; ++rep) {
      Bufs bf = plan_bufs(p);
      bf.skip_fft = false;
      bk_status sst = timed_launch(p, bf, st);
      if (sst != BK_OK) {
        p->fft_tb = saved[0];
        p->k2_tb = saved[1];
        p->k3_chunk = saved[2];
        p->lds_k3 = saved_lds;
        return sst;
      }
    }
    // p->ev still points at the set of the second run
    BK_HIP(hipEventSynchronize(p->ev[4]));
    float ms[3];
    for (int k = 0; k < 3; ++k) BK_HIP(hipEventElapsedTime(&ms[k], p->ev[k], p->ev[k + 1]));
    if (i < c_fft.size()) t_fft[i] = ms[0];
    if (i < c_k2.size()) t_k2[i] = ms[1];
    if (i < c_k3.size()) t_k3[i] = ms[2];
  }
  auto best = [](const std::vector<int>& c, const std::vector<double>& t) {
    return c[size_t(std::min_element(t.begin(), t.end()) - t.begin())];
  };
  p->fft_tb = best(c_fft, t_fft);
  p->k2_tb = best(c_k2, t_k2);
  p->k3_chunk = best(c_k3, t_k3);
  p->lds_k3 = k3_lds_bytes(p->tab, p->prec, p->k3_chunk);
  p->tuned = 1;
  p->d_injected = 0;
  // the last configuration timed ran the whole path: its results and stage
  // times stand
  p->stream = st;
  p->estimated = 1;
  p->ev_count = 1;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[tune_key(p)] = {p->fft_tb, p->k2_tb, p->k3_chunk};
  }
  if (choices) {
    choices[0] = p->fft_tb;
    choices[1] = p->k2_tb;
    choices[2] = p->k3_chunk;
  }
  return BK_OK;
}

// ---------------------------------------------------------------- allocation-free estimate
// Working set of bk_estimate_noalloc: one array per device, in the library's
// code object, that holds that call's Delta planes, ring sums D, contraction
// outputs S and binning partials.  Host code never passes `scratch` itself to
// a kernel (its host-side name is no device address); it takes the device's
// address once from hipGetSymbolAddress and uses that.
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;
}
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mutex;
std::map<int, void*> g_scratch_ptr;  // device -> device address of its `scratch`

// The calling thread's current device must be `device`.
bk_status scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return BK_OK;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr)
    return fail(BK_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  *out = ptr;
  return BK_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" bk_status bk_estimate_noalloc(bk_plan p, const void* delta, int dtype, int batch, double* B_out,
                                         void* hip_stream) {
  g_last_error.clear();
  if (!p || !delta || !B_out) return fail(BK_ERR_ARG, "null argument");
  if (dtype != BK_F32 && dtype != BK_F64) return fail(BK_ERR_ARG, "dtype must be BK_F32 or BK_F64");
  if (batch < 1) return fail(BK_ERR_ARG, "batch must be >= 1");
  const size_t cs = 2 * p->elem;
  const size_t b = size_t(batch);
  const size_t n2 = size_t(p->sh.n) * p->sh.n;
  const size_t nlm = p->tab.lm_l.size();
  const size_t f_bytes = align256(b * p->nkeep * n2 * cs);
  const size_t d_bytes = align256(b * size_t(p->tab.d_elems) * cs);
  const size_t s_bytes = align256(b * size_t(p->n_items) * size_t(p->item_out) * sizeof(double));
  const size_t part_bytes = align256(b * size_t(std::max(1L, p->k4[0].n_chunks)) * nlm * sizeof(double));
  const size_t need = f_bytes + d_bytes + s_bytes + part_bytes;
  if (need > kScratchBytes)
    return fail(BK_ERR_SIZE, "this plan needs " + std::to_string(need) + " bytes of scratch for " +
                                 std::to_string(batch) + " field(s); the allocation-free path holds " +
                                 std::to_string(kScratchBytes));
  BK_HIP(hipSetDevice(p->device));
  void* base = nullptr;
  bk_status st = scratch_address(p->device, &base);
  if (st != BK_OK) return st;
  char* c = static_cast<char*>(base);
  Bufs bf;
  bf.in = delta;
  bf.in_dtype = dtype;
  bf.batch = batch;
  bf.F = c;
  bf.D = c + f_bytes;
  bf.S = reinterpret_cast<double*>(c + f_bytes + d_bytes);
  bf.part = reinterpret_cast<double*>(c + f_bytes + d_bytes + s_bytes);
  bf.B = B_out;
  bf.first_res_only = true;
  // every scratch element an estimate reads was written earlier in the same
  // estimate, so nothing needs clearing between calls
  hipStream_t hs = reinterpret_cast<hipStream_t>(hip_stream);
  return p->prec == BK_F32 ? launch_all<float>(p, bf, hs, false) : launch_all<double>(p, bf, hs, false);
}
