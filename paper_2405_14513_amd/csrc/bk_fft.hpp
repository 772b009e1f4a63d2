// LDS-resident Stockham FFT building blocks for gfx950 (HIP).
//
// All transforms here are forward DFTs, y[k] = sum_j x[j] e^{-2 pi i j k / N}:
// the 3-D transform of the field (Sec. II) and the ring sums of Eq. 9, whose
// exponent carries the same minus sign.  N = 2^a 3^b 5^c; stages use radix
// 4, then one radix 2 if a is odd, then radix 3 and radix 5 (the runtime-
// length lds_fft takes b, c <= 1, as the host's fft_shape; lds_fft_c has N
// and every stage's stride as compile-time constants).  Twiddles are a table
// exp(-2 pi i t / N), t < N, computed on the host in float64 and cast.
#pragma once

#include <hip/hip_runtime.h>

namespace bk {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.x - b.x, a.y - b.y};
}

struct FftShape {
  int n;            // transform length
  int nstages;
  int radix[12];
};

// In-register radix-R DFT of v[0..R-1] (forward sign).
template <typename T, int R>
__device__ __forceinline__ void butterfly(cplx<T> (&v)[R]) {
  if constexpr (R == 2) {
    const cplx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    // e^{-2 pi i / 3} = -1/2 - i sqrt(3)/2
    const T h = T(0.5);
    const T s3 = T(0.86602540378443864676);
    const cplx<T> t1 = cadd(v[1], v[2]);
    const cplx<T> t2 = {v[0].x - h * t1.x, v[0].y - h * t1.y};
    const cplx<T> t3 = {s3 * (v[1].y - v[2].y), -s3 * (v[1].x - v[2].x)};  // -i sqrt3/2 (v1 - v2)
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  } else if constexpr (R == 5) {
    // y_k = sum_j v_j w^{jk}, w = e^{-2 pi i / 5}: pair j with 5 - j
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
    const cplx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    const cplx<T> t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    const cplx<T> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
    const cplx<T> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
    const cplx<T> b1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    const cplx<T> b2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = {a1.x + b1.y, a1.y - b1.x};  // a1 - i b1
    v[4] = {a1.x - b1.y, a1.y + b1.x};  // a1 + i b1
    v[2] = {a2.x + b2.y, a2.y - b2.x};
    v[3] = {a2.x - b2.y, a2.y + b2.x};
  } else if constexpr (R == 4) {
    const cplx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    const cplx<T> b0 = cadd(v[1], v[3]), b1 = csub(v[1], v[3]);
    const cplx<T> mib1 = {b1.y, -b1.x};  // -i * b1
    v[0] = cadd(a0, b0);
    v[1] = cadd(a1, mib1);
    v[2] = csub(a0, b0);
    v[3] = csub(a1, mib1);
  }
}

// One Stockham pass over `lines` transforms held in LDS, src -> dst.
// Element i of line l lives at buf[l * ls + i].
template <typename T, int R>
__device__ __forceinline__ void stockham_pass(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                              const cplx<T>* __restrict__ tw, int n, int ns, int lines, int ls) {
  const int nb = n / R;  // butterflies per line
  const int total = lines * nb;
  const int tw_step = n / (ns * R);
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    const int l = q / nb;
    const int j = q - l * nb;
    const int k = j % ns;
    const cplx<T>* s = src + l * ls;
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    if (ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[(k * r * tw_step) % n]);
    }
    butterfly<T, R>(v);
    cplx<T>* d = dst + l * ls + (j / ns) * ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[r * ns] = v[r];
  }
}

// The same pass with the length N and the stride NS known at compile time:
// the index arithmetic becomes shifts and constant multiplies (unsigned, so
// no sign fix-ups), and the twiddle index k r (N / (NS R)) < N needs no
// reduction.
template <typename T, int R, int N, int NS>
__device__ __forceinline__ void stockham_pass_c(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst,
                                                const cplx<T>* __restrict__ tw, int lines, int ls) {
  constexpr unsigned nb = N / R;
  constexpr unsigned tw_step = N / (NS * R);
  const unsigned total = unsigned(lines) * nb;
  for (unsigned q = threadIdx.x; q < total; q += blockDim.x) {
    const unsigned l = q / nb;
    const unsigned j = q - l * nb;
    const unsigned k = j % NS;
    const cplx<T>* s = src + l * unsigned(ls);
    cplx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * nb];
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * tw_step]);
    }
    butterfly<T, R>(v);
    cplx<T>* d = dst + l * unsigned(ls) + (j / NS) * (NS * R) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[r * NS] = v[r];
  }
}

// Radix sequence of a compile-time length N = 2^a 3^b 5^c: radix 4 while it
// divides the power of two, one radix 2 if a is odd, then 3s, then 5s (the
// order of fft_shape on the host).
template <int N>
struct Radices {
  static constexpr int pw(int n, int p) { return n % p == 0 ? 1 + pw(n / p, p) : 0; }
  static constexpr int p2 = pw(N, 2), p3 = pw(N, 3), p5 = pw(N, 5);
  static constexpr int n4 = p2 / 2, n2 = p2 % 2;
  static constexpr int count = n4 + n2 + p3 + p5;
  static constexpr int radix(int s) { return s < n4 ? 4 : s < n4 + n2 ? 2 : s < n4 + n2 + p3 ? 3 : 5; }
};

// Passes S.. of a compile-time-length transform, stride NS so far; returns
// the buffer holding the result.
template <typename T, int N, int S = 0, int NS = 1>
__device__ cplx<T>* lds_fft_c(cplx<T>* src, cplx<T>* dst, const cplx<T>* tw, int lines, int ls) {
  if constexpr (S == Radices<N>::count) {
    return src;
  } else {
    constexpr int R = Radices<N>::radix(S);
    stockham_pass_c<T, R, N, NS>(src, dst, tw, lines, ls);
    __syncthreads();
    return lds_fft_c<T, N, S + 1, NS * R>(dst, src, tw, lines, ls);
  }
}

// In-place variant for a block of THREADS threads transforming LINES lines of
// a compile-time length N held in one LDS buffer (line l at buf + l * LS):
// every thread first loads the inputs of all its butterflies, the block
// synchronises, then every thread writes its outputs to their Stockham
// positions.  One buffer instead of two, at the cost of one more barrier
// per pass.
template <typename T, int R, int N, int NS, int LINES, int THREADS, int LS>
__device__ __forceinline__ void stockham_pass_ip(cplx<T>* __restrict__ buf, const cplx<T>* __restrict__ tw) {
  constexpr unsigned nb = N / R;
  constexpr unsigned total = LINES * nb;
  constexpr unsigned bpt = (total + THREADS - 1) / THREADS;  // butterflies per thread
  constexpr unsigned tw_step = N / (NS * R);
  cplx<T> v[bpt][R];
#pragma unroll
  for (unsigned i = 0; i < bpt; ++i) {
    const unsigned q = threadIdx.x + i * THREADS;
    if (total % THREADS == 0 || q < total) {
      const unsigned l = q / nb, j = q - l * nb;
      const cplx<T>* s = buf + l * LS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[i][r] = s[j + r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (unsigned i = 0; i < bpt; ++i) {
    const unsigned q = threadIdx.x + i * THREADS;
    if (total % THREADS == 0 || q < total) {
      const unsigned l = q / nb, j = q - l * nb;
      const unsigned k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[k * r * tw_step]);
      }
      butterfly<T, R>(v[i]);
      cplx<T>* d = buf + l * LS + (j / NS) * (NS * R) + k;
#pragma unroll
      for (int r = 0; r < R; ++r) d[r * NS] = v[i][r];
    }
  }
  __syncthreads();
}

// All passes of the in-place transform, starting at pass S with stride NS.
template <typename T, int N, int LINES, int THREADS, int LS, int S = 0, int NS = 1>
__device__ void lds_fft_ip(cplx<T>* buf, const cplx<T>* tw) {
  if constexpr (S < Radices<N>::count) {
    constexpr int R = Radices<N>::radix(S);
    stockham_pass_ip<T, R, N, NS, LINES, THREADS, LS>(buf, tw);
    lds_fft_ip<T, N, LINES, THREADS, LS, S + 1, NS * R>(buf, tw);
  }
}

// Full transform of `lines` lines in LDS.  Returns the buffer holding the result.
template <typename T>
__device__ cplx<T>* lds_fft(cplx<T>* b0, cplx<T>* b1, const cplx<T>* tw, const FftShape& sh, int lines, int ls) {
  int ns = 1;
  cplx<T>* src = b0;
  cplx<T>* dst = b1;
  for (int s = 0; s < sh.nstages; ++s) {
    const int R = sh.radix[s];
    if (R == 4)
      stockham_pass<T, 4>(src, dst, tw, sh.n, ns, lines, ls);
    else if (R == 2)
      stockham_pass<T, 2>(src, dst, tw, sh.n, ns, lines, ls);
    else if (R == 3)
      stockham_pass<T, 3>(src, dst, tw, sh.n, ns, lines, ls);
    else
      stockham_pass<T, 5>(src, dst, tw, sh.n, ns, lines, ls);
    __syncthreads();
    ns *= R;
    cplx<T>* t = src;
    src = dst;
    dst = t;
  }
  return src;
}

}  // namespace bk
