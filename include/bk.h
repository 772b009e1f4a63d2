/*
 * bk.h -- C ABI of the MI355X bispectrum-multipole estimator.
 *
 * Computes the angular multipoles B_l^m(k1, mu, t) of the redshift-space
 * bispectrum of a gridded periodic field with the plane x annular-ring FFT
 * estimator of Gill & Bharadwaj (arXiv:2405.14513, Sec. II):
 *
 *   Delta(k)      forward 3-D DFT of delta(x), Delta = (V/N_g^3) DFT       (Sec. II)
 *   D(r, n, x)    sum over ring r of plane n of Delta(u, n) e^{-i u.x}     (Eq. 9)
 *   S(c)          sum_x D(r1,n1,x) D(r2,n2,x) D(r3,n3,x), n1+n2+n3 = 0     (Eq. 8)
 *   N_tri(c)      number of closed (u, v, w) in the three rings             (Eq. 10)
 *   B_l^m(bin)    sqrt((2l+1)/4pi) sum Y* B_hat N_tri / sum |Y|^2 N_tri     (Eq. 13)
 *
 * The sum over x in Eq. 8 only has to resolve wave vectors that close:
 * modes of the three rings reach |u_x|, |u_y| <= U_1, U_2, U_3, so on an
 * m x m grid with m > U_1 + U_2 + U_3 the only closure mod m is the exact one,
 * and S on that grid is (m / N_g)^2 times S on the N_g grid.  Each
 * combination is summed on the smallest such grid of size 2^a, 3 * 2^a or 5 * 2^a
 * (>= 16, and > 2 max U so D needs no wrapped modes), with D evaluated on
 * that grid: the same result, up to rounding, at a fraction of the points.
 *
 * Conventions (the paper leaves these open; the library fixes them):
 *   - wave vectors are integer lattice vectors, k in units of k_f = 2 pi / L;
 *     z (the fastest grid index) is the line of sight;
 *   - ring edges R_0 = 0, R_r = R_{r-1} + 2^floor((r-1)/10), last edge clipped
 *     to N_g/3, membership R_{r-1} <= |u| < R_r; mean radius = average |u|;
 *   - a combination is a multiset of three (ring, plane) sides with
 *     n1 + n2 + n3 = 0 and N_tri > 0, kept if k1 in [k1_min, k1_max) and
 *     mu, t in [0.5, 1] on the mean-value sides (Eq. 2);
 *   - Y* is replaced by its average over the two mirror images that every ring
 *     combination contains, N_lm P_l^m(p_z) cos(m phi) (Eq. 3 orientation,
 *     p_y >= 0), averaged over labellings of sides with equal k;
 *   - outputs are the even-l multipoles 0 <= m <= min(l, m_max), l <= l_max,
 *     ordered by l then m (16 values for l_max = m_max = 6); empty bins are NaN.
 *
 * Error behaviour: every call returns a bk_status; 0 is success.  Nothing is
 * thrown across the ABI.  bk_last_error() returns a message for the last
 * failing call on the calling thread (valid until that thread's next call).
 *
 * Ownership: the caller owns every host buffer it passes and every device
 * buffer it passes as input.  A plan owns all device memory it allocates and
 * releases it in bk_plan_destroy.  get_* calls copy into caller buffers and
 * fail with BK_ERR_SIZE if the capacity (in elements) is too small.
 */
#ifndef BK_H
#define BK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bk_plan_s* bk_plan;

typedef enum { BK_F32 = 1, BK_F64 = 2 } bk_prec;

typedef enum {
  BK_OK = 0,
  BK_ERR_ARG = -1,   /* invalid argument (sizes, ranges, null pointers)          */
  BK_ERR_STATE = -2, /* call out of order (e.g. estimate before a grid is loaded) */
  BK_ERR_SIZE = -3,  /* caller buffer too small                                  */
  BK_ERR_OOM = -4,   /* device or host allocation failed                         */
  BK_ERR_HIP = -5    /* a HIP runtime call failed; bk_last_error has the reason  */
} bk_status;

/* Second-level binning and outputs (Eq. 13).  k1 limits in units of k_f. */
typedef struct {
  int ng;            /* N_g per side: 2^a or 3*2^a, a multiple of 8, 8 <= N_g <= 512     */
  double box_len;    /* L (V = L^3); <= 0 means L = N_g (unit cell)                       */
  int n_k1;          /* linear k1 bins on [k1_min, k1_max)                                 */
  double k1_min;     /* >= 0                                                               */
  double k1_max;     /* <= N_g / 3 (periodic-box limit of the rings)                       */
  int n_mu;          /* linear mu bins on [0.5, 1], top bin closed                         */
  int n_t;           /* linear t bins on [0.5, 1], top bin closed                          */
  int l_max;         /* <= 12                                                              */
  int m_max;         /* <= l_max                                                           */
  int even_l_only;   /* 1: even l only; 0: every l (at most 64 (l, m) outputs), see below  */
} bk_binning;
/* Outputs are (l, m) with l = 0..l_max (every l, or even l only) and
 * m = 0..min(l, m_max).  For a real field a combination of sides and its
 * partner with every n negated carry conjugate sums S and, with the
 * mirror-averaged orientation weights, Y weights of equal sign for even l
 * and opposite sign for odd l.  So the numerator of Eq. 13 is real for even l
 * and imaginary for odd l.  Each output is the part that does not vanish:
 * sqrt((2l+1)/4pi) Re(num)/den for even l, sqrt((2l+1)/4pi) Im(num)/den for
 * odd l (computed from Im S).  Asking for odd l doubles the contraction's
 * matrix work. */

/* Build the geometry tables (rings, N_tri, combinations, weights, bins) on the
 * host and allocate the device working set on `device` for up to `max_batch`
 * fields of this size.  The tables are the paper's first-level geometry: the
 * plane x annular-ring cells with the ring widths of Sec. II's implementation
 * paragraph, N_tri of Eq. 10 per ring triple, the shape (Eq. 2) and
 * orientation (Eq. 3) of every combination, and its (k1, mu, t) bin and Y
 * weights for Eq. 13.  prec selects float32 (BK_F32: FFTs, D and the products
 * in float32, blocked float32 partial sums combined in float64) or float64
 * (BK_F64: every step in float64).  The final per-bin sums are float64 in both.
 * Setting the environment variable BK_FULL_GRID=1 sums every combination on
 * the full N_g x N_g grid instead (same results up to rounding; slower).
 * The contraction's work-item shape can be overridden the same way (results
 * equal up to rounding): BK_K3_PAIRS=32 or 64 (ring pairs per item, one item
 * per wave), BK_K3_ITEMS=1 or 2 (16-pair items per wave, default 2) and
 * BK_K3_SIDES (staged sides per workgroup, 1..254; with two items per wave at
 * most 159, since those workgroups stage into two fixed 160-slot buffers).
 * An invalid combination, or one whose staging does not fit the LDS, fails
 * with BK_ERR_ARG. */
bk_status bk_plan_create(const bk_binning* binning, int prec, int device, int max_batch, bk_plan* out);

/* A plan with several second-level binnings ("resolutions") of the same
 * combinations, as the validation of Sec. III uses finer (mu, t) bins for
 * low l than for high l.  Resolution 0 is `binning`'s own (n_k1, n_mu, n_t);
 * resolution r = 1..n_extra has the counts extra_bins[3(r-1) .. 3(r-1)+2]
 * (n_k1, n_mu, n_t), on the same k1 range and (l, m) list.  One estimate
 * runs the FFTs, ring sums and triple products once and the binning of
 * Eq. 13 once per resolution; every resolution's outputs are bit-identical
 * to those of a separate plan created with that binning.  Read them with the
 * *_res calls below (the calls without _res read resolution 0).  Errors as
 * bk_plan_create, plus BK_ERR_ARG if n_extra is not in [0, 7], extra_bins is
 * NULL with n_extra > 0, a count is < 1 or a resolution has over 10^7 bins.
 * bk_plan_create(b, ...) is bk_plan_create_multires(b, NULL, 0, ...). */
bk_status bk_plan_create_multires(const bk_binning* binning, const int* extra_bins, int n_extra, int prec, int device,
                                  int max_batch, bk_plan* out);
bk_status bk_plan_destroy(bk_plan plan);

/* Copy `batch` fields delta(x), C order [batch][x][y][z] (z = line of sight),
 * of type dtype (BK_F32 or BK_F64), into the plan: the gridded redshift-space
 * field delta^s(x) of Sec. II on N_g^3 cells of the periodic box V = L^3.  `delta` is a device pointer
 * if is_device_ptr != 0, else a host pointer.  The copy is enqueued on
 * hip_stream (a hipStream_t, NULL = default stream); a device input must stay
 * valid until the stream reaches this point. */
bk_status bk_load_grid(bk_plan plan, const void* delta, int dtype, int batch, int is_device_ptr,
                       void* hip_stream);

/* Enqueue the whole estimator for the loaded fields on hip_stream:
 * forward FFT, ring-masked 2-D FFTs (Step I, Eq. 9), triple-product sums
 * (Step II, Eq. 8) and the binned multipoles (Eq. 13).  Asynchronous; results
 * are read with get_*.  The plan's kernels are captured once into a hipGraph
 * (again when the loaded batch size, the input type or the tile choices
 * change) and every call replays it with one hipGraphLaunch; the graph
 * records no per-stage events, so bk_get_stage_times needs
 * bk_estimate_timed. */
bk_status bk_estimate(bk_plan plan, void* hip_stream);

/* The same estimate launched kernel by kernel, with hipEvents recorded on
 * hip_stream between the four stages (read them with bk_get_stage_times).
 * Results are identical to bk_estimate's. */
bk_status bk_estimate_timed(bk_plan plan, void* hip_stream);

/* Wait for all work the plan enqueued. */
bk_status bk_synchronize(bk_plan plan);

/* Output sizes: number of (l, m) pairs and bins per axis. */
bk_status bk_query_sizes(bk_plan plan, int* n_lm, int* n_k1, int* n_mu, int* n_t);

/* (l, m) of each output row, as pairs: lm_pairs[2 i] = l, lm_pairs[2 i + 1] = m. cap >= 2 n_lm. */
bk_status bk_get_lm_list(bk_plan plan, int* lm_pairs, size_t cap);

/* B_l^m as float64 [batch][n_lm][n_k1][n_mu][n_t] for the last estimate
 * (synchronises the plan's stream): the bin averages of Eq. 13,
 * sqrt((2l+1)/4pi) sum Y* B_hat N_tri / sum |Y|^2 N_tri over the bin's
 * combinations, with B_hat N_tri = S / (V N_g^2) from Eq. 8.  NaN where a bin
 * holds no combination.  cap >= batch * n_lm * n_bins. */
bk_status bk_get_multipoles(bk_plan plan, double* out, size_t cap);

/* Sum of N_tri (Eq. 10: ordered (u, v, w) with u + v + w = 0 in the three
 * rings) over the combinations of each bin, a combination and its n -> -n
 * partner both counted, int64 [n_k1][n_mu][n_t].  Geometry only (independent
 * of the field); exact. */
bk_status bk_get_triangle_counts(bk_plan plan, int64_t* out, size_t cap);

/* N_tri-weighted mean (k1, mu, t) of each bin (Eq. 2 on the combinations'
 * mean-value sides, weighted as in Eq. 13), float64 [n_bins][3]; NaN if empty. */
bk_status bk_get_bin_means(bk_plan plan, double* k1_mu_t, size_t cap);

/* Number of resolutions of the plan (1 + n_extra; 0 for a NULL plan). */
int bk_n_resolutions(bk_plan plan);

/* Bins per axis of resolution `res`.  BK_ERR_ARG if res is out of range. */
bk_status bk_query_resolution(bk_plan plan, int res, int* n_k1, int* n_mu, int* n_t);

/* bk_get_multipoles, bk_get_triangle_counts and bk_get_bin_means for
 * resolution `res` (its n_k1 x n_mu x n_t bins).  BK_ERR_ARG if res is out of
 * range; otherwise the same layout, synchronisation and errors. */
bk_status bk_get_multipoles_res(bk_plan plan, int res, double* out, size_t cap);
bk_status bk_get_triangle_counts_res(bk_plan plan, int res, int64_t* out, size_t cap);
bk_status bk_get_bin_means_res(bk_plan plan, int res, double* k1_mu_t, size_t cap);

/* Plan statistics, float64 [cap] with 9 <= cap (11 filled at most):
 * combinations (an n -> -n partner pair counted once), work items, sides,
 * rings, dense products per field (contraction terms incl. padding, summed
 * over each combination's grid points), useful products (combinations x their
 * grid points), device bytes held, number of canonical plane triples,
 * combinations that are their own partner, grid sides (a side evaluated on
 * one grid size), complex elements of D per field. */
bk_status bk_get_plan_info(bk_plan plan, double* info, size_t cap);

/* Device time of each stage in milliseconds, float64 [4]: forward FFT, ring
 * FFTs, triple products, binning (hipEvents recorded on the stream around
 * each stage), averaged over the consecutive timed estimates
 * (bk_estimate_timed) since the last bk_estimate or bk_load_grid, the latest
 * 32 at most.  With cap >= 5, out[4] receives the number averaged.
 * bk_plan_autotune and a bk_debug_set_D estimate leave one timed estimate.
 * BK_ERR_STATE if there is none. */
bk_status bk_get_stage_times(bk_plan plan, double* ms, size_t cap);

/* Tile autotuning.  With a grid loaded, times every valid tile choice of the
 * three tiled stages on hip_stream (lines per block of the forward FFT 2..16,
 * columns per block of the ring sums 4..16, staged slots per chunk of the
 * triple products 16..64, each within its LDS limit) and keeps the fastest of
 * each; the results do not depend on these choices beyond rounding order.
 * The choice is cached in the process per (N_g, precision, device, number of
 * sides, number of workgroups), and later plans with the same key start from
 * it.  Blocks until the timing is done.  On return the plan holds a complete
 * estimate of the loaded grid (stage times included).  choices, if not NULL,
 * receives int32 [3]: FFT lines, ring-sum columns, slots per chunk.  Errors:
 * BK_ERR_STATE with no grid loaded, BK_ERR_HIP from a failed launch (the
 * previous choices are then kept). */
bk_status bk_plan_autotune(bk_plan plan, void* hip_stream, int* choices);

/* A group of plans on one device (for example fields of different N_g, each
 * plan batched) estimated together.  On the first bk_group_estimate the
 * kernels of every plan are captured into one hipGraph with one branch per
 * plan; every call replays it with a single hipGraphLaunch on hip_stream.
 * The capture uses the batch each plan has loaded; loading a different batch
 * size into a member plan makes the next call capture again.  Every member
 * must have a grid loaded.  The plans stay owned by the caller and must
 * outlive the group; results are read from each plan with bk_get_*. */
typedef struct bk_group_s* bk_group;
bk_status bk_group_create(const bk_plan* plans, int n_plans, bk_group* out);
bk_status bk_group_estimate(bk_group group, void* hip_stream);
bk_status bk_group_destroy(bk_group group);

/* Host-only geometry (no device needed): the same per-bin sums of N_tri that
 * bk_get_triangle_counts returns, int64 [n_k1][n_mu][n_t], and optionally the
 * number of kept combinations (counting an n -> -n partner pair once).  Useful
 * to inspect a binning before committing device memory. */
bk_status bk_count_triangles(const bk_binning* binning, int64_t* out, size_t cap, int64_t* n_combinations);

/* The paper's model field, for its analytic predictions: power spectrum
 * P(k) = amp k^n_s (k in units of k_f = 2 pi / L, the same units as the
 * field's DFT normalisation), real-space bispectrum to first order in f_NG
 * (Eq. 15) B_r = 2 f_NG (P1 P2 + P2 P3 + P3 P1), linear redshift-space
 * distortion (Eq. 17) B_s = B_r prod_i (1 + beta mu_i^2). */
typedef struct {
  double amp;
  double n_s;
  double f_ng;
  double beta;
} bk_model;

/* Host-only: the discrete prediction [B_l^m]_d (Sec. III.C) for a binning:
 * B_s at every kept combination's mean-value sides (mu_i = n_i / k_i), binned
 * with exactly the estimator's weights and N_tri (Eq. 13).  Same layout and
 * units as bk_get_multipoles for one field, float64
 * [n_lm][n_k1][n_mu][n_t], NaN where the estimator's bin is empty; odd l are
 * exactly 0 in non-empty bins (the model is the same on a combination and
 * its n -> -n partner, whose odd-l weights cancel).  Builds the
 * plan geometry on the host (no device needed).  Errors: BK_ERR_ARG for an
 * invalid binning or non-finite model, BK_ERR_SIZE if cap is too small. */
bk_status bk_discrete_prediction(const bk_binning* binning, const bk_model* model, double* out, size_t cap);

/* Host-only: the continuum multipoles [B_l^m]_c / B_r (Eq. 4 with the
 * orientation of Eq. 3 and the angular factor of Eq. 17) for shape (mu, t),
 * in the output order of bk_get_lm_list for (l_max, m_max) (even l).  Exact
 * Gauss-Legendre x uniform-phase quadrature of the polynomial integrand.  The
 * ratio [B]_d / ([B]_c B_r) gives the discreteness weights of a bin.  Errors:
 * BK_ERR_ARG unless 0 <= m_max <= l_max <= 12, -1 <= mu <= 1, 0 < t <= 1 and
 * k3 > 0; BK_ERR_SIZE if cap is too small. */
bk_status bk_continuum_multipoles(int l_max, int m_max, double mu, double t, double beta, double* out, size_t cap);

/* Test support: copy an intermediate device buffer of the last estimate into
 * host memory.  which = 0: Delta planes, complex [batch][nkeep][N][N] (scaled
 * by N^-3/2, planes n = 0..nkeep-1, indices u mod N); 1: D of every grid side
 * (a stored side n >= 0 on one grid size m), complex [batch][sum of m^2] with
 * the grid sides one after the other, x_perp index x * m + y; 2: the grid-side
 * table in that order, int32 [grid sides][3] = (ring, n, m); 3, 4, 5: the contraction's work
 * items, workgroups and staged-side lists as stored on the host (raw bytes);
 * 6: the contraction outputs, float64 [batch][work item][cells], per item Re S
 * of cell (pair p, slot-B ring j) at p * 16 + j, then Im S of every cell when
 * odd l are requested (S = sum over the item's m x m grid of
 * D_A D_B conj(D_C) in the units of buffer 1; Eq. 8 on that grid).
 * Elements of 0 and 1 are float32 pairs for BK_F32 plans, float64 pairs for
 * BK_F64.  *needed receives the size in bytes; BK_ERR_SIZE if cap_bytes is
 * smaller.  Buffers 2-5 do not need a device. */
bk_status bk_debug_get_buffer(bk_plan plan, int which, void* out, size_t cap_bytes, size_t* needed);

/* Test support: copy `bytes` bytes from offset_bytes of device buffer 0, 1 or
 * 6 (as in bk_debug_get_buffer) of the last estimate into host memory, so
 * large grids can be sampled.  BK_ERR_SIZE if the range leaves the buffer. */
bk_status bk_debug_read_range(bk_plan plan, int which, size_t offset_bytes, void* out, size_t bytes);

/* Test support: set the ring sums D (Eq. 9) of `batch` fields directly, in the
 * layout and units of bk_debug_get_buffer's buffer 1 (complex of the plan's
 * precision), from a host or device pointer; the next bk_estimate then runs
 * only the triple products (Eq. 8) and the binning (Eq. 13) on it, as a
 * timed eager launch.  The copy is enqueued on hip_stream. */
bk_status bk_debug_set_D(bk_plan plan, const void* D, int batch, int is_device_ptr, void* hip_stream);

/* Test support: runs one 16x16x4 MFMA of the given precision (BK_F32 or BK_F64)
 * with A[i][k] = i + 16 k and B[k][j] = 1 if j == k else 0 (k < 4), and returns
 * per lane the four accumulator values, float64 [64][4], so tests can check
 * the lane layout the contraction kernel assumes. */
bk_status bk_debug_mfma_probe(int prec, double* out, size_t cap);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * estimate of bk_estimate for `batch` fields delta (a device pointer, C order
 * [batch][x][y][z], dtype BK_F32 or BK_F64) into B_out (a device pointer to
 * float64 [batch][n_lm][n_k1][n_mu][n_t], the layout of bk_get_multipoles).
 * The plan supplies its geometry tables (allocated at bk_plan_create); the
 * Delta planes, ring sums, contraction outputs and binning partials live in a
 * static device array of the library, 64 MiB per device (enough for one
 * N_g = 64 field in float64, two in float32), held by each device the library
 * runs on until the process ends.  Only resolution 0 is binned (a plan's
 * extra resolutions are left to bk_estimate).  The call allocates nothing, enqueues the
 * kernels on hip_stream and returns; it does not touch the plan's loaded
 * fields, results or stage times.  Errors: BK_ERR_ARG for null pointers, a
 * bad dtype or batch < 1; BK_ERR_SIZE (nothing launched) if the plan's
 * working set for `batch` fields exceeds the array.  Every call on one device
 * shares that device's array: calls that overlap in time on one device (on
 * different streams or host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are ordered and safe. */
bk_status bk_estimate_noalloc(bk_plan plan, const void* delta, int dtype, int batch, double* B_out,
                              void* hip_stream);

/* Message for the last failing call on this thread ("" if none). */
const char* bk_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BK_H */
