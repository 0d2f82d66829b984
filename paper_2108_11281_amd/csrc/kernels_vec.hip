// Vector, reduction, Krylov-scalar, probe and dense kernels.
#include <type_traits>

#include "kernels.h"
#include "vec_body.h"

namespace mlmc {

namespace {

inline dim3 grid_cols(int64_t n, int nb, int per_thread = 1) {
  int64_t per_block = (int64_t)kThreads * per_thread;
  return dim3((unsigned)((n + per_block - 1) / per_block), (unsigned)nb);
}

template <typename T>
__global__ void k_zero(T* x, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) x[(int64_t)k * n + i] = zero_of(T());
}

template <typename To, typename From>
__global__ void k_convert(const From* x, To* y, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[(int64_t)k * n + i] = convert<To, From>(x[(int64_t)k * n + i]);
}

template <typename T>
__global__ void k_sub(const T* a, const T* b, T* out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    const int64_t j = (int64_t)blockIdx.y * n + i;
    out[j] = a[j] - b[j];
  }
}

template <typename T>
__global__ void k_add_to(T* y, const T* x, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    const int64_t j = (int64_t)k * n + i;
    y[j] = y[j] + x[j];
  }
}

// grid (nblk, nb): block b of column k reduces a contiguous chunk
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot(const T* x, const T* y, int64_t n,
                                                  const int* active, c64* partials) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  body::dot(x, y, n, gridDim.x, blockIdx.x, k, true, partials, lds, threadIdx.x);
}

__global__ __launch_bounds__(kThreads) void k_finish(const c64* partials, int nblk,
                                                     c64* out) {
  __shared__ double lds[16];
  const int k = blockIdx.x;
  const c64 v = body::finish(partials, nblk, k, lds);
  if (threadIdx.x == 0) out[k] = v;
}

// k_finish followed by the CG step length (k_finish_alpha) or direction
// coefficient (k_finish_beta) of the same column in one launch: the same sum
// in the same order, then the scalar rule of k_cg_alpha / k_cg_beta
__global__ __launch_bounds__(kThreads) void k_finish_alpha(const c64* partials, int nblk,
                                                           c64* pq, const c64* rz,
                                                           const int* active, c64* alpha) {
  __shared__ double lds[16];
  const int k = blockIdx.x;
  const c64 v = body::finish(partials, nblk, k, lds);
  if (threadIdx.x == 0) {
    pq[k] = v;
    body::alpha_rule(v, rz, active, k, alpha);
  }
}

__global__ __launch_bounds__(kThreads) void k_finish_beta(const c64* partials, int nblk,
                                                          c64* rz_new, c64* rz,
                                                          const int* active, c64* beta) {
  __shared__ double lds[16];
  const int k = blockIdx.x;
  const c64 v = body::finish(partials, nblk, k, lds);
  if (threadIdx.x == 0) {
    rz_new[k] = v;
    body::beta_rule(v, rz, active, k, beta);
  }
}

__global__ void k_cg_alpha(const c64* rz, const c64* pq, const int* active, c64* alpha,
                           int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  double a = 0.0;
  if ((!active || active[k]) && pq[k].re != 0.0 && isfinite(pq[k].re))
    a = rz[k].re / pq[k].re;
  alpha[k] = {a, 0.0};
}

__global__ void k_cg_beta(const c64* rz_new, c64* rz, const int* active, c64* beta,
                          int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  double b = 0.0;
  if ((!active || active[k]) && rz[k].re != 0.0) b = rz_new[k].re / rz[k].re;
  beta[k] = {b, 0.0};
  rz[k] = rz_new[k];
}

__global__ void k_mark(const c64* rr, const c64* ref, double tol2, int* active, int nb,
                       int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += blockDim.x)
    if (body::mark_rule(rr, ref, tol2, active, k)) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

__global__ void k_count(const int* active, int nb, int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += blockDim.x)
    if (active[k]) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

__global__ void k_ir_err(const c64* bd, const c64* rr_old, const c64* rr_new,
                         const int* active, c64* err, int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb || !active[k]) return;
  body::ir_err_rule(bd, rr_old, rr_new, err, k);
}

// after a refinement: where the new FP64 residual exceeds the FP32 recursion's
// own residual by more than `factor` (in squared norm), the kept direction no
// longer fits the new residual; zeroing rz makes the next beta 0 (a restart)
__global__ void k_cg_restart(const c64* rr_new, const c64* rr_rec, c64* rz, const int* active,
                             double factor, int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb || !active[k]) return;
  body::restart_rule(rr_new, rr_rec, rz, factor, k);
}

__global__ void k_set_count(int* c, int v) { *c = v; }

__global__ void k_refine_due(const c64* rr, const c64* rr_upd, const c64* bb, double delta2,
                             double tol2, const int* active, int nb, int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    if (!active[k]) continue;
    if (body::due_rule(rr, rr_upd, bb, delta2, tol2, k)) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

__global__ void k_set_ones(int* a, int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nb) a[k] = 1;
}

__global__ void k_select(c64* dst, const c64* src, const int* active, int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nb && active[k]) dst[k] = src[k];
}

__global__ void k_lastcorr(const c64* alpha, const c64* rz, const int* active, c64* lc,
                           int nb) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nb && (!active || active[k])) lc[k] = {alpha[k].re * rz[k].re, 0.0};
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_xr(T* x, T* r, const T* p, const T* q,
                                                    const c64* alpha, int64_t n,
                                                    const int* active, c64* partials,
                                                    int* tlog, int x_zero) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (active && !active[k]) return;
  body::cg_xr(x, r, p, q, alpha[k], n, gridDim.x, blockIdx.x, k, partials, lds, x_zero != 0);
}

template <typename T>
__global__ void k_cg_p(T* p, const T* z, const c64* beta, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t j = (int64_t)k * n + i;
  const c64 b = beta[k];
  p[j] = z[j] + scale_by(b.re, b.im, p[j]);
}

template <typename T64, typename T32>
__global__ void k_ir_acc(T64* y, const T32* d, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t j = (int64_t)k * n + i;
  y[j] = y[j] + convert<T64, T32>(d[j]);
}

// The FP64 refinement's fold of the FP32 correction (one pass, per column k;
// blocks as in k_dot)
template <typename Tb>
__global__ __launch_bounds__(kThreads) void k_ir_fold(double* y, float* d, const Tb* b,
                                                      int64_t n, const int* active,
                                                      c64* partials, int* tlog, int y_zero) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (active && !active[k]) return;
  body::ir_fold(y, d, b, n, gridDim.x, blockIdx.x, k, partials, lds, y_zero != 0);
}

// r = b32 = (float)b, *inexact = 1 when some b_i is not an FP32 number, and the
// partials of b^T b (the blocks and per-thread order of k_dot on (b, b), so the
// sums equal vec_dot_partials' bit for bit)
__global__ __launch_bounds__(kThreads) void k_rhs_fp32(const double* __restrict__ b,
                                                       float* __restrict__ r,
                                                       float* __restrict__ b32, int64_t n,
                                                       int* inexact, c64* partials) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  int64_t lo = 0, hi = 0;
  body::chunk_of(n, gridDim.x, blockIdx.x, lo, hi);
  const int64_t off = (int64_t)k * n;
  double re = 0.0, im = 0.0;
  bool exact = true;
  for (int64_t i = lo + threadIdx.x; i < hi; i += body::kNT) {
    const double v = b[off + i];
    const float f = (float)v;
    r[off + i] = f;
    b32[off + i] = f;
    exact = exact && (double)f == v;
    cdot_acc(re, im, v, v);
  }
  if (!exact) *inexact = 1;
  body::vsum2<body::kNT>(re, im, lds, threadIdx.x);
  if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {re, im};
}

__global__ void k_fill_ints(int* p, int count, int v) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename T>
__global__ void k_axpy_cols(T* y, const T* x, const c64* a, int64_t n, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t j = (int64_t)k * n + i;
  y[j] = y[j] + scale_by(a[k].re, a[k].im, x[j]);
}

// ---- probes: a block computes 256 Philox blocks into LDS, then expands them.
constexpr int kProbeWordsPerBlock = kThreads * 4;  // 64-bit words

template <typename T> struct ProbeLayout;
template <> struct ProbeLayout<double> { static constexpr int bits = 1; };
template <> struct ProbeLayout<float> { static constexpr int bits = 1; };
template <> struct ProbeLayout<c64> { static constexpr int bits = 2; };
template <> struct ProbeLayout<c32> { static constexpr int bits = 2; };

template <typename T>
__device__ __forceinline__ T probe_from_words(const uint64_t* words, int64_t local);

template <>
__device__ __forceinline__ double probe_from_words<double>(const uint64_t* w, int64_t l) {
  return ((w[l >> 6] >> (l & 63)) & 1ull) ? -1.0 : 1.0;
}
template <>
__device__ __forceinline__ float probe_from_words<float>(const uint64_t* w, int64_t l) {
  return ((w[l >> 6] >> (l & 63)) & 1ull) ? -1.f : 1.f;
}
template <>
__device__ __forceinline__ c64 probe_from_words<c64>(const uint64_t* w, int64_t l) {
  int f = (int)((w[l >> 5] >> (2 * (l & 31))) & 3ull);
  c64 r;
  r.re = (f == 0) ? 1.0 : (f == 2 ? -1.0 : 0.0);
  r.im = (f == 1) ? 1.0 : (f == 3 ? -1.0 : 0.0);
  return r;
}
template <>
__device__ __forceinline__ c32 probe_from_words<c32>(const uint64_t* w, int64_t l) {
  c64 z = probe_from_words<c64>(w, l);
  return {(float)z.re, (float)z.im};
}

// entries covered by one thread block: 256 Philox blocks of 256 bits
template <typename T> constexpr int64_t probe_chunk() {
  return (int64_t)kThreads * 256 / ProbeLayout<T>::bits;
}

template <typename T>
__device__ __forceinline__ void probe_fill_lds(uint64_t* words, int64_t chunk_index,
                                               const ProbeKey& key) {
  // Philox block index of this thread: entry e belongs to block e >> (8 - bits + 1)
  // i.e. 256 (Rademacher) or 128 (Z4) entries per Philox block.
  const uint64_t blk = (uint64_t)chunk_index * kThreads + threadIdx.x;
  u64x4 w = philox4x64_10(blk, key.sample, key.level, key.stream, key.seed, key.problem);
  words[4 * threadIdx.x + 0] = w.v[0];
  words[4 * threadIdx.x + 1] = w.v[1];
  words[4 * threadIdx.x + 2] = w.v[2];
  words[4 * threadIdx.x + 3] = w.v[3];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_probes(T* out, int64_t n, ProbeKey key) {
  __shared__ uint64_t words[kProbeWordsPerBlock];
  const int k = blockIdx.y;
  ProbeKey kk = key;
  kk.sample = key.sample + k;
  probe_fill_lds<T>(words, blockIdx.x, kk);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * probe_chunk<T>();
  T* o = out + (int64_t)k * n;
  for (int64_t l = threadIdx.x; l < probe_chunk<T>(); l += kThreads) {
    int64_t i = base + l;
    if (i < n) o[i] = probe_from_words<T>(words, l);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_probe_dot(const T* y, int64_t n, ProbeKey key,
                                                        c64* partials) {
  __shared__ uint64_t words[kProbeWordsPerBlock];
  __shared__ double lds[16];
  const int k = blockIdx.y;
  ProbeKey kk = key;
  kk.sample = key.sample + k;
  probe_fill_lds<T>(words, blockIdx.x, kk);
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * probe_chunk<T>();
  const T* yc = y + (int64_t)k * n;
  double re = 0.0, im = 0.0;
  // four loads of y in flight per thread, then the products in the order of a
  // plain strided loop (the chunk is a multiple of 4 * kThreads)
  constexpr int U = 4;
  static_assert(probe_chunk<T>() % (U * kThreads) == 0, "probe chunk");
  for (int64_t l0 = threadIdx.x; l0 < probe_chunk<T>(); l0 += U * kThreads) {
    T yv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + l0 + (int64_t)u * kThreads;
      const T v = yc[i < n ? i : 0];
      yv[u] = i < n ? v : zero_of(T());
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t l = l0 + (int64_t)u * kThreads;
      if (base + l < n) cdot_acc(re, im, probe_from_words<T>(words, l), yv[u]);
    }
  }
  block_sum2<kThreads>(re, im, lds);
  if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {re, im};
}

// ---- dense inverse: blocked Gauss-Jordan with partial pivoting -------------
// Sweep form of the elimination.  Pivoting on (row p, column c) with a = M[p][c]
// sets M[p][c] = 1/a, scales the rest of row p by 1/a, scales the rest of
// column c by -1/a and subtracts M[i][c] M[p][j] / a from every other entry.
// Column c's pivot p is its largest-modulus entry among the free rows (a row is
// free until it has been a pivot; rows are never moved).  With phys[c] the
// pivot row of column c, sweeping every column once leaves
//   M[phys[r]][j] = A^{-1}[r][phys[j]].
// Columns are swept in panels K of kGjPanel: the panel's own columns are swept
// one at a time, and the other columns J receive the whole panel's effect as
// one rank-|K| product with the panel's pivot rows as they stood before it,
//   M[i][J] <- [i not a pivot of K] M[i][J] + M[i][K] Mold[phys[K]][J].
// ipiv holds phys[0..n), then used[0..n) (0 = free, else the column it
// pivoted + 1), then a flag set when a pivot is zero or not a number (A
// singular).

__device__ __forceinline__ double recip(double a) { return 1.0 / a; }
__device__ __forceinline__ c64 recip(c64 a) {
  double d = a.re * a.re + a.im * a.im;
  return {a.re / d, -a.im / d};
}

__device__ __forceinline__ void gj_fma(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ __forceinline__ void gj_fma(c64& acc, c64 a, c64 b) {
  acc.re = fma(a.re, b.re, acc.re);
  acc.re = fma(-a.im, b.im, acc.re);
  acc.im = fma(a.re, b.im, acc.im);
  acc.im = fma(a.im, b.re, acc.im);
}

__global__ void k_gj_init(int* ipiv, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i <= 2 * n; i += gridDim.x * blockDim.x)
    ipiv[i] = 0;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gj_pivot(const T* M, int n, int64_t lda, int c,
                                                       int* ipiv) {
  __shared__ double bv[kThreads];
  __shared__ int bi[kThreads];
  const int* used = ipiv + n;
  double best = -1.0;
  int besti = n;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    if (used[i]) continue;
    double v = abs2_of(M[(int64_t)i * lda + c]);
    if (v > best || besti == n) {  // a NaN entry is taken only when nothing else is
      best = v;
      besti = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = besti;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      double o = bv[threadIdx.x + s];
      int oi = bi[threadIdx.x + s];
      const int mi = bi[threadIdx.x];
      if (oi != n && (mi == n || o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < mi))) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // a free row always exists (c < n rows have been used), so bi[0] < n; ties
    // go to the smallest row index
    ipiv[c] = bi[0];
    ipiv[n + bi[0]] = c + 1;
    if (!(bv[0] > 0.0)) ipiv[2 * n] = 1;
  }
}

// colbuf = column c, rowbuf[0..bw) = the pivot row's panel entries over a,
// rowbuf[bw] = 1/a
template <typename T>
__global__ void k_gj_extract(const T* M, int n, int64_t lda, int c, int k0, int bw,
                             const int* ipiv, T* rowbuf, T* colbuf) {
  const int p = ipiv[c];
  const T inv = recip(M[(int64_t)p * lda + c]);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    colbuf[t] = M[(int64_t)t * lda + c];
    if (t < bw) rowbuf[t] = M[(int64_t)p * lda + k0 + t] * inv;
    if (t == 0) rowbuf[bw] = inv;
  }
}

// sweep of column c restricted to the panel columns [k0, k0 + bw)
template <typename T>
__global__ void k_gj_panel(T* M, int n, int64_t lda, int c, int k0, int bw, const int* ipiv,
                           const T* rowbuf, const T* colbuf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * bw) return;
  const int i = (int)(t / bw), j = (int)(t % bw), col = k0 + j;
  const int p = ipiv[c];
  const T inv = rowbuf[bw];
  T& m = M[(int64_t)i * lda + col];
  if (i == p)
    m = (col == c) ? inv : rowbuf[j];
  else if (col == c)
    m = -(colbuf[i] * inv);
  else
    m = m - colbuf[i] * rowbuf[j];
}

// tbuf[r][j] = M[phys[k0 + r]][j]: the panel's pivot rows before their sweep
// reaches the columns outside the panel
template <typename T>
__global__ void k_gj_gather(const T* M, int n, int64_t lda, int k0, const int* ipiv, T* tbuf) {
  const int r = blockIdx.y;
  const int64_t src = (int64_t)ipiv[k0 + r] * lda;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    tbuf[(int64_t)r * n + j] = M[src + j];
}

// the panel's rank-bw update of every column outside it; 64 x 64 output tile
// per block, 4 x 4 per thread, the panel dimension staged through LDS 16 at a time
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gj_update(T* M, int n, int64_t lda, int k0,
                                                        int bw, const int* ipiv,
                                                        const T* tbuf) {
  constexpr int TR = 16;
  __shared__ T As[64][TR + 1];
  __shared__ T Ts[TR][64 + 1];
  const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
  if (col0 >= k0 && col0 + 64 <= k0 + bw) return;  // a tile inside the panel
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const T z = zero_of(T());
  T acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = z;
  for (int rb = 0; rb < bw; rb += TR) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + kThreads * q;
      const int ii = e >> 4, rr = e & 15;
      const int gi = row0 + ii;
      As[ii][rr] = (gi < n && rb + rr < bw) ? M[(int64_t)gi * lda + k0 + rb + rr] : z;
      const int jj = e & 63, r2 = e >> 6;
      const int gj = col0 + jj;
      Ts[r2][jj] = (gj < n && rb + r2 < bw) ? tbuf[(int64_t)(rb + r2) * n + gj] : z;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < TR; ++rr) {
      T av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[ty + 16 * a][rr];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Ts[rr][tx + 16 * b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gj_fma(acc[a][b], av[a], bv[b]);
    }
    __syncthreads();
  }
  const int* used = ipiv + n;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = row0 + ty + 16 * a;
    if (i >= n) continue;
    const bool pivot_row = used[i] > k0;  // pivoted one of the panel's columns
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int j = col0 + tx + 16 * b;
      if (j >= n || (j >= k0 && j < k0 + bw)) continue;
      T& m = M[(int64_t)i * lda + j];
      m = (pivot_row ? z : m) + acc[a][b];
    }
  }
}

// out[r][phys[j]] = M[phys[r]][j]
template <typename T>
__global__ void k_gj_unpermute(const T* M, int n, int64_t lda, const int* ipiv, T* out) {
  const int r = blockIdx.y;
  const int64_t src = (int64_t)ipiv[r] * lda;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    out[(int64_t)r * n + ipiv[j]] = M[src + j];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_trace(const T* A, int n, c64* out) {
  __shared__ double lds[16];
  double re = 0.0, im = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) {
    c64 one = {1.0, 0.0};
    T o = convert<T, c64>(one);
    cdot_acc(re, im, o, A[(int64_t)i * n + i]);
  }
  block_sum2<kThreads>(re, im, lds);
  if (threadIdx.x == 0) *out = {re, im};
}

// Z[k][i] = sum_j At[j][i] B[k][j] (At = A transposed, so a wave reads 64
// consecutive i): tile of 64 outputs i x 4 columns k per block; B rows in LDS.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_dense_apply(const T* At, const T* B, T* Z,
                                                          int n, int nb, const int* active) {
  constexpr int TK = 64;   // j tile
  __shared__ T bs[4][TK];
  const int i = blockIdx.x * 64 + (threadIdx.x & 63);
  const int kl = threadIdx.x >> 6;          // 0..3
  const int k = blockIdx.y * 4 + kl;
  const bool kok = k < nb && (!active || active[k]);
  T acc = zero_of(T());
  for (int j0 = 0; j0 < n; j0 += TK) {
    __syncthreads();
    {
      int jj = threadIdx.x & 63;
      bs[kl][jj] = (k < nb && j0 + jj < n) ? B[(int64_t)k * n + j0 + jj] : zero_of(T());
    }
    __syncthreads();
    if (i < n && kok) {
      const int jmax = (n - j0) < TK ? (n - j0) : TK;
      const T* acol = At + (int64_t)j0 * n + i;
      for (int jj = 0; jj < jmax; ++jj) acc += acol[(int64_t)jj * n] * bs[kl][jj];
    }
  }
  if (i < n && kok) Z[(int64_t)k * n + i] = acc;
}

// streaming copy (measurement of the sustained HBM rate): 16-byte loads and
// stores, four per thread with all loads issued before the stores
__global__ __launch_bounds__(kThreads) void k_stream_copy(const uint4* __restrict__ src,
                                                          uint4* __restrict__ dst, int64_t n16) {
  constexpr int U = 4;
  const int64_t base = (int64_t)blockIdx.x * kThreads * U + threadIdx.x;
  uint4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * kThreads;
    v[u] = i < n16 ? src[i] : uint4{0, 0, 0, 0};
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t i = base + (int64_t)u * kThreads;
    if (i < n16) dst[i] = v[u];
  }
}

// coarsest solve as an MFMA GEMM (the body's comment gives the tiling): a
// workgroup of kDenseParts waves per tile, one reduction range each, so every
// wave has a single round of loads in flight for coarsest levels up to 1024
// unknowns (the coarsest solves are latency-bound, not bandwidth-bound)
constexpr int kDenseThreads = body::kDenseParts * 64;
template <typename T>
__global__ __launch_bounds__(kDenseThreads) void k_dense_apply_mfma(const T* __restrict__ At,
                                                                    const T* __restrict__ B,
                                                                    T* __restrict__ Z, int n,
                                                                    int ld, int nb,
                                                                    const int* active) {
  __shared__ T part[body::kDenseParts * 4 * 64];
  body::dense_apply_mfma<T, body::kDenseParts>(At, B, Z, n, ld, nb, active, blockIdx.x,
                                               blockIdx.y, true, part, (int)threadIdx.x);
}

}  // namespace

// ============================================================================
template <typename T>
void vec_zero(T* x, int64_t n, int nb, const int* active, hipStream_t s) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_zero<T>, grid_cols(n, nb), dim3(kThreads), 0, s, x, n, active);
}
template <typename T>
void vec_copy(const T* x, T* y, int64_t n, int nb, const int* active, hipStream_t s) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL((k_convert<T, T>), grid_cols(n, nb), dim3(kThreads), 0, s, x, y, n,
                     active);
}
template <typename T>
void vec_sub(const T* a, const T* b, T* out, int64_t n, int nb, hipStream_t s) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_sub<T>, grid_cols(n, nb), dim3(kThreads), 0, s, a, b, out, n);
}
template <typename T>
void vec_add_to(T* y, const T* x, int64_t n, int nb, const int* active, hipStream_t s) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_add_to<T>, grid_cols(n, nb), dim3(kThreads), 0, s, y, x, n, active);
}
template <typename To, typename From>
void vec_convert(const From* x, To* y, int64_t n, int nb, const int* active, hipStream_t s) {
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL((k_convert<To, From>), grid_cols(n, nb), dim3(kThreads), 0, s, x, y, n,
                     active);
}

void stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return;
  const int64_t per_block = (int64_t)kThreads * 4;
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n16 + per_block - 1) / per_block)),
                     dim3(kThreads), 0, s, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), n16);
}

int*& timing_log() {
  thread_local int* slot = nullptr;
  return slot;
}

LaunchEvents*& timing_events() {
  thread_local LaunchEvents* slot = nullptr;
  return slot;
}

int reduce_blocks(int64_t n) {
  int64_t b = (n + 4 * kThreads - 1) / (4 * kThreads);
  if (b < 1) b = 1;
  if (b > kMaxPartials) b = kMaxPartials;
  return (int)b;
}

template <typename T>
void vec_dot_partials(const T* x, const T* y, int64_t n, int nb, const int* active,
                      c64* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dot<T>, dim3(reduce_blocks(n), nb), dim3(kThreads), 0, s, x, y, n,
                     active, partials);
}

void finish_sums(const c64* partials, int nblk, int nb, c64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(nb), dim3(kThreads), 0, s, partials, nblk, out);
}

void finish_alpha(const c64* partials, int nblk, int nb, c64* pq, const c64* rz,
                  const int* active, c64* alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_alpha, dim3(nb), dim3(kThreads), 0, s, partials, nblk, pq, rz,
                     active, alpha);
}
void finish_beta(const c64* partials, int nblk, int nb, c64* rz_new, c64* rz, const int* active,
                 c64* beta, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_beta, dim3(nb), dim3(kThreads), 0, s, partials, nblk, rz_new, rz,
                     active, beta);
}
void cg_alpha(const c64* rz, const c64* pq, const int* active, c64* alpha, int nb,
              hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3((nb + 255) / 256), dim3(256), 0, s, rz, pq, active,
                     alpha, nb);
}
void cg_beta(const c64* rz_new, c64* rz, const int* active, c64* beta, int nb,
             hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3((nb + 255) / 256), dim3(256), 0, s, rz_new, rz, active,
                     beta, nb);
}
void mark_converged(const c64* rr, const c64* ref, double tol2, int* active, int nb,
                    int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_mark, dim3(1), dim3(256), 0, s, rr, ref, tol2, active, nb, count);
}
void count_active(const int* active, int nb, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(256), 0, s, active, nb, count);
}

void cg_restart_on_drift(const c64* rr_new, const c64* rr_rec, c64* rz, const int* active,
                         double factor, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_restart, dim3((nb + 255) / 256), dim3(256), 0, s, rr_new, rr_rec, rz,
                     active, factor, nb);
}
void ir_stated_error(const c64* bd, const c64* rr_old, const c64* rr_new, const int* active,
                     c64* err, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_err, dim3((nb + 255) / 256), dim3(256), 0, s, bd, rr_old, rr_new,
                     active, err, nb);
}
void refine_due(const c64* rr, const c64* rr_upd, const c64* bb, double delta2, double tol2,
                const int* active, int nb, int* count, hipStream_t s) {
  hipLaunchKernelGGL(k_refine_due, dim3(1), dim3(256), 0, s, rr, rr_upd, bb, delta2, tol2,
                     active, nb, count);
}
void set_count(int* count, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_count, dim3(1), dim3(1), 0, s, count, value);
}
void set_all_active(int* active, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_set_ones, dim3((nb + 255) / 256), dim3(256), 0, s, active, nb);
}
void select_active(c64* dst, const c64* src, const int* active, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3((nb + 255) / 256), dim3(256), 0, s, dst, src, active, nb);
}
void cg_lastcorr(const c64* alpha, const c64* rz, const int* active, c64* lastcorr, int nb,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_lastcorr, dim3((nb + 255) / 256), dim3(256), 0, s, alpha, rz, active,
                     lastcorr, nb);
}

template <typename T>
void cg_update_xr(T* x, T* r, const T* p, const T* q, const c64* alpha, int64_t n, int nb,
                  const int* active, c64* partials, hipStream_t s, bool x_zero) {
  MLMC_LAUNCH(k_cg_xr<T>, dim3(reduce_blocks(n), nb), dim3(kThreads), 0, s, x, r, p, q, alpha,
              n, active, partials, timing_log(), x_zero ? 1 : 0);
}
template <typename T>
void cg_update_p(T* p, const T* z, const c64* beta, int64_t n, int nb, const int* active,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p<T>, grid_cols(n, nb), dim3(kThreads), 0, s, p, z, beta, n,
                     active);
}
void ir_fold(double* y, float* d, const double* b, int64_t n, int nb, const int* active,
             c64* partials, hipStream_t s, bool y_zero) {
  if (n <= 0 || nb <= 0) return;
  MLMC_LAUNCH(k_ir_fold<double>, dim3(reduce_blocks(n), nb), dim3(kThreads), 0, s, y, d, b, n,
              active, partials, timing_log(), y_zero ? 1 : 0);
}
void ir_fold(double* y, float* d, const float* b, int64_t n, int nb, const int* active,
             c64* partials, hipStream_t s, bool y_zero) {
  if (n <= 0 || nb <= 0) return;
  MLMC_LAUNCH(k_ir_fold<float>, dim3(reduce_blocks(n), nb), dim3(kThreads), 0, s, y, d, b, n,
              active, partials, timing_log(), y_zero ? 1 : 0);
}
void rhs_fp32(const double* b, float* r, float* b32, int64_t n, int nb, int* inexact,
              c64* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_ints, dim3(1), dim3(kThreads), 0, s, inexact, 1, 0);
  if (n <= 0 || nb <= 0) return;
  hipLaunchKernelGGL(k_rhs_fp32, dim3(reduce_blocks(n), nb), dim3(kThreads), 0, s, b, r, b32,
                     n, inexact, partials);
}
template <typename T64, typename T32>
void ir_accumulate(T64* y, const T32* d, int64_t n, int nb, const int* active,
                   hipStream_t s) {
  hipLaunchKernelGGL((k_ir_acc<T64, T32>), grid_cols(n, nb), dim3(kThreads), 0, s, y, d, n,
                     active);
}
template <typename T>
void vec_axpy_cols(T* y, const T* x, const c64* a, int64_t n, int nb, const int* active,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_cols<T>, grid_cols(n, nb), dim3(kThreads), 0, s, y, x, a, n,
                     active);
}

template <typename T>
void probes_write(T* out, int64_t n, int nb, uint64_t seed, uint64_t problem,
                  uint64_t first_sample, uint64_t level, uint64_t stream, hipStream_t s) {
  ProbeKey key{seed, problem, first_sample, level, stream};
  const int64_t chunk = probe_chunk<T>();
  dim3 grid((unsigned)((n + chunk - 1) / chunk), (unsigned)nb);
  hipLaunchKernelGGL(k_probes<T>, grid, dim3(kThreads), 0, s, out, n, key);
}

template <typename T>
void probe_dot_partials(const T* y, int64_t n, int nb, uint64_t seed, uint64_t problem,
                        uint64_t first_sample, uint64_t level, uint64_t stream,
                        c64* partials, hipStream_t s) {
  ProbeKey key{seed, problem, first_sample, level, stream};
  const int64_t chunk = probe_chunk<T>();
  dim3 grid((unsigned)((n + chunk - 1) / chunk), (unsigned)nb);
  hipLaunchKernelGGL(k_probe_dot<T>, grid, dim3(kThreads), 0, s, y, n, key, partials);
}

template <typename T>
void dense_inverse(T* M, int n, int64_t lda, T* out, T* rowbuf, T* colbuf, T* tbuf,
                   int* ipiv, hipStream_t s) {
  const unsigned gn = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_gj_init, dim3((2 * n + 256) / 256), dim3(256), 0, s, ipiv, n);
  for (int k0 = 0; k0 < n; k0 += kGjPanel) {
    const int bw = std::min(kGjPanel, n - k0);
    const unsigned gp = (unsigned)(((int64_t)n * bw + 255) / 256);
    for (int c = k0; c < k0 + bw; ++c) {
      hipLaunchKernelGGL(k_gj_pivot<T>, dim3(1), dim3(kThreads), 0, s, M, n, lda, c, ipiv);
      hipLaunchKernelGGL(k_gj_extract<T>, dim3(gn), dim3(256), 0, s, M, n, lda, c, k0, bw,
                         ipiv, rowbuf, colbuf);
      hipLaunchKernelGGL(k_gj_panel<T>, dim3(gp), dim3(256), 0, s, M, n, lda, c, k0, bw, ipiv,
                         rowbuf, colbuf);
    }
    if (bw == n) continue;
    hipLaunchKernelGGL(k_gj_gather<T>, dim3(gn, bw), dim3(256), 0, s, M, n, lda, k0, ipiv,
                       tbuf);
    const unsigned gt = (unsigned)((n + 63) / 64);
    hipLaunchKernelGGL(k_gj_update<T>, dim3(gt, gt), dim3(kThreads), 0, s, M, n, lda, k0, bw,
                       ipiv, tbuf);
  }
  hipLaunchKernelGGL(k_gj_unpermute<T>, dim3(gn, n), dim3(256), 0, s, M, n, lda, ipiv, out);
}

template <typename T>
void dense_trace(const T* A, int n, c64* out, hipStream_t s) {
  hipLaunchKernelGGL(k_trace<T>, dim3(1), dim3(kThreads), 0, s, A, n, out);
}

template <typename T>
void dense_apply(const T* At, const T* B, T* Z, int n, int nb, const int* active,
                 hipStream_t s, int ld) {
  if (ld == 0) ld = n;
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (dense_mfma_layout<T>(ld)) {
      dim3 grid((unsigned)(ld / 16), (unsigned)((nb + 15) / 16));
      hipLaunchKernelGGL(k_dense_apply_mfma<T>, grid, dim3(kDenseThreads), 0, s, At, B, Z, n,
                         ld, nb, active);
      return;
    }
  }
  if (ld != n) throw Error(MLMC_EINVAL, "dense_apply: padded inverse needs ld % 16 == 0");
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nb + 3) / 4));
  hipLaunchKernelGGL(k_dense_apply<T>, grid, dim3(kThreads), 0, s, At, B, Z, n, nb, active);
}

// ---- explicit instantiations ----------------------------------------------
#define MLMC_INST_T(T)                                                                    \
  template void vec_zero<T>(T*, int64_t, int, const int*, hipStream_t);                  \
  template void vec_copy<T>(const T*, T*, int64_t, int, const int*, hipStream_t);        \
  template void vec_sub<T>(const T*, const T*, T*, int64_t, int, hipStream_t);           \
  template void vec_add_to<T>(T*, const T*, int64_t, int, const int*, hipStream_t);       \
  template void vec_dot_partials<T>(const T*, const T*, int64_t, int, const int*, c64*,  \
                                    hipStream_t);                                        \
  template void cg_update_xr<T>(T*, T*, const T*, const T*, const c64*, int64_t, int,    \
                                const int*, c64*, hipStream_t, bool);                    \
  template void cg_update_p<T>(T*, const T*, const c64*, int64_t, int, const int*,       \
                               hipStream_t);                                             \
  template void vec_axpy_cols<T>(T*, const T*, const c64*, int64_t, int, const int*,     \
                                 hipStream_t);                                           \
  template void probes_write<T>(T*, int64_t, int, uint64_t, uint64_t, uint64_t, uint64_t, \
                                uint64_t, hipStream_t);                                  \
  template void probe_dot_partials<T>(const T*, int64_t, int, uint64_t, uint64_t,        \
                                      uint64_t, uint64_t, uint64_t, c64*, hipStream_t);  \
  template void dense_trace<T>(const T*, int, c64*, hipStream_t);                        \
  template void dense_apply<T>(const T*, const T*, T*, int, int, const int*, hipStream_t, int);

MLMC_INST_T(float)
MLMC_INST_T(double)
MLMC_INST_T(c32)
MLMC_INST_T(c64)

template void dense_inverse<double>(double*, int, int64_t, double*, double*, double*, double*,
                                    int*, hipStream_t);
template void dense_inverse<c64>(c64*, int, int64_t, c64*, c64*, c64*, c64*, int*,
                                 hipStream_t);

template void vec_convert<float, double>(const double*, float*, int64_t, int, const int*,
                                         hipStream_t);
template void vec_convert<double, float>(const float*, double*, int64_t, int, const int*,
                                         hipStream_t);
template void vec_convert<c32, c64>(const c64*, c32*, int64_t, int, const int*, hipStream_t);
template void vec_convert<c64, c32>(const c32*, c64*, int64_t, int, const int*, hipStream_t);
template void ir_accumulate<double, float>(double*, const float*, int64_t, int, const int*,
                                           hipStream_t);
template void ir_accumulate<c64, c32>(c64*, const c32*, int64_t, int, const int*,
                                      hipStream_t);
template void ir_accumulate<double, double>(double*, const double*, int64_t, int,
                                            const int*, hipStream_t);
template void ir_accumulate<c64, c64>(c64*, const c64*, int64_t, int, const int*,
                                      hipStream_t);

}  // namespace mlmc

namespace mlmc {
namespace {
template <typename T>
__global__ void k_transpose(const T* in, T* out, int n) {
  const int i = blockIdx.y;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x)
    out[(int64_t)j * n + i] = in[(int64_t)i * n + j];
}
}  // namespace
template <typename T>
void dense_transpose(const T* in, T* out, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose<T>, dim3((n + 255) / 256, n), dim3(256), 0, s, in, out, n);
}
namespace {
template <typename T>
__global__ void k_pack4(const T* __restrict__ in, T* __restrict__ out, int ld) {
  const int j = blockIdx.y;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < ld; i += gridDim.x * blockDim.x)
    out[((int64_t)(j >> 2) * ld + i) * 4 + (j & 3)] = in[(int64_t)j * ld + i];
}
}  // namespace
template <typename T>
void dense_pack4(const T* At, T* out, int ld, hipStream_t s) {
  if (ld % 4 != 0) throw Error(MLMC_EINVAL, "dense_pack4: ld must be a multiple of 4");
  hipLaunchKernelGGL(k_pack4<T>, dim3((ld + 255) / 256, ld), dim3(256), 0, s, At, out, ld);
}
// real representation of a complex matrix for the real MFMA product: with
// A_ij = At[j][i] (complex, transposed), M (2n x 2n) acts on interleaved
// (re, im) vectors -- M[2i+a][2j+c] = Re A_ij if a == c, -Im A_ij for (0, 1),
// Im A_ij for (1, 0) -- and is written transposed: Mt[j'][i'] = M[i'][j']
template <typename T, typename R>
__global__ void k_complex_to_real(const T* __restrict__ At, R* __restrict__ Mt, int n) {
  const int n2 = 2 * n;
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;  // i'
  const int jp = blockIdx.y;                             // j'
  if (ip >= n2) return;
  const int i = ip >> 1, a = ip & 1, j = jp >> 1, c = jp & 1;
  const T v = At[(int64_t)j * n + i];
  const R m = (a == c) ? v.re : (a == 0 ? -v.im : v.im);
  Mt[(int64_t)jp * n2 + ip] = m;
}

template <typename T, typename R>
void dense_complex_to_real(const T* At, R* Mt, int n, hipStream_t s) {
  hipLaunchKernelGGL((k_complex_to_real<T, R>), dim3((2 * n + 255) / 256, 2 * n), dim3(256), 0,
                     s, At, Mt, n);
}
template void dense_complex_to_real<c32, float>(const c32*, float*, int, hipStream_t);
template void dense_complex_to_real<c64, double>(const c64*, double*, int, hipStream_t);

template void dense_transpose<float>(const float*, float*, int, hipStream_t);
template void dense_transpose<double>(const double*, double*, int, hipStream_t);
template void dense_transpose<c32>(const c32*, c32*, int, hipStream_t);
template void dense_transpose<c64>(const c64*, c64*, int, hipStream_t);
template void dense_pack4<float>(const float*, float*, int, hipStream_t);
template void dense_pack4<double>(const double*, double*, int, hipStream_t);
}  // namespace mlmc
