// General sparse operators given in compressed sparse row form: residual and
// product, the CG direction update fused with the product, one colour class of
// a multicolour Gauss-Seidel sweep, and the aggregation transfers (orthonormal
// piecewise constants, Sec. 4.1).  Vectors are RHS-major blocks.  The matrix
// is read from sliced ELLPACK copies (SELL-64, described with CsrMat): a wave
// takes the 64 rows of one slice, so each load of column indices and values is
// one coalesced 256-byte access and all lanes run the same trip count.  A
// thread takes one row (or one aggregate) and COLS right-hand sides, so each
// index and value is loaded once for COLS columns; the gathers from x stay
// close in memory when neighbouring unknowns carry nearby indices.  Row sums
// run in the stored column order.  Indices are 32-bit (n, nnz < 2^31); column
// offsets 64-bit.
#include "kernels.h"

namespace mlmc {
namespace {

__device__ __forceinline__ bool col_on(const int* active, int col, int nb) {
  return col < nb && (!active || active[col]);
}

// U entries of a SELL-64 row: indices and values first, then the gathers of
// every column, so U gathers per column are in flight; sums in entry order
template <typename T, int COLS, int U>
__device__ __forceinline__ void sell_chunk(const int* __restrict__ sci, const T* __restrict__ sv,
                                           int at, const T* __restrict__ x, int64_t n, int col0,
                                           const bool* on, T* acc) {
  int j[U];
  T a[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    j[u] = sci[at + u * 64];
    a[u] = sv[at + u * 64];
  }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    if (!on[q]) continue;
    const T* xq = x + (int64_t)(col0 + q) * n;
    T g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) g[u] = xq[j[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[q] += a[u] * g[u];
  }
}

// Row sum over one SELL-64 slice: acc[q] += sum_e v_e x_q[j_e] for the w
// entries of this lane's row, in stored order, in chunks of 8, 4 and 1
template <typename T, int COLS>
__device__ __forceinline__ void sell_row_sum(const int* __restrict__ sci,
                                             const T* __restrict__ sv, int base, int w,
                                             const T* __restrict__ x, int64_t n, int col0,
                                             const bool* on, T* acc) {
  int e = 0;
  for (; e + 8 <= w; e += 8) sell_chunk<T, COLS, 8>(sci, sv, base + e * 64, x, n, col0, on, acc);
  if (e + 4 <= w) {
    sell_chunk<T, COLS, 4>(sci, sv, base + e * 64, x, n, col0, on, acc);
    e += 4;
  }
  for (; e < w; ++e) sell_chunk<T, COLS, 1>(sci, sv, base + e * 64, x, n, col0, on, acc);
}

// r = b - A x (or r = A x when b is null); partials (nullable): per column and
// block of |r|^2 (or x^T A x).  Block = 4 slices = 256 consecutive rows.
template <typename Tb, typename T, typename Tr, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_residual(
    const Tb* __restrict__ b, const T* __restrict__ x, Tr* __restrict__ r,
    const int* __restrict__ sptr, const int* __restrict__ sci, const T* __restrict__ sv, int n,
    int nb, const int* active, c64* partials, int* tlog) {
  __shared__ double red[16];
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const bool in = i < n;
  bool on[COLS];
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);  // uniform over the block
    acc[q] = T(0);
  }
  if (in) {
    const int sl = i >> 6;
    const int base = sptr[sl] + (i & 63);
    sell_row_sum<T, COLS>(sci, sv, base, (sptr[sl + 1] - sptr[sl]) >> 6, x, n, col0, on, acc);
  }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    if (!on[q]) continue;
    const int64_t off = (int64_t)(col0 + q) * n;
    double dre = 0.0, dim = 0.0;
    if (in) {
      T val = acc[q];
      if (b) {
        val = convert<T, Tb>(b[off + i]) - val;
        cdot_acc(dre, dim, val, val);
      } else {
        cdot_acc(dre, dim, x[off + i], val);
      }
      r[off + i] = convert<Tr, T>(val);
    }
    if (partials) {
      block_sum2<kThreads>(dre, dim, red);
      if (threadIdx.x == 0) partials[(int64_t)(col0 + q) * gridDim.x + blockIdx.x] = {dre, dim};
    }
  }
}

// p_new = z + beta p_old ; q = A p_new ; partials of p_new^T q.  The
// neighbours' p_new values are recomputed from z and p_old, so the update and
// the product need a single pass.
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_update_apply(
    const T* __restrict__ p_old, const T* __restrict__ z, const c64* __restrict__ beta,
    T* __restrict__ p_new, T* __restrict__ qv, const int* __restrict__ sptr,
    const int* __restrict__ sci, const T* __restrict__ sv, int n, int nb, const int* active,
    c64* partials, int* tlog) {
  __shared__ double red[16];
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const bool in = i < n;
  bool on[COLS];
  T bt[COLS], acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);
    bt[q] = on[q] ? (T)beta[col0 + q].re : T(0);
    acc[q] = T(0);
  }
  if (in) {
    const int sl = i >> 6;
    const int base = sptr[sl] + (i & 63);
    const int w = (sptr[sl + 1] - sptr[sl]) >> 6;
    // chunks of 4 entries: indices and values first, then 8 gathers per column
    int e = 0;
    for (; e < w; e += 4) {
      const int m = w - e < 4 ? w - e : 4;
      int j[4];
      T a[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = u < m ? sci[base + (e + u) * 64] : i;
        a[u] = u < m ? sv[base + (e + u) * 64] : T(0);
      }
#pragma unroll
      for (int q = 0; q < COLS; ++q) {
        if (!on[q]) continue;
        const int64_t off = (int64_t)(col0 + q) * n;
        T zz[4], pp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          zz[u] = z[off + j[u]];
          pp[u] = p_old[off + j[u]];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (u < m) acc[q] += a[u] * (zz[u] + bt[q] * pp[u]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    if (!on[q]) continue;
    const int64_t off = (int64_t)(col0 + q) * n;
    double dre = 0.0, dim = 0.0;
    if (in) {
      const T pi = z[off + i] + bt[q] * p_old[off + i];
      p_new[off + i] = pi;
      qv[off + i] = acc[q];
      cdot_acc(dre, dim, pi, acc[q]);
    }
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)(col0 + q) * gridDim.x + blockIdx.x] = {dre, dim};
  }
}

// Row update of a Gauss-Seidel colour class, in place: position k = 64 sl +
// lane of slice sl holds row i = srow[k] (an independent set of the matrix
// graph; -1 pads the last slice of a class) and x_i = (b_i - sum_{j != i}
// a_ij x_j) / a_ii with the off-diagonal entries of the slice
template <typename T, int COLS>
__device__ __forceinline__ void gs_row(const T* __restrict__ b, T* __restrict__ x,
                                       const int* __restrict__ srow,
                                       const int* __restrict__ sptr,
                                       const int* __restrict__ sci, const T* __restrict__ sv,
                                       const T* __restrict__ sdi, int sl, int lane, int n,
                                       int col0, const bool* on) {
  const int k = sl * 64 + lane;
  const int i = srow[k];
  if (i < 0) return;
  T acc[COLS], sum[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    acc[q] = on[q] ? b[(int64_t)(col0 + q) * n + i] : T(0);
    sum[q] = T(0);
  }
  sell_row_sum<T, COLS>(sci, sv, sptr[sl] + lane, (sptr[sl + 1] - sptr[sl]) >> 6, x, n, col0,
                        on, sum);
  const T d = sdi[k];
#pragma unroll
  for (int q = 0; q < COLS; ++q)
    if (on[q]) x[(int64_t)(col0 + q) * n + i] = (acc[q] - sum[q]) * d;
}

// one colour class of a Gauss-Seidel sweep: the class owns slices s0..s1-1,
// a wave per slice
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_gs(
    const T* __restrict__ b, T* __restrict__ x, const int* __restrict__ srow,
    const int* __restrict__ sptr, const int* __restrict__ sci, const T* __restrict__ sv,
    const T* __restrict__ sdi, int s0, int s1, int n, int nb, const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int sl = s0 + blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (sl >= s1) return;
  bool on[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) on[q] = col_on(active, col0 + q, nb);
  gs_row<T, COLS>(b, x, srow, sptr, sci, sv, sdi, sl, threadIdx.x & 63, n, col0, on);
}

// Several consecutive colour classes of a sweep in one launch (the small
// classes a greedy colouring leaves at its end): one workgroup per column
// group runs the classes one after another, in the sweep's direction, its
// waves taking the slices of a class in turn; rows of one class are
// independent, so only the class boundaries need the workgroup's barrier
// (which also orders its waves' global stores before the next class's loads).
template <typename T, int COLS>
__global__ __launch_bounds__(kTailWaves * 64) void k_csr_gs_tail(
    const T* __restrict__ b, T* __restrict__ x, const int* __restrict__ srow,
    const int* __restrict__ sptr, const int* __restrict__ sci, const T* __restrict__ sv,
    const T* __restrict__ sdi, CsrTail t, int n, int nb, const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  bool on[COLS], any = false;
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);
    any = any || on[q];
  }
  if (!any) return;  // the whole workgroup: its columns are all inactive
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = 0; c < t.count; ++c) {
    const int cc = t.reverse ? t.count - 1 - c : c;
    for (int sl = t.soff[cc] + wave; sl < t.soff[cc + 1]; sl += kTailWaves)
      gs_row<T, COLS>(b, x, srow, sptr, sci, sv, sdi, sl, lane, n, col0, on);
    __syncthreads();
  }
}

// y = beta y + w M x, M rectangular (m rows, x of length nx per column)
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_spmm(
    const T* __restrict__ x, T* __restrict__ y, const int* __restrict__ sptr,
    const int* __restrict__ sci, const T* __restrict__ sv, int m, int nx, T w, T beta, int nb,
    const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= m) return;
  bool on[COLS];
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);
    acc[q] = T(0);
  }
  const int sl = i >> 6;
  sell_row_sum<T, COLS>(sci, sv, sptr[sl] + (i & 63), (sptr[sl + 1] - sptr[sl]) >> 6, x, nx,
                        col0, on, acc);
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    if (!on[q]) continue;
    T* yq = y + (int64_t)(col0 + q) * m + i;
    *yq = (beta == T(0)) ? w * acc[q] : beta * *yq + w * acc[q];
  }
}

// rc_J = s_J sum_{i in J} r_i, a thread per aggregate J, members in ascending order
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_agg_sum(
    const T* __restrict__ r, T* __restrict__ rc, const int* __restrict__ aptr,
    const int* __restrict__ arows, const T* __restrict__ cs, int n, int nc, int nb,
    const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int J = blockIdx.x * kThreads + threadIdx.x;
  if (J >= nc) return;
  bool on[COLS];
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);
    acc[q] = T(0);
  }
  const int m1 = aptr[J + 1];
  for (int m = aptr[J]; m < m1; ++m) {
    const int i = arows[m];
#pragma unroll
    for (int q = 0; q < COLS; ++q)
      if (on[q]) acc[q] += r[(int64_t)(col0 + q) * n + i];
  }
  const T sj = cs[J];
#pragma unroll
  for (int q = 0; q < COLS; ++q)
    if (on[q]) rc[(int64_t)(col0 + q) * nc + J] = sj * acc[q];
}

// x_i = beta x_i + w s_{J(i)} ec_{J(i)}  (x_i = w s ec when beta = 0)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_csr_prolong(
    const T* __restrict__ ec, T* __restrict__ x, const int* __restrict__ agg,
    const T* __restrict__ fs, int n, int nc, T w, T beta, const int* active, int* tlog) {
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const T e = w * fs[i] * ec[(int64_t)col * nc + agg[i]];
  T* xk = x + (int64_t)col * n;
  xk[i] = (beta == T(0)) ? e : beta * xk[i] + e;
}

// row i of the left half of the n x 2n augmented matrix: A's row
__global__ __launch_bounds__(kThreads) void k_csr_dense(const int* __restrict__ rp,
                                                        const int* __restrict__ ci,
                                                        const double* __restrict__ v, int n,
                                                        double* __restrict__ aug) {
  const int i = blockIdx.x;
  double* row = aug + (int64_t)i * 2 * n;
  for (int c = threadIdx.x; c < n; c += kThreads) row[c] = 0.0;
  __syncthreads();
  for (int e = rp[i] + threadIdx.x; e < rp[i + 1]; e += kThreads) row[ci[e]] = v[e];
}

}  // namespace

int csr_blocks(int n) { return (n + kThreads - 1) / kThreads; }

#define CSR_COLS_DISPATCH(COLSV, ...)                                           \
  switch (COLSV) {                                                             \
    case 1: { constexpr int C = 1; __VA_ARGS__; break; }                       \
    case 2: { constexpr int C = 2; __VA_ARGS__; break; }                       \
    case 4: { constexpr int C = 4; __VA_ARGS__; break; }                       \
    case 8: { constexpr int C = 8; __VA_ARGS__; break; }                       \
    default: throw Error(MLMC_EINVAL, "columns per thread must be 1, 2, 4 or 8"); \
  }

static dim3 csr_grid(int rows, int nb, int cols) {
  return dim3((unsigned)((rows + kThreads - 1) / kThreads), (unsigned)((nb + cols - 1) / cols));
}

template <typename Tb, typename T, typename Tr>
void csr_residual(const Tb* b, const T* x, Tr* r, const CsrMat<T>& A, int nb, int cols,
                  const int* active, c64* partials, hipStream_t s) {
  if (A.n == 0) return;
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_residual<Tb, T, Tr, C>), csr_grid(A.n, nb, C),
                                      dim3(kThreads), 0, s, b, x, r, A.sptr, A.sci, A.sv, A.n,
                                      nb, active, partials, timing_log()));
}

template <typename T>
void csr_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                      const CsrMat<T>& A, int nb, int cols, const int* active, c64* partials,
                      hipStream_t s) {
  if (A.n == 0) return;
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_update_apply<T, C>), csr_grid(A.n, nb, C),
                                      dim3(kThreads), 0, s, p_old, z, beta, p_new, q, A.sptr,
                                      A.sci, A.sv, A.n, nb, active, partials, timing_log()));
}

template <typename T>
void csr_gs_sweep(const T* b, T* x, const CsrSweep<T>& S, int n, int nb, int cols,
                  int tail_slices, const int* active, bool reverse, hipStream_t s) {
  const int classes = (int)S.soff.size() - 1;
  const int tail = csr_tail_start(S.soff, tail_slices);
  const unsigned gy = (unsigned)((nb + cols - 1) / cols);
  auto one_class = [&](int c) {
    const int s0 = S.soff[c], s1 = S.soff[c + 1];
    if (s1 == s0) return;
    const int per = kThreads / 64;  // slices per block
    const dim3 g((unsigned)((s1 - s0 + per - 1) / per), gy);
    CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_gs<T, C>), g, dim3(kThreads), 0, s, b, x, S.srow,
                                        S.sptr, S.sci, S.sv, S.sdi, s0, s1, n, nb, active,
                                        timing_log()));
  };
  auto fused = [&](int c0, int c1) {  // classes [c0, c1), at most kMaxTailClasses
    CsrTail t;
    t.count = c1 - c0;
    t.reverse = reverse ? 1 : 0;
    for (int c = c0; c <= c1; ++c) t.soff[c - c0] = S.soff[c];
    CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_gs_tail<T, C>), dim3(1u, gy),
                                        dim3(kTailWaves * 64), 0, s, b, x, S.srow, S.sptr,
                                        S.sci, S.sv, S.sdi, t, n, nb, active, timing_log()));
  };
  if (!reverse) {
    for (int c = 0; c < tail; ++c) one_class(c);
    for (int c0 = tail; c0 < classes; c0 += kMaxTailClasses)
      fused(c0, std::min(classes, c0 + kMaxTailClasses));
  } else {
    for (int c1 = classes; c1 > tail; c1 -= kMaxTailClasses)
      fused(std::max(tail, c1 - kMaxTailClasses), c1);
    for (int c = tail - 1; c >= 0; --c) one_class(c);
  }
}

template <typename T>
void csr_restrict(const T* b, const T* x, T* xc, T* rtmp, const CsrMat<T>& A,
                  const CsrAgg<T>& G, int nb, int cols, const int* active, hipStream_t s) {
  if (G.nc == 0) return;
  const T* src = x;
  if (b) {
    csr_residual<T, T, T>(b, x, rtmp, A, nb, cols, active, nullptr, s);
    src = rtmp;
  }
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_agg_sum<T, C>), csr_grid(G.nc, nb, C),
                                      dim3(kThreads), 0, s, src, xc, G.aptr, G.arows, G.cs, A.n,
                                      G.nc, nb, active, timing_log()));
}

template <typename T>
void csr_prolong(const T* ec, T* x, const CsrAgg<T>& G, int n, double omega, double beta, int nb,
                 const int* active, hipStream_t s) {
  if (n == 0) return;
  MLMC_LAUNCH(k_csr_prolong<T>, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb),
              dim3(kThreads), 0, s, ec, x, G.agg, G.fs, n, G.nc, (T)omega, (T)beta, active,
              timing_log());
}

template <typename T>
void csr_spmm(const T* x, T* y, const CsrMat<T>& M, double w, double beta, int nb, int cols,
              const int* active, hipStream_t s) {
  if (M.n == 0) return;
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_spmm<T, C>), csr_grid(M.n, nb, C), dim3(kThreads), 0,
                                      s, x, y, M.sptr, M.sci, M.sv, M.n, M.ncol, (T)w, (T)beta, nb,
                                      active, timing_log()));
}

void csr_dense(const CsrMat<double>& A, double* aug, hipStream_t s) {
  if (A.n == 0) return;
  MLMC_LAUNCH(k_csr_dense, dim3((unsigned)A.n), dim3(kThreads), 0, s, A.rp, A.ci, A.v, A.n, aug);
}

#define CSR_INST(T)                                                                           \
  template void csr_spmm<T>(const T*, T*, const CsrMat<T>&, double, double, int, int,          \
                            const int*, hipStream_t);                                         \
  template void csr_update_apply<T>(const T*, const T*, const c64*, T*, T*, const CsrMat<T>&,  \
                                    int, int, const int*, c64*, hipStream_t);                 \
  template void csr_gs_sweep<T>(const T*, T*, const CsrSweep<T>&, int, int, int, int,         \
                                const int*, bool, hipStream_t);                               \
  template void csr_restrict<T>(const T*, const T*, T*, T*, const CsrMat<T>&,                  \
                                const CsrAgg<T>&, int, int, const int*, hipStream_t);         \
  template void csr_prolong<T>(const T*, T*, const CsrAgg<T>&, int, double, double, int,       \
                               const int*, hipStream_t);
CSR_INST(float)
CSR_INST(double)
template void csr_residual<double, double, double>(const double*, const double*, double*,
                                                   const CsrMat<double>&, int, int, const int*,
                                                   c64*, hipStream_t);
template void csr_residual<double, double, float>(const double*, const double*, float*,
                                                  const CsrMat<double>&, int, int, const int*,
                                                  c64*, hipStream_t);
template void csr_residual<float, float, float>(const float*, const float*, float*,
                                                const CsrMat<float>&, int, int, const int*, c64*,
                                                hipStream_t);

}  // namespace mlmc
