// General sparse operators given in compressed sparse row form: residual and
// product, the CG direction update fused with the product, one colour class of
// a multicolour Gauss-Seidel sweep, and the aggregation transfers (orthonormal
// piecewise constants, Sec. 4.1).  Vectors are RHS-major blocks.  A thread
// takes one row (or one aggregate) and COLS right-hand sides, so each column
// index and value of the row is loaded once for COLS columns; the lanes of a
// wave take consecutive rows, whose gathers from x stay close in memory when
// neighbouring unknowns carry nearby indices.  Row sums run in the stored
// column order.  Indices are 32-bit (n, nnz < 2^31); column offsets 64-bit.
#include "kernels.h"

namespace mlmc {
namespace {

__device__ __forceinline__ bool col_on(const int* active, int col, int nb) {
  return col < nb && (!active || active[col]);
}

// r = b - A x (or r = A x when b is null); partials: per column and block of
// |r|^2 (or x^T A x)
template <typename Tb, typename T, typename Tr, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_residual(
    const Tb* __restrict__ b, const T* __restrict__ x, Tr* __restrict__ r,
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v, int n,
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
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) {
      const int j = ci[e];
      const T a = v[e];
#pragma unroll
      for (int q = 0; q < COLS; ++q)
        if (on[q]) acc[q] += a * x[(int64_t)(col0 + q) * n + j];
    }
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
    T* __restrict__ p_new, T* __restrict__ qv, const int* __restrict__ rp,
    const int* __restrict__ ci, const T* __restrict__ v, int n, int nb, const int* active,
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
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; ++e) {
      const int j = ci[e];
      const T a = v[e];
#pragma unroll
      for (int q = 0; q < COLS; ++q) {
        if (!on[q]) continue;
        const int64_t off = (int64_t)(col0 + q) * n;
        acc[q] += a * (z[off + j] + bt[q] * p_old[off + j]);
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

// one colour class of a Gauss-Seidel sweep, in place: for the sorted positions
// k0..k0+cnt-1 (rows crow[k] of one class, an independent set of the matrix
// graph) x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii; the off-diagonal entries
// of position k are cci/cv[cp[k]..cp[k+1]-1], cdi[k] = 1 / a_ii
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_gs(
    const T* __restrict__ b, T* __restrict__ x, const int* __restrict__ crow,
    const int* __restrict__ cp, const int* __restrict__ cci, const T* __restrict__ cv,
    const T* __restrict__ cdi, int k0, int cnt, int n, int nb, const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= cnt) return;
  const int k = k0 + t;
  const int i = crow[k];
  bool on[COLS];
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    on[q] = col_on(active, col0 + q, nb);
    acc[q] = on[q] ? b[(int64_t)(col0 + q) * n + i] : T(0);
  }
  const int e1 = cp[k + 1];
  for (int e = cp[k]; e < e1; ++e) {
    const int j = cci[e];
    const T a = cv[e];
#pragma unroll
    for (int q = 0; q < COLS; ++q)
      if (on[q]) acc[q] -= a * x[(int64_t)(col0 + q) * n + j];
  }
  const T d = cdi[k];
#pragma unroll
  for (int q = 0; q < COLS; ++q)
    if (on[q]) x[(int64_t)(col0 + q) * n + i] = acc[q] * d;
}

// rc_J = s_J sum_{i in J} (b - A x)_i when residual, else s_J sum_{i in J} x_i;
// a thread per aggregate J, whose members are arows[aptr[J]..aptr[J+1]-1]
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_csr_restrict(
    const T* __restrict__ b, const T* __restrict__ x, T* __restrict__ rc,
    const int* __restrict__ aptr, const int* __restrict__ arows, const T* __restrict__ cs,
    const int* __restrict__ rp, const int* __restrict__ ci, const T* __restrict__ v, int n,
    int nc, int residual, int nb, const int* active, int* tlog) {
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
    if (residual) {
      T s[COLS];
#pragma unroll
      for (int q = 0; q < COLS; ++q) s[q] = T(0);
      const int e1 = rp[i + 1];
      for (int e = rp[i]; e < e1; ++e) {
        const int j = ci[e];
        const T a = v[e];
#pragma unroll
        for (int q = 0; q < COLS; ++q)
          if (on[q]) s[q] += a * x[(int64_t)(col0 + q) * n + j];
      }
#pragma unroll
      for (int q = 0; q < COLS; ++q)
        if (on[q]) acc[q] += b[(int64_t)(col0 + q) * n + i] - s[q];
    } else {
#pragma unroll
      for (int q = 0; q < COLS; ++q)
        if (on[q]) acc[q] += x[(int64_t)(col0 + q) * n + i];
    }
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
                                      dim3(kThreads), 0, s, b, x, r, A.rp, A.ci, A.v, A.n, nb,
                                      active, partials, timing_log()));
}

template <typename T>
void csr_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                      const CsrMat<T>& A, int nb, int cols, const int* active, c64* partials,
                      hipStream_t s) {
  if (A.n == 0) return;
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_update_apply<T, C>), csr_grid(A.n, nb, C),
                                      dim3(kThreads), 0, s, p_old, z, beta, p_new, q, A.rp, A.ci,
                                      A.v, A.n, nb, active, partials, timing_log()));
}

template <typename T>
void csr_gs_sweep(const T* b, T* x, const CsrSweep<T>& S, int n, int nb, int cols,
                  const int* active, bool reverse, hipStream_t s) {
  const int classes = (int)S.coff.size() - 1;
  for (int t = 0; t < classes; ++t) {
    const int c = reverse ? classes - 1 - t : t;
    const int k0 = S.coff[c], cnt = S.coff[c + 1] - S.coff[c];
    if (cnt == 0) continue;
    CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_gs<T, C>), csr_grid(cnt, nb, C), dim3(kThreads), 0,
                                        s, b, x, S.crow, S.cp, S.cci, S.cv, S.cdi, k0, cnt, n, nb,
                                        active, timing_log()));
  }
}

template <typename T>
void csr_restrict(const T* b, const T* x, T* xc, const CsrMat<T>& A, const CsrAgg<T>& G,
                  bool residual, int nb, int cols, const int* active, hipStream_t s) {
  if (G.nc == 0) return;
  CSR_COLS_DISPATCH(cols, MLMC_LAUNCH((k_csr_restrict<T, C>), csr_grid(G.nc, nb, C),
                                      dim3(kThreads), 0, s, b, x, xc, G.aptr, G.arows, G.cs, A.rp,
                                      A.ci, A.v, A.n, G.nc, residual ? 1 : 0, nb, active,
                                      timing_log()));
}

template <typename T>
void csr_prolong(const T* ec, T* x, const CsrAgg<T>& G, int n, double omega, double beta, int nb,
                 const int* active, hipStream_t s) {
  if (n == 0) return;
  MLMC_LAUNCH(k_csr_prolong<T>, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb),
              dim3(kThreads), 0, s, ec, x, G.agg, G.fs, n, G.nc, (T)omega, (T)beta, active,
              timing_log());
}

void csr_dense(const CsrMat<double>& A, double* aug, hipStream_t s) {
  if (A.n == 0) return;
  MLMC_LAUNCH(k_csr_dense, dim3((unsigned)A.n), dim3(kThreads), 0, s, A.rp, A.ci, A.v, A.n, aug);
}

#define CSR_INST(T)                                                                           \
  template void csr_update_apply<T>(const T*, const T*, const c64*, T*, T*, const CsrMat<T>&,  \
                                    int, int, const int*, c64*, hipStream_t);                 \
  template void csr_gs_sweep<T>(const T*, T*, const CsrSweep<T>&, int, int, int, const int*,   \
                                bool, hipStream_t);                                           \
  template void csr_restrict<T>(const T*, const T*, T*, const CsrMat<T>&, const CsrAgg<T>&,    \
                                bool, int, int, const int*, hipStream_t);                     \
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
