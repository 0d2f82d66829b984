// 2D Poisson stencil kernels, matrix-free: A = d I - c (grid neighbours) on an
// N x N Dirichlet grid, unknown i = y*N + x.  With 2x2 orthonormal aggregation
// the Galerkin operator of such a stencil is again one (d' = d - 2c, c' = c/2),
// so every level of the hierarchy runs on these kernels.
#include "kernels.h"

namespace mlmc {
namespace {

template <typename T> using R_t = typename Traits<T>::real;

// neighbour sum with Dirichlet truncation
template <typename T>
__device__ __forceinline__ T nbr_sum(const T* u, int x, int y, int N, int64_t i) {
  T s = zero_of(T());
  if (x > 0) s += u[i - 1];
  if (x < N - 1) s += u[i + 1];
  if (y > 0) s += u[i - N];
  if (y < N - 1) s += u[i + N];
  return s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_apply(const T* x, T* y, int N, R_t<T> d,
                                                    R_t<T> c, const int* active,
                                                    c64* partials) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t n = (int64_t)N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const T* xc = x + (int64_t)k * n;
  double re = 0.0, im = 0.0;
  if (i < n) {
    const int yy = (int)(i / N), xx = (int)(i - (int64_t)yy * N);
    T xi = xc[i];
    T v = d * xi - c * nbr_sum(xc, xx, yy, N, i);
    y[(int64_t)k * n + i] = v;
    cdot_acc(re, im, xi, v);
  }
  if (partials) {
    block_sum2<kThreads>(re, im, lds);
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {re, im};
  }
}

template <typename Tb, typename Tx, typename Tr>
__global__ __launch_bounds__(kThreads) void k_residual(const Tb* b, const Tx* x, Tr* r, int N,
                                                       R_t<Tx> d, R_t<Tx> c,
                                                       const int* active, c64* partials) {
  __shared__ double lds[16];
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t n = (int64_t)N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const Tx* xc = x + (int64_t)k * n;
  double re = 0.0, im = 0.0;
  if (i < n) {
    const int yy = (int)(i / N), xx = (int)(i - (int64_t)yy * N);
    Tx v = convert<Tx, Tb>(b[(int64_t)k * n + i]) - (d * xc[i] - c * nbr_sum(xc, xx, yy, N, i));
    r[(int64_t)k * n + i] = convert<Tr, Tx>(v);
    cdot_acc(re, im, v, v);
  }
  if (partials) {
    block_sum2<kThreads>(re, im, lds);
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {re, im};
  }
}

// one colour of a red-black Gauss-Seidel sweep, in place
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gs_colour(const T* b, T* x, int N, R_t<T> dinv,
                                                        R_t<T> c, int colour, int zero_nbrs,
                                                        const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t n = (int64_t)N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int yy = (int)(i / N), xx = (int)(i - (int64_t)yy * N);
  if (((xx + yy) & 1) != colour) return;
  T* xc = x + (int64_t)k * n;
  const T bi = b[(int64_t)k * n + i];
  if (zero_nbrs)
    xc[i] = dinv * bi;
  else
    xc[i] = dinv * (bi + c * nbr_sum(xc, xx, yy, N, i));
}

// one thread per coarse point: rc = 1/2 sum over the 2x2 block of (b - A x)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_res_restrict(const T* b, const T* x, T* rc,
                                                           int N, R_t<T> d, R_t<T> c,
                                                           const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int Nc = N / 2;
  const int64_t nc = (int64_t)Nc * Nc, n = (int64_t)N * N;
  const int64_t I = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (I >= nc) return;
  const int Y = (int)(I / Nc), X = (int)(I - (int64_t)Y * Nc);
  const T* xc = x + (int64_t)k * n;
  const T* bc = b + (int64_t)k * n;
  T acc = zero_of(T());
#pragma unroll
  for (int dy = 0; dy < 2; ++dy)
#pragma unroll
    for (int dx = 0; dx < 2; ++dx) {
      const int xx = 2 * X + dx, yy = 2 * Y + dy;
      const int64_t i = (int64_t)yy * N + xx;
      acc += bc[i] - (d * xc[i] - c * nbr_sum(xc, xx, yy, N, i));
    }
  rc[(int64_t)k * nc + I] = (R_t<T>)0.5 * acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(const T* x, T* xcoarse, int N,
                                                       const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int Nc = N / 2;
  const int64_t nc = (int64_t)Nc * Nc, n = (int64_t)N * N;
  const int64_t I = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (I >= nc) return;
  const int Y = (int)(I / Nc), X = (int)(I - (int64_t)Y * Nc);
  const T* xc = x + (int64_t)k * n;
  const int64_t i0 = (int64_t)(2 * Y) * N + 2 * X;
  T acc = xc[i0] + xc[i0 + 1] + xc[i0 + N] + xc[i0 + N + 1];
  xcoarse[(int64_t)k * nc + I] = (R_t<T>)0.5 * acc;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong(const T* ec, T* x, int N, R_t<T> omega_half,
                                                      R_t<T> beta, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int Nc = N / 2;
  const int64_t nc = (int64_t)Nc * Nc, n = (int64_t)N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int yy = (int)(i / N), xx = (int)(i - (int64_t)yy * N);
  const T e = ec[(int64_t)k * nc + (int64_t)(yy >> 1) * Nc + (xx >> 1)];
  T* xcol = x + (int64_t)k * n;
  if (beta == (R_t<T>)0)
    xcol[i] = omega_half * e;
  else
    xcol[i] = beta * xcol[i] + omega_half * e;
}

template <typename T>
__global__ void k_dense_build(T* M, int N, R_t<T> d, R_t<T> c) {
  const int64_t n = (int64_t)N * N, ld = 2 * n;
  const int64_t i = blockIdx.y;
  const int yy = (int)(i / N), xx = (int)(i - (int64_t)yy * N);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int jy = (int)(j / N), jx = (int)(j - (int64_t)jy * N);
    T v = zero_of(T());
    if (j == i)
      v = d;
    else if ((jy == yy && (jx == xx - 1 || jx == xx + 1)) ||
             (jx == xx && (jy == yy - 1 || jy == yy + 1)))
      v = -c;
    M[i * ld + j] = v;
  }
}

inline dim3 grid_pts(int64_t n, int nb) {
  return dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb);
}

}  // namespace

template <typename T>
void poisson_dense_build(T* aug, int N, double d, double c, hipStream_t s) {
  const int64_t n = (int64_t)N * N;
  hipLaunchKernelGGL(k_dense_build<T>, dim3((unsigned)((n + 255) / 256), (unsigned)n),
                     dim3(256), 0, s, aug, N, (R_t<T>)d, (R_t<T>)c);
}

template <typename T>
void poisson_apply(const T* x, T* y, int N, double d, double c, int nb, const int* active,
                   c64* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_apply<T>, grid_pts((int64_t)N * N, nb), dim3(kThreads), 0, s, x, y,
                     N, (R_t<T>)d, (R_t<T>)c, active, partials);
}

template <typename Tb, typename Tx, typename Tr>
void poisson_residual(const Tb* b, const Tx* x, Tr* r, int N, double d, double c, int nb,
                      const int* active, c64* partials, hipStream_t s) {
  hipLaunchKernelGGL((k_residual<Tb, Tx, Tr>), grid_pts((int64_t)N * N, nb), dim3(kThreads),
                     0, s, b, x, r, N, (R_t<Tx>)d, (R_t<Tx>)c, active, partials);
}

template <typename T>
void poisson_rbgs(const T* b, T* x, int N, double d, double c, int nb, const int* active,
                  bool zero_init, bool reverse, hipStream_t s) {
  const dim3 g = grid_pts((int64_t)N * N, nb);
  const int first = reverse ? 1 : 0;
  hipLaunchKernelGGL(k_gs_colour<T>, g, dim3(kThreads), 0, s, b, x, N, (R_t<T>)(1.0 / d),
                     (R_t<T>)c, first, zero_init ? 1 : 0, active);
  hipLaunchKernelGGL(k_gs_colour<T>, g, dim3(kThreads), 0, s, b, x, N, (R_t<T>)(1.0 / d),
                     (R_t<T>)c, 1 - first, 0, active);
}

template <typename T>
void poisson_residual_restrict(const T* b, const T* x, T* rc, int N, double d, double c,
                               int nb, const int* active, hipStream_t s) {
  const int64_t nc = (int64_t)(N / 2) * (N / 2);
  hipLaunchKernelGGL(k_res_restrict<T>, grid_pts(nc, nb), dim3(kThreads), 0, s, b, x, rc, N,
                     (R_t<T>)d, (R_t<T>)c, active);
}

template <typename T>
void agg2d_restrict(const T* x, T* xc, int N, int nb, const int* active, hipStream_t s) {
  const int64_t nc = (int64_t)(N / 2) * (N / 2);
  hipLaunchKernelGGL(k_restrict<T>, grid_pts(nc, nb), dim3(kThreads), 0, s, x, xc, N, active);
}

template <typename T>
void agg2d_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                   const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_prolong<T>, grid_pts((int64_t)N * N, nb), dim3(kThreads), 0, s, ec, x,
                     N, (R_t<T>)(0.5 * omega), (R_t<T>)beta, active);
}

#define MLMC_INST_P(T)                                                                     \
  template void poisson_dense_build<T>(T*, int, double, double, hipStream_t);             \
  template void poisson_apply<T>(const T*, T*, int, double, double, int, const int*, c64*, \
                                 hipStream_t);                                            \
  template void poisson_rbgs<T>(const T*, T*, int, double, double, int, const int*, bool, \
                                bool, hipStream_t);                                       \
  template void poisson_residual_restrict<T>(const T*, const T*, T*, int, double, double, \
                                             int, const int*, hipStream_t);               \
  template void agg2d_restrict<T>(const T*, T*, int, int, const int*, hipStream_t);       \
  template void agg2d_prolong<T>(const T*, T*, int, double, double, int, const int*,      \
                                 hipStream_t);

MLMC_INST_P(float)
MLMC_INST_P(double)

template void poisson_residual<double, double, double>(const double*, const double*, double*,
                                                       int, double, double, int, const int*,
                                                       c64*, hipStream_t);
template void poisson_residual<double, double, float>(const double*, const double*, float*,
                                                      int, double, double, int, const int*,
                                                      c64*, hipStream_t);
template void poisson_residual<float, float, float>(const float*, const float*, float*, int,
                                                    double, double, int, const int*, c64*,
                                                    hipStream_t);

}  // namespace mlmc
