// 3D 7-point variable-coefficient diffusion operator with Dirichlet faces:
//   A = sum_interior faces k_f (e_i - e_j)(e_i - e_j)^T
//     + sum_boundary faces k_f e_i e_i^T + shift I,
// cell i = (z*N + y)*N + x.  Face arrays (one level): k[d][a][b][f], d = 0 x-faces
// ([z][y][f]), 1 y-faces ([z][x][f]), 2 z-faces ([y][x][f]); face f lies between
// cells f-1 and f along d (f = 0 and f = N are boundary faces).  diag[i] = shift +
// the six faces of cell i.  With 2x2x2 orthonormal aggregation (entries
// 1/sqrt(8)) the Galerkin operator is again of this form: a coarse face is 1/8
// of the sum of the four fine faces it covers and the shift is kept.
#include "kernels.h"

namespace mlmc {
namespace {

template <typename T> using R_t = typename Traits<T>::real;

struct Cell {
  int x, y, z;
};

__device__ __forceinline__ Cell cell_of(int i, int N) {
  Cell c;
  c.z = i / (N * N);
  const int r = i - c.z * N * N;
  c.y = r / N;
  c.x = r - c.y * N;
  return c;
}

__device__ __forceinline__ int64_t face_idx(int d, int a, int b, int f, int N) {
  return (((int64_t)d * N + a) * N + b) * (N + 1) + f;
}

// sum over the six neighbours j of k_ij * u_j (interior faces only)
template <typename T, typename K>
__device__ __forceinline__ T nbr_sum(const T* u, const K* k, int N, Cell c, int i) {
  T s = zero_of(T());
  const int NN = N * N;
  if (c.x > 0) s += (R_t<T>)k[face_idx(0, c.z, c.y, c.x, N)] * u[i - 1];
  if (c.x + 1 < N) s += (R_t<T>)k[face_idx(0, c.z, c.y, c.x + 1, N)] * u[i + 1];
  if (c.y > 0) s += (R_t<T>)k[face_idx(1, c.z, c.x, c.y, N)] * u[i - N];
  if (c.y + 1 < N) s += (R_t<T>)k[face_idx(1, c.z, c.x, c.y + 1, N)] * u[i + N];
  if (c.z > 0) s += (R_t<T>)k[face_idx(2, c.y, c.x, c.z, N)] * u[i - NN];
  if (c.z + 1 < N) s += (R_t<T>)k[face_idx(2, c.y, c.x, c.z + 1, N)] * u[i + NN];
  return s;
}

template <typename Tb, typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_vc_residual(const Tb* __restrict__ b,
                                                          const T* __restrict__ x,
                                                          Tr* __restrict__ r,
                                                          const R_t<T>* __restrict__ k,
                                                          const R_t<T>* __restrict__ diag, int N,
                                                          const int* active, c64* partials,
                                                          int* tlog) {
  __shared__ double red[16];
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int n = N * N * N;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const int64_t off = (int64_t)col * n;
  double dre = 0.0, dim = 0.0;
  if (i < n) {
    const Cell c = cell_of(i, N);
    const T* xc = x + off;
    T v = diag[i] * xc[i] - nbr_sum(xc, k, N, c, i);
    if (b) {
      v = convert<T, Tb>(b[off + i]) - v;
      cdot_acc(dre, dim, v, v);
    } else {
      cdot_acc(dre, dim, xc[i], v);
    }
    r[off + i] = convert<Tr, T>(v);
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)col * gridDim.x + blockIdx.x] = {dre, dim};
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vc_gs(const T* __restrict__ b, T* __restrict__ x,
                                                    const R_t<T>* __restrict__ k,
                                                    const R_t<T>* __restrict__ diag, int N,
                                                    int colour, int zero_nbrs, const int* active,
                                                    int* tlog) {
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int n = N * N * N;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const Cell c = cell_of(i, N);
  if (((c.x + c.y + c.z) & 1) != colour) return;
  const int64_t off = (int64_t)col * n;
  T v = b[off + i];
  if (!zero_nbrs) v += nbr_sum(x + off, k, N, c, i);
  x[off + i] = ((R_t<T>)1 / diag[i]) * v;
}

// rc = R (b - A x), or rc = R x when b == nullptr and res == false
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vc_restrict(const T* __restrict__ b,
                                                          const T* __restrict__ x,
                                                          T* __restrict__ rc,
                                                          const R_t<T>* __restrict__ k,
                                                          const R_t<T>* __restrict__ diag, int N,
                                                          int residual, const int* active,
                                                          int* tlog) {
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int Nc = N / 2, nc = Nc * Nc * Nc, n = N * N * N;
  const int I = blockIdx.x * kThreads + threadIdx.x;
  if (I >= nc) return;
  const Cell C = cell_of(I, Nc);
  const int64_t off = (int64_t)col * n;
  const T* xc = x + off;
  T acc = zero_of(T());
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        Cell c = {2 * C.x + dx, 2 * C.y + dy, 2 * C.z + dz};
        const int i = (c.z * N + c.y) * N + c.x;
        if (residual)
          acc += b[off + i] - (diag[i] * xc[i] - nbr_sum(xc, k, N, c, i));
        else
          acc += xc[i];
      }
  rc[(int64_t)col * nc + I] = (R_t<T>)0.35355339059327373 * acc;  // 1/sqrt(8)
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vc_prolong(const T* __restrict__ ec, T* __restrict__ x,
                                                         int N, R_t<T> wscaled, R_t<T> beta,
                                                         const int* active) {
  const int col = blockIdx.y;
  if (active && !active[col]) return;
  const int Nc = N / 2, n = N * N * N;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const Cell c = cell_of(i, N);
  const T e = ec[(int64_t)col * Nc * Nc * Nc + ((c.z >> 1) * Nc + (c.y >> 1)) * Nc + (c.x >> 1)];
  T* xk = x + (int64_t)col * n;
  xk[i] = (beta == (R_t<T>)0) ? wscaled * e : beta * xk[i] + wscaled * e;
}

// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q.  The
// neighbours' p_new values are recomputed from z and p_old, so the update and
// the operator need a single pass.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vc_update_apply(
    const T* __restrict__ p_old, const T* __restrict__ z, const c64* __restrict__ beta,
    T* __restrict__ p_new, T* __restrict__ q, const R_t<T>* __restrict__ k,
    const R_t<T>* __restrict__ diag, int N, const int* active, c64* partials, int* tlog) {
  __shared__ double red[16];
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int n = N * N * N;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  const int64_t off = (int64_t)col * n;
  const R_t<T> bt = (R_t<T>)beta[col].re;
  const T* zc = z + off;
  const T* pc = p_old + off;
  double dre = 0.0, dim = 0.0;
  if (i < n) {
    const Cell c = cell_of(i, N);
    const int NN = N * N;
    auto P = [&](int j) { return zc[j] + bt * pc[j]; };
    const T pi = P(i);
    T s = zero_of(T());
    if (c.x > 0) s += (R_t<T>)k[face_idx(0, c.z, c.y, c.x, N)] * P(i - 1);
    if (c.x + 1 < N) s += (R_t<T>)k[face_idx(0, c.z, c.y, c.x + 1, N)] * P(i + 1);
    if (c.y > 0) s += (R_t<T>)k[face_idx(1, c.z, c.x, c.y, N)] * P(i - N);
    if (c.y + 1 < N) s += (R_t<T>)k[face_idx(1, c.z, c.x, c.y + 1, N)] * P(i + N);
    if (c.z > 0) s += (R_t<T>)k[face_idx(2, c.y, c.x, c.z, N)] * P(i - NN);
    if (c.z + 1 < N) s += (R_t<T>)k[face_idx(2, c.y, c.x, c.z + 1, N)] * P(i + NN);
    const T qv = diag[i] * pi - s;
    p_new[off + i] = pi;
    q[off + i] = qv;
    cdot_acc(dre, dim, pi, qv);
  }
  block_sum2<kThreads>(dre, dim, red);
  if (threadIdx.x == 0) partials[(int64_t)col * gridDim.x + blockIdx.x] = {dre, dim};
}

__global__ void k_vc_coarsen(const double* __restrict__ kf, double* __restrict__ kc, int N) {
  const int Nc = N / 2;
  const int64_t total = 3LL * Nc * Nc * (Nc + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(t % (Nc + 1));
    const int64_t r = t / (Nc + 1);
    const int bb = (int)(r % Nc), a = (int)((r / Nc) % Nc), d = (int)(r / ((int64_t)Nc * Nc));
    double s = 0.0;
    for (int u = 0; u < 2; ++u)
      for (int v = 0; v < 2; ++v) s += kf[face_idx(d, 2 * a + u, 2 * bb + v, 2 * f, N)];
    kc[t] = 0.125 * s;
  }
}

__global__ void k_vc_diag(const double* __restrict__ k, double shift, int N, double* d64,
                          float* d32, float* k32) {
  const int n = N * N * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const Cell c = cell_of(i, N);
    const double s = shift + k[face_idx(0, c.z, c.y, c.x, N)] + k[face_idx(0, c.z, c.y, c.x + 1, N)] +
                     k[face_idx(1, c.z, c.x, c.y, N)] + k[face_idx(1, c.z, c.x, c.y + 1, N)] +
                     k[face_idx(2, c.y, c.x, c.z, N)] + k[face_idx(2, c.y, c.x, c.z + 1, N)];
    d64[i] = s;
    d32[i] = (float)s;
  }
  const int64_t nf = 3LL * N * N * (N + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nf;
       t += (int64_t)gridDim.x * blockDim.x)
    k32[t] = (float)k[t];
}

__global__ void k_vc_dense(const double* __restrict__ k, const double* __restrict__ diag, int N,
                           double* __restrict__ M) {
  const int n = N * N * N;
  const int64_t ld = 2LL * n;
  const int i = blockIdx.x;
  double* row = M + (int64_t)i * ld;
  for (int j = threadIdx.x; j < n; j += blockDim.x) row[j] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const Cell c = cell_of(i, N);
    const int NN = N * N;
    row[i] = diag[i];
    if (c.x > 0) row[i - 1] = -k[face_idx(0, c.z, c.y, c.x, N)];
    if (c.x + 1 < N) row[i + 1] = -k[face_idx(0, c.z, c.y, c.x + 1, N)];
    if (c.y > 0) row[i - N] = -k[face_idx(1, c.z, c.x, c.y, N)];
    if (c.y + 1 < N) row[i + N] = -k[face_idx(1, c.z, c.x, c.y + 1, N)];
    if (c.z > 0) row[i - NN] = -k[face_idx(2, c.y, c.x, c.z, N)];
    if (c.z + 1 < N) row[i + NN] = -k[face_idx(2, c.y, c.x, c.z + 1, N)];
  }
}

inline dim3 grid_cells(int64_t n, int nb) {
  return dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb);
}

}  // namespace

int varcoef_blocks(int N) { return (N * N * N + kThreads - 1) / kThreads; }

template <typename Tb, typename T, typename Tr>
void varcoef_residual(const Tb* b, const T* x, Tr* r, const typename Traits<T>::real* k,
                      const typename Traits<T>::real* diag, int N, int nb, const int* active,
                      c64* partials, hipStream_t s) {
  MLMC_LAUNCH((k_vc_residual<Tb, T, Tr>), grid_cells((int64_t)N * N * N, nb),
                     dim3(kThreads), 0, s, b, x, r, k, diag, N, active, partials, timing_log());
}

template <typename T>
void varcoef_rbgs(const T* b, T* x, const typename Traits<T>::real* k,
                  const typename Traits<T>::real* diag, int N, int nb, const int* active,
                  bool zero_init, bool reverse, hipStream_t s) {
  const dim3 g = grid_cells((int64_t)N * N * N, nb);
  const int first = reverse ? 1 : 0;
  MLMC_LAUNCH(k_vc_gs<T>, g, dim3(kThreads), 0, s, b, x, k, diag, N, first,
                     zero_init ? 1 : 0, active, timing_log());
  MLMC_LAUNCH(k_vc_gs<T>, g, dim3(kThreads), 0, s, b, x, k, diag, N, 1 - first, 0,
                     active, (int*)nullptr);
}

template <typename T>
void varcoef_restrict(const T* b, const T* x, T* xc, const typename Traits<T>::real* k,
                      const typename Traits<T>::real* diag, int N, bool residual, int nb,
                      const int* active, hipStream_t s) {
  const int Nc = N / 2;
  MLMC_LAUNCH(k_vc_restrict<T>, grid_cells((int64_t)Nc * Nc * Nc, nb), dim3(kThreads), 0,
                     s, b, x, xc, k, diag, N, residual ? 1 : 0, active, timing_log());
}

template <typename T>
void varcoef_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                     const int* active, hipStream_t s) {
  MLMC_LAUNCH(k_vc_prolong<T>, grid_cells((int64_t)N * N * N, nb), dim3(kThreads), 0, s,
                     ec, x, N, (typename Traits<T>::real)(omega * 0.35355339059327373),
                     (typename Traits<T>::real)beta, active);
}

template <typename T>
void varcoef_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                          const typename Traits<T>::real* k,
                          const typename Traits<T>::real* diag, int N, int nb, const int* active,
                          c64* partials, hipStream_t s) {
  MLMC_LAUNCH(k_vc_update_apply<T>, grid_cells((int64_t)N * N * N, nb), dim3(kThreads), 0,
                     s, p_old, z, beta, p_new, q, k, diag, N, active, partials, timing_log());
}

void varcoef_coarsen(const double* kf, double* kc, int N, hipStream_t s) {
  MLMC_LAUNCH(k_vc_coarsen, dim3(256), dim3(256), 0, s, kf, kc, N);
}

void varcoef_diag(const double* k, double shift, int N, double* d64, float* d32, float* k32,
                  hipStream_t s) {
  MLMC_LAUNCH(k_vc_diag, dim3(256), dim3(256), 0, s, k, shift, N, d64, d32, k32);
}

void varcoef_dense(const double* k, const double* diag, int N, double* aug, hipStream_t s) {
  MLMC_LAUNCH(k_vc_dense, dim3(N * N * N), dim3(256), 0, s, k, diag, N, aug);
}

template void varcoef_residual<double, double, double>(const double*, const double*, double*,
                                                       const double*, const double*, int, int,
                                                       const int*, c64*, hipStream_t);
template void varcoef_residual<double, double, float>(const double*, const double*, float*,
                                                      const double*, const double*, int, int,
                                                      const int*, c64*, hipStream_t);
template void varcoef_residual<float, float, float>(const float*, const float*, float*,
                                                    const float*, const float*, int, int,
                                                    const int*, c64*, hipStream_t);
template void varcoef_rbgs<float>(const float*, float*, const float*, const float*, int, int,
                                  const int*, bool, bool, hipStream_t);
template void varcoef_rbgs<double>(const double*, double*, const double*, const double*, int,
                                   int, const int*, bool, bool, hipStream_t);
template void varcoef_restrict<float>(const float*, const float*, float*, const float*,
                                      const float*, int, bool, int, const int*, hipStream_t);
template void varcoef_restrict<double>(const double*, const double*, double*, const double*,
                                       const double*, int, bool, int, const int*, hipStream_t);
template void varcoef_update_apply<float>(const float*, const float*, const c64*, float*,
                                          float*, const float*, const float*, int, int,
                                          const int*, c64*, hipStream_t);
template void varcoef_update_apply<double>(const double*, const double*, const c64*, double*,
                                           double*, const double*, const double*, int, int,
                                           const int*, c64*, hipStream_t);
template void varcoef_prolong<float>(const float*, float*, int, double, double, int, const int*,
                                     hipStream_t);
template void varcoef_prolong<double>(const double*, double*, int, double, double, int,
                                      const int*, hipStream_t);

}  // namespace mlmc
