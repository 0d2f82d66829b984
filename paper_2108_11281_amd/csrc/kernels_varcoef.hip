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
#include "lanes.h"

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

// Stencil kernels read the level's couplings in a cell-major layout:
// kl[d][i] = coefficient of the face below cell i in direction d (x, y, z),
// zero on the boundary, each of the three arrays padded with N^2 zeros, so that
// the six couplings of cell i are kl[0][i], kl[0][i+1], kl[1][i], kl[1][i+N],
// kl[2][i], kl[2][i+N^2] -- coalesced and branch-free.  Neighbour loads use
// clamped indices (their coupling is zero wherever the clamp acts).  A thread
// serves COLS right-hand sides, so the couplings are loaded once per COLS
// columns.
template <typename R>
struct Couplings {
  R cx0, cx1, cy0, cy1, cz0, cz1, d;
  int64_t im1, ip1, imN, ipN, imNN, ipNN;
};

template <typename R>
__device__ __forceinline__ Couplings<R> couplings(const R* __restrict__ kl,
                                                  const R* __restrict__ dg, int64_t i, int N) {
  const int64_t n = (int64_t)N * N * N, NN = (int64_t)N * N, stride = n + NN;
  Couplings<R> c;
  c.cx0 = kl[i];
  c.cx1 = kl[i + 1];
  c.cy0 = kl[stride + i];
  c.cy1 = kl[stride + i + N];
  c.cz0 = kl[2 * stride + i];
  c.cz1 = kl[2 * stride + i + NN];
  c.d = dg[i];
  c.im1 = i > 0 ? i - 1 : 0;
  c.ip1 = i + 1 < n ? i + 1 : n - 1;
  c.imN = i >= N ? i - N : 0;
  c.ipN = i + N < n ? i + N : n - 1;
  c.imNN = i >= NN ? i - NN : 0;
  c.ipNN = i + NN < n ? i + NN : n - 1;
  return c;
}

// coupling times neighbour value, selected (not multiplied) to zero where the
// coupling is zero: a clamped index may point at a cell that the current sweep
// has not written yet, whose stale contents need not be finite
template <typename T, typename R>
__device__ __forceinline__ T term(R cf, T v) {
  return cf != (R)0 ? cf * v : zero_of(T());
}

// sum of the six couplings times the neighbours of u (one column)
template <typename T, typename R>
__device__ __forceinline__ T nbr_sum(const T* __restrict__ u, const Couplings<R>& c) {
  return term(c.cx0, u[c.im1]) + term(c.cx1, u[c.ip1]) + term(c.cy0, u[c.imN]) +
         term(c.cy1, u[c.ipN]) + term(c.cz0, u[c.imNN]) + term(c.cz1, u[c.ipNN]);
}

__device__ __forceinline__ bool col_on(const int* active, int col, int nb) {
  return col < nb && (!active || active[col]);
}

// r = b - A x (or r = A x when b is null); partials: per column and block of
// |r|^2 (or conj(x)^T r)
template <typename Tb, typename T, typename Tr, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_residual(const Tb* __restrict__ b,
                                                          const T* __restrict__ x,
                                                          Tr* __restrict__ r,
                                                          const R_t<T>* __restrict__ kl,
                                                          const R_t<T>* __restrict__ dg, int N,
                                                          int nb, const int* active,
                                                          c64* partials, int* tlog) {
  __shared__ double red[16];
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int64_t n = (int64_t)N * N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool in = i < n;
  Couplings<R_t<T>> c = couplings(kl, dg, in ? i : 0, N);
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    const int col = col0 + q;
    if (!col_on(active, col, nb)) continue;  // uniform over the block
    const int64_t off = (int64_t)col * n;
    double dre = 0.0, dim = 0.0;
    if (in) {
      const T* xc = x + off;
      T v = c.d * xc[i] - nbr_sum(xc, c);
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
}

// one colour of a red-black Gauss-Seidel sweep, in place; a thread per cell of
// that colour (cell x = 2j + ((colour + y + z) & 1) of row (y, z)).  With ec
// (first colour after the coarse solve), the neighbours are read as
// x + wscaled * ec(aggregate): the prolongation and correction of the other
// colour's cells folded into the sweep (this colour's own cells are
// overwritten, so their correction is never needed).
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_gs(const T* __restrict__ b, T* __restrict__ x,
                                                    const R_t<T>* __restrict__ kl,
                                                    const R_t<T>* __restrict__ dg, int N,
                                                    int colour, int zero_nbrs, int nb,
                                                    const int* active, const T* __restrict__ ec,
                                                    R_t<T> wscaled, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int half = N >> 1;
  const int64_t n = (int64_t)N * N * N;
  // 32-bit index arithmetic (N^3 < 2^31 for every supported side)
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= (int)(n / 2)) return;
  const int row = t / half;
  const int j = t - row * half;
  const int z = row / N, y = row - z * N;
  const int xx = 2 * j + ((colour + y + z) & 1);
  const int64_t i = (int64_t)row * N + xx;
  Couplings<R_t<T>> c = couplings(kl, dg, i, N);
  const R_t<T> inv_d = (R_t<T>)1 / c.d;
  // aggregates of the six neighbours (coordinates clamped; their coupling is
  // zero wherever the clamp acts)
  const int Nc = N >> 1;
  auto agg = [&](int ax, int ay, int az) { return ((az >> 1) * Nc + (ay >> 1)) * Nc + (ax >> 1); };
  int ga[6] = {0, 0, 0, 0, 0, 0};
  if (ec) {
    ga[0] = agg(xx > 0 ? xx - 1 : 0, y, z);
    ga[1] = agg(xx + 1 < N ? xx + 1 : N - 1, y, z);
    ga[2] = agg(xx, y > 0 ? y - 1 : 0, z);
    ga[3] = agg(xx, y + 1 < N ? y + 1 : N - 1, z);
    ga[4] = agg(xx, y, z > 0 ? z - 1 : 0);
    ga[5] = agg(xx, y, z + 1 < N ? z + 1 : N - 1);
  }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    const int col = col0 + q;
    if (!col_on(active, col, nb)) continue;
    const int64_t off = (int64_t)col * n;
    T v = b[off + i];
    if (ec) {
      const T* u = x + off;
      const T* e = ec + (int64_t)col * Nc * Nc * Nc;
      v += term(c.cx0, u[c.im1] + wscaled * e[ga[0]]) + term(c.cx1, u[c.ip1] + wscaled * e[ga[1]]) +
           term(c.cy0, u[c.imN] + wscaled * e[ga[2]]) + term(c.cy1, u[c.ipN] + wscaled * e[ga[3]]) +
           term(c.cz0, u[c.imNN] + wscaled * e[ga[4]]) +
           term(c.cz1, u[c.ipNN] + wscaled * e[ga[5]]);
    } else if (!zero_nbrs) {
      v += nbr_sum(x + off, c);
    }
    x[off + i] = inv_d * v;
  }
}

// rc = R (b - A x) when residual, else rc = R x (2x2x2 aggregates, 1/sqrt(8))
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_restrict(const T* __restrict__ b,
                                                          const T* __restrict__ x,
                                                          T* __restrict__ rc,
                                                          const R_t<T>* __restrict__ kl,
                                                          const R_t<T>* __restrict__ dg, int N,
                                                          int residual, int nb,
                                                          const int* active, int* tlog) {
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int Nc = N / 2;
  const int64_t nc = (int64_t)Nc * Nc * Nc, n = (int64_t)N * N * N;
  const int I = blockIdx.x * kThreads + threadIdx.x;
  if (I >= (int)nc) return;
  const int Z = I / (Nc * Nc);
  const int rem = I - Z * Nc * Nc;
  const int Y = rem / Nc, X = rem - Y * Nc;
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) acc[q] = zero_of(T());
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int64_t i = ((int64_t)(2 * Z + dz) * N + (2 * Y + dy)) * N + (2 * X + dx);
        if (residual) {
          Couplings<R_t<T>> c = couplings(kl, dg, i, N);
#pragma unroll
          for (int q = 0; q < COLS; ++q) {
            const int col = col0 + q;
            if (!col_on(active, col, nb)) continue;
            const int64_t off = (int64_t)col * n;
            const T* xc = x + off;
            acc[q] += b[off + i] - (c.d * xc[i] - nbr_sum(xc, c));
          }
        } else {
#pragma unroll
          for (int q = 0; q < COLS; ++q) {
            const int col = col0 + q;
            if (!col_on(active, col, nb)) continue;
            acc[q] += x[(int64_t)col * n + i];
          }
        }
      }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    const int col = col0 + q;
    if (!col_on(active, col, nb)) continue;
    rc[(int64_t)col * nc + I] = (R_t<T>)0.35355339059327373 * acc[q];  // 1/sqrt(8)
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_vc_prolong(const T* __restrict__ ec, T* __restrict__ x,
                                                         int N, R_t<T> wscaled, R_t<T> beta,
                                                         const int* active, int* tlog) {
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const int Nc = N / 2;
  const int64_t n = (int64_t)N * N * N;
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= (int)n) return;
  const int z = i / (N * N);
  const int rem = i - z * N * N;
  const int y = rem / N, xx = rem - y * N;
  const T e = ec[(int64_t)col * Nc * Nc * Nc + ((z >> 1) * Nc + (y >> 1)) * Nc + (xx >> 1)];
  T* xk = x + (int64_t)col * n;
  xk[i] = (beta == (R_t<T>)0) ? wscaled * e : beta * xk[i] + wscaled * e;
}

// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q.  The
// neighbours' p_new values are recomputed from z and p_old, so the update and
// the operator need a single pass.
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_update_apply(
    const T* __restrict__ p_old, const T* __restrict__ z, const c64* __restrict__ beta,
    T* __restrict__ p_new, T* __restrict__ q, const R_t<T>* __restrict__ kl,
    const R_t<T>* __restrict__ dg, int N, int nb, const int* active, c64* partials, int* tlog) {
  __shared__ double red[16];
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int64_t n = (int64_t)N * N * N;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const bool in = i < n;
  Couplings<R_t<T>> c = couplings(kl, dg, in ? i : 0, N);
#pragma unroll
  for (int qq = 0; qq < COLS; ++qq) {
    const int col = col0 + qq;
    if (!col_on(active, col, nb)) continue;
    const int64_t off = (int64_t)col * n;
    const R_t<T> bt = (R_t<T>)beta[col].re;
    const T* zc = z + off;
    const T* pc = p_old + off;
    double dre = 0.0, dim = 0.0;
    if (in) {
      auto P = [&](int64_t j) { return zc[j] + bt * pc[j]; };
      const T pi = P(i);
      const T s = term(c.cx0, P(c.im1)) + term(c.cx1, P(c.ip1)) + term(c.cy0, P(c.imN)) +
                  term(c.cy1, P(c.ipN)) + term(c.cz0, P(c.imNN)) + term(c.cz1, P(c.ipNN));
      const T qv = c.d * pi - s;
      p_new[off + i] = pi;
      q[off + i] = qv;
      cdot_acc(dre, dim, pi, qv);
    }
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)col * gridDim.x + blockIdx.x] = {dre, dim};
  }
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

// diagonal (shift + the six faces of each cell) and the cell-major couplings
// kl[d][i] (boundary zero, each array padded with N^2 zeros), FP64 and FP32
__global__ void k_vc_diag(const double* __restrict__ k, double shift, int N, double* d64,
                          float* d32, double* kl64, float* kl32) {
  const int n = N * N * N, NN = N * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const Cell c = cell_of(i, N);
    const double s = shift + k[face_idx(0, c.z, c.y, c.x, N)] + k[face_idx(0, c.z, c.y, c.x + 1, N)] +
                     k[face_idx(1, c.z, c.x, c.y, N)] + k[face_idx(1, c.z, c.x, c.y + 1, N)] +
                     k[face_idx(2, c.y, c.x, c.z, N)] + k[face_idx(2, c.y, c.x, c.z + 1, N)];
    d64[i] = s;
    d32[i] = (float)s;
  }
  const int64_t stride = (int64_t)n + NN;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < 3 * stride;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(t / stride);
    const int64_t i = t - d * stride;
    double v = 0.0;
    if (i < n) {
      const Cell c = cell_of((int)i, N);
      if (d == 0 && c.x > 0) v = k[face_idx(0, c.z, c.y, c.x, N)];
      if (d == 1 && c.y > 0) v = k[face_idx(1, c.z, c.x, c.y, N)];
      if (d == 2 && c.z > 0) v = k[face_idx(2, c.y, c.x, c.z, N)];
    }
    kl64[t] = v;
    kl32[t] = (float)v;
  }
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

// rc = R (b - A x) (2x2x2 aggregates, 1/sqrt(8)), the aggregate read as four
// rows of two cells: a thread per coarse cell (lanes along coarse x, so each
// row is a 2-element load contiguous over the wave), COLS right-hand sides
// sharing the couplings; neighbours outside the grid read as zero
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_res_restrict(const T* __restrict__ b,
                                                              const T* __restrict__ x,
                                                              T* __restrict__ rc,
                                                              const R_t<T>* __restrict__ kl,
                                                              const R_t<T>* __restrict__ dg,
                                                              int N, int nb, const int* active,
                                                              int* tlog) {
  using R = R_t<T>;
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int Nc = N >> 1;
  const int nc = Nc * Nc * Nc;
  const int I = blockIdx.x * kThreads + threadIdx.x;
  if (I >= nc) return;
  const int Z = I / (Nc * Nc);
  const int rem = I - Z * Nc * Nc;
  const int Y = rem / Nc, X = rem - Y * Nc;
  const int x0 = 2 * X;
  const int NN = N * N;
  const int64_t n = (int64_t)NN * N, stride = n + NN;
  const T zero = zero_of(T());
  T acc[COLS];
#pragma unroll
  for (int q = 0; q < COLS; ++q) acc[q] = zero;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int y = 2 * Y + dy, z = 2 * Z + dz;
      const int64_t i = ((int64_t)z * N + y) * N + x0;
      // couplings of the pair (faces below each cell and the ones above, which
      // are the faces below the next cells; zero on the boundary, padded)
      const R kx0 = kl[i], kx1 = kl[i + 1], kx2 = kl[i + 2];
      const R ky0 = kl[stride + i], ky1 = kl[stride + i + 1];
      const R kyu0 = kl[stride + i + N], kyu1 = kl[stride + i + N + 1];
      const R kz0 = kl[2 * stride + i], kz1 = kl[2 * stride + i + 1];
      const R kzu0 = kl[2 * stride + i + NN], kzu1 = kl[2 * stride + i + NN + 1];
      const R d0 = dg[i], d1 = dg[i + 1];
      const bool xl_in = x0 > 0, xr_in = x0 + 2 < N;
      const bool yl_in = y > 0, yu_in = y + 1 < N, zl_in = z > 0, zu_in = z + 1 < N;
#pragma unroll
      for (int q = 0; q < COLS; ++q) {
        const int col = col0 + q;
        if (!col_on(active, col, nb)) continue;  // uniform over the block
        const T* xc = x + (int64_t)col * n;
        const T* bc = b + (int64_t)col * n;
        const T c0 = xc[i], c1 = xc[i + 1];
        const T xl = xl_in ? xc[i - 1] : zero, xr = xr_in ? xc[i + 2] : zero;
        const T yl0 = yl_in ? xc[i - N] : zero, yl1 = yl_in ? xc[i - N + 1] : zero;
        const T yu0 = yu_in ? xc[i + N] : zero, yu1 = yu_in ? xc[i + N + 1] : zero;
        const T zl0 = zl_in ? xc[i - NN] : zero, zl1 = zl_in ? xc[i - NN + 1] : zero;
        const T zu0 = zu_in ? xc[i + NN] : zero, zu1 = zu_in ? xc[i + NN + 1] : zero;
        const T r0 = bc[i] - (d0 * c0 - (kx0 * xl + kx1 * c1 + ky0 * yl0 + kyu0 * yu0 +
                                          kz0 * zl0 + kzu0 * zu0));
        const T r1 = bc[i + 1] - (d1 * c1 - (kx1 * c0 + kx2 * xr + ky1 * yl1 + kyu1 * yu1 +
                                              kz1 * zl1 + kzu1 * zu1));
        acc[q] += r0;
        acc[q] += r1;
      }
    }
#pragma unroll
  for (int q = 0; q < COLS; ++q) {
    const int col = col0 + q;
    if (!col_on(active, col, nb)) continue;
    rc[(int64_t)col * nc + I] = (R)0.35355339059327373 * acc[q];  // 1/sqrt(8)
  }
}

// ---------------------------------------------------------------------------
// One fused red-black sweep, out of place, marching along z:
//   x_out = S(x_in + ws * P ec ; b)      (ws = omega / sqrt(8); F = first colour)
// A workgroup of 8 waves owns TY = 8 RPW - 2 consecutive rows y0 .. y0+TY-1
// of COLS right-hand sides and walks a segment of SZ planes.  It holds the
// rows y0-1 .. y0+TY as lane pairs (x = 2*pl, 2*pl+1), RPW rows per wave of
// 64/RPW lanes each (2*64/RPW >= N, so a row needs no x halo; a wave's rows
// have one parity), with five planes of each row in registers.  At step p a
// wave loads plane p+2, updates the first colour on plane p and the second
// colour on plane p-1, and writes plane p-1 (owned rows).  In a row both
// updates of a step hit the same element of the pair, and the y-neighbours each
// needs are one value per lane of the rows above and below: the rows swap them
// through LDS (double-buffered, one barrier per step); the two outermost rows
// also load the row beyond them.  Cells outside the grid read as zero, so no
// coupling ever multiplies a value that was not written.
// ---------------------------------------------------------------------------
// couplings of a row pair on one plane; d0, d1 hold 1 / diagonal
template <typename R>
struct PlaneK {
  R kx0, kx1, kyl0, kyl1, kyu0, kyu1, kz0, kz1, d0, d1;
};

constexpr int kMarchWaves = 8;

template <typename T, int COLS, int RPW, bool HX, bool HE, int F>
__global__ __launch_bounds__(kMarchWaves * 64) void k_vc_march(
    const T* __restrict__ xin, const T* __restrict__ b, T* __restrict__ xout,
    const T* __restrict__ ec, R_t<T> ws, const R_t<T>* __restrict__ kl,
    const R_t<T>* __restrict__ dg, int N, int SZ, int nb, const int* active, int* tlog) {
  using R = R_t<T>;
  constexpr int RW = kMarchWaves * RPW;  // rows held, incl. one halo row each side
  constexpr int TY = RW - 2;             // rows owned
  constexpr int LPR = 64 / RPW;          // lanes (pairs) per row
  __shared__ T xa[2][RW][COLS][LPR];  // a row's second-colour cell at plane p (x_in)
  __shared__ T xb[2][RW][COLS][LPR];  // a row's first-colour cell at plane p-1 (updated)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int col0 = blockIdx.y * COLS;
  if (tlog && blockIdx.x == 0 && blockIdx.z == 0 && threadIdx.x < COLS &&
      col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  bool con[COLS];
  bool any = false;
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    con[c] = col_on(active, col0 + c, nb);
    any = any || con[c];
  }
  if (!any) return;  // uniform over the workgroup
  const int seg = lane / LPR, pl = lane - seg * LPR;
  // row slot: wave w holds slots of parity w & 1 (so e below is wave-uniform)
  const int r = (w & 1) + 2 * (seg + RPW * (w >> 1));
  const int y = blockIdx.x * TY - 1 + r;
  // a row of the wave's parity (uniform; y has this parity in every lane)
  const int ybase = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * TY - 1 + (w & 1)));
  const int x0 = 2 * pl;
  const bool xok = x0 < N;
  const bool row_in = y >= 0 && y < N;
  const bool cell_ok = row_in && xok;
  const bool edge = (r == 0) || (r == RW - 1);
  const int ye = (r == 0) ? y - 1 : y + 1;  // the outermost rows' outer neighbour row
  const bool eok = edge && ye >= 0 && ye < N && xok;
  const bool inner = r >= 1 && r <= TY;
  const bool owner = inner && row_in;
  const int NN = N * N;
  const int64_t n = (int64_t)NN * N, stride = n + NN;
  const int Nc = N >> 1;
  const T zero = zero_of(T());

  // column base pointers (inactive columns point at column 0 and are never stored)
  const T* xc[COLS];
  const T* bc[COLS];
  const T* ecc[COLS];
  T* xo[COLS];
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    const int64_t col = con[c] ? col0 + c : 0;
    xc[c] = xin + (HX ? col * n : 0);
    bc[c] = b + col * n;
    ecc[c] = ec + (HE ? col * (int64_t)Nc * Nc * Nc : 0);
    xo[c] = xout + col * n;
  }
  auto ld2 = [&](const T* base, int64_t i, bool ok, T& v0, T& v1) {
    v0 = ok ? base[i] : zero;
    v1 = ok ? base[i + 1] : zero;
  };
  auto ldk2 = [&](const R* base, int64_t i, bool ok, R& v0, R& v1) {
    v0 = ok ? base[i] : (R)0;
    v1 = ok ? base[i + 1] : (R)0;
  };
  // x_in of row yy, plane z (with the folded correction)
  auto load_x = [&](int c, int yy, int z, bool ok, T& v0, T& v1) {
    v0 = zero;
    v1 = zero;
    const int64_t i = ((int64_t)z * N + yy) * N + x0;
    if constexpr (HX) ld2(xc[c], i, ok, v0, v1);
    if constexpr (HE) {
      const T e = ok ? ecc[c][((int64_t)(z >> 1) * Nc + (yy >> 1)) * Nc + (x0 >> 1)] : zero;
      v0 += ws * e;
      v1 += ws * e;
    }
  };
  auto load_k = [&](int z, bool ok, PlaneK<R>& k) {
    const int64_t i = ((int64_t)z * N + y) * N + x0;
    ldk2(kl, i, ok, k.kx0, k.kx1);
    ldk2(kl + stride, i, ok, k.kyl0, k.kyl1);
    ldk2(kl + stride, i + N, ok, k.kyu0, k.kyu1);
    ldk2(kl + 2 * stride, i, ok, k.kz0, k.kz1);
    ldk2(dg, i, ok, k.d0, k.d1);
    // reciprocals of the diagonal, shared by the columns (1 outside the grid)
    k.d0 = ok ? (R)1 / k.d0 : (R)1;
    k.d1 = ok ? (R)1 / k.d1 : (R)1;
  };

  // planes p+2 (m, loads in flight), p+1 (n), p (c), p-1 (p), p-2 (q) of the
  // wave's row, per column
  T Xm0[COLS], Xm1[COLS], Xn0[COLS], Xn1[COLS], Xc0[COLS], Xc1[COLS], Xp0[COLS], Xp1[COLS],
      Xq0[COLS], Xq1[COLS];
  // edge waves: outer row, planes p+2, p+1, p
  T Em0[COLS], Em1[COLS], En0[COLS], En1[COLS], Ec0[COLS], Ec1[COLS];
  T Bm0[COLS], Bm1[COLS], Bn0[COLS], Bn1[COLS], Bc0[COLS], Bc1[COLS], Bp0[COLS], Bp1[COLS];
  PlaneK<R> Km, Kn, Kc, Kp;
#pragma unroll
  for (int c = 0; c < COLS; ++c) {
    Xn0[c] = Xn1[c] = Xc0[c] = Xc1[c] = Xp0[c] = Xp1[c] = Xq0[c] = Xq1[c] = zero;
    En0[c] = En1[c] = Ec0[c] = Ec1[c] = zero;
    Bn0[c] = Bn1[c] = Bc0[c] = Bc1[c] = Bp0[c] = Bp1[c] = zero;
  }
  Kn = PlaneK<R>{};
  Kc = PlaneK<R>{};
  Kp = PlaneK<R>{};
  auto load_plane = [&](int z) {
    const bool zok = z < N;
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      load_x(c, y, z, cell_ok && zok, Xm0[c], Xm1[c]);
      if (edge) load_x(c, ye, z, eok && zok, Em0[c], Em1[c]);
      else Em0[c] = Em1[c] = zero;
      const int64_t i = ((int64_t)z * N + y) * N + x0;
      ld2(bc[c], i, cell_ok && zok, Bm0[c], Bm1[c]);
    }
    load_k(z, cell_ok && zok, Km);
  };
  auto shift = [&]() {
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      Xq0[c] = Xp0[c]; Xq1[c] = Xp1[c];
      Xp0[c] = Xc0[c]; Xp1[c] = Xc1[c];
      Xc0[c] = Xn0[c]; Xc1[c] = Xn1[c];
      Xn0[c] = Xm0[c]; Xn1[c] = Xm1[c];
      Ec0[c] = En0[c]; Ec1[c] = En1[c];
      En0[c] = Em0[c]; En1[c] = Em1[c];
      Bp0[c] = Bc0[c]; Bp1[c] = Bc1[c];
      Bc0[c] = Bn0[c]; Bc1[c] = Bn1[c];
      Bn0[c] = Bm0[c]; Bn1[c] = Bm1[c];
    }
    Kp = Kc;
    Kc = Kn;
    Kn = Km;
  };
  // this workgroup's planes zs .. ze-1 (segments of SZ): the march starts one
  // plane early (first colour only there) and reads one plane more below it
  const int zs = blockIdx.z * SZ;
  const int ze = zs + SZ < N ? zs + SZ : N;
  const int p0 = zs > 0 ? zs - 1 : 0;
  const int pe = ze < N ? ze : N;
  // prologue: planes p0-1 (zero below the grid), p0 and p0+1 into the c, n and
  // m slots, so that the first shift of the loop sees p0-1, p0, p0+1
  if (p0 >= 1) {
    load_plane(p0 - 1);
    shift();
  }
  load_plane(p0);
  shift();
  load_plane(p0 + 1);
  for (int p = p0; p <= pe; ++p) {
    // shift planes: p+1 moves into the "next" slot; plane p+2 is loaded a step
    // ahead of its first use
    shift();
    load_plane(p + 2);  // zeros beyond the last plane
    // element of the pair updated in this step (first colour on plane p,
    // second colour on plane p-1): e = (F + y + p) & 1, uniform per wave
    const int e = (F + ybase + p) & 1;
    const int buf = p & 1;
    // publish: this row's second-colour cell of plane p (x_in, element 1-e) and
    // first-colour cell of plane p-1 (updated last step, element 1-e)
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
      xa[buf][r][c][pl] = e ? Xc0[c] : Xc1[c];
      xb[buf][r][c][pl] = e ? Xp0[c] : Xp1[c];
    }
    __syncthreads();
    // first colour on plane p, element e (all rows of the workgroup)
    if (p < N) {
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const T alo = xa[buf][r > 0 ? r - 1 : 0][c][pl];
        const T ahi = xa[buf][r < RW - 1 ? r + 1 : RW - 1][c][pl];
        const T ev = e ? Ec1[c] : Ec0[c];
        const T ylo = r > 0 ? alo : ev;
        const T yhi = r < RW - 1 ? ahi : ev;
        T v;
        if (e == 0) {
          const T sh = wave_shr1(Xc1[c]);
          const T l = pl > 0 ? sh : zero;
          v = Bc0[c] + Kc.kx0 * l + Kc.kx1 * Xc1[c] + Kc.kyl0 * ylo + Kc.kyu0 * yhi +
              Kc.kz0 * Xp0[c] + Kn.kz0 * Xn0[c];
          Xc0[c] = cell_ok ? Kc.d0 * v : zero;
        } else {
          const T sh = wave_shl1(Xc0[c]);
          const R shk = wave_shl1(Kc.kx0);
          const T rr = x0 + 2 < N ? sh : zero;
          const R kr = x0 + 2 < N ? shk : (R)0;
          v = Bc1[c] + Kc.kx1 * Xc0[c] + kr * rr + Kc.kyl1 * ylo + Kc.kyu1 * yhi +
              Kc.kz1 * Xp1[c] + Kn.kz1 * Xn1[c];
          Xc1[c] = cell_ok ? Kc.d1 * v : zero;
        }
      }
    }
    // second colour on plane p-1, element e (rows y0 .. y0+TY-1), and output
    if (p - 1 >= zs) {
      const int z = p - 1;
#pragma unroll
      for (int c = 0; c < COLS; ++c) {
        const T ylo = xb[buf][r > 0 ? r - 1 : 0][c][pl];
        const T yhi = xb[buf][r < RW - 1 ? r + 1 : RW - 1][c][pl];
        {
          if (e == 0) {
            const T sh = wave_shr1(Xp1[c]);
            const T l = pl > 0 ? sh : zero;
            const T v = Bp0[c] + Kp.kx0 * l + Kp.kx1 * Xp1[c] + Kp.kyl0 * ylo + Kp.kyu0 * yhi +
                        Kp.kz0 * Xq0[c] + Kc.kz0 * Xc0[c];
            if (inner) Xp0[c] = cell_ok ? Kp.d0 * v : zero;
          } else {
            const T sh = wave_shl1(Xp0[c]);
            const R shk = wave_shl1(Kp.kx0);
            const T rr = x0 + 2 < N ? sh : zero;
            const R kr = x0 + 2 < N ? shk : (R)0;
            const T v = Bp1[c] + Kp.kx1 * Xp0[c] + kr * rr + Kp.kyl1 * ylo + Kp.kyu1 * yhi +
                        Kp.kz1 * Xq1[c] + Kc.kz1 * Xc1[c];
            if (inner) Xp1[c] = cell_ok ? Kp.d1 * v : zero;
          }
          if (owner && xok && con[c]) {
            const int64_t i = ((int64_t)z * N + y) * N + x0;
            xo[c][i] = Xp0[c];
            xo[c][i + 1] = Xp1[c];
          }
        }
      }
    }
  }
}

}  // namespace

int varcoef_blocks(int N) { return (N * N * N + kThreads - 1) / kThreads; }

#define VC_COLS_DISPATCH(COLSV, ...)                                           \
  switch (COLSV) {                                                            \
    case 1: { constexpr int C = 1; __VA_ARGS__; break; }                      \
    case 2: { constexpr int C = 2; __VA_ARGS__; break; }                      \
    case 4: { constexpr int C = 4; __VA_ARGS__; break; }                      \
    case 8: { constexpr int C = 8; __VA_ARGS__; break; }                      \
    default: throw Error(MLMC_EINVAL, "columns per thread must be 1, 2, 4 or 8"); \
  }

template <typename Tb, typename T, typename Tr>
void varcoef_residual(const Tb* b, const T* x, Tr* r, const typename Traits<T>::real* kl,
                      const typename Traits<T>::real* dg, int N, int nb, int cols,
                      const int* active, c64* partials, hipStream_t s) {
  const dim3 g((unsigned)varcoef_blocks(N), (unsigned)((nb + cols - 1) / cols));
  VC_COLS_DISPATCH(cols, MLMC_LAUNCH((k_vc_residual<Tb, T, Tr, C>), g, dim3(kThreads), 0, s, b, x,
                                     r, kl, dg, N, nb, active, partials, timing_log()));
}

template <typename T>
void varcoef_rbgs(const T* b, T* x, const typename Traits<T>::real* kl,
                  const typename Traits<T>::real* dg, int N, int nb, int cols, const int* active,
                  bool zero_init, bool reverse, const T* ec, double omega, hipStream_t s) {
  using R = typename Traits<T>::real;
  const int64_t half = (int64_t)N * N * N / 2;
  const dim3 g((unsigned)((half + kThreads - 1) / kThreads), (unsigned)((nb + cols - 1) / cols));
  const int first = reverse ? 1 : 0;
  const R ws = (R)(omega * 0.35355339059327373);  // omega / sqrt(8)
  VC_COLS_DISPATCH(cols, {
    MLMC_LAUNCH((k_vc_gs<T, C>), g, dim3(kThreads), 0, s, b, x, kl, dg, N, first,
                zero_init ? 1 : 0, nb, active, ec, ws, timing_log());
    MLMC_LAUNCH((k_vc_gs<T, C>), g, dim3(kThreads), 0, s, b, x, kl, dg, N, 1 - first, 0, nb,
                active, (const T*)nullptr, (R)0, (int*)nullptr);
  });
}

template <typename T, int RPW>
static void vc_march_launch(const T* xin, const T* b, T* xout, const T* ec, double omega,
                            const typename Traits<T>::real* kl,
                            const typename Traits<T>::real* dg, int N, int nb, int cols,
                            const int* active, bool reverse, hipStream_t s) {
  using R = typename Traits<T>::real;
  constexpr int TY = kMarchWaves * RPW - 2;
  const R ws = (R)(omega * 0.35355339059327373);  // omega / sqrt(8)
  const T* xp = xin ? xin : b;  // placeholders (never read) for the templated forms
  const T* ep = ec ? ec : b;
  const dim3 blk(kMarchWaves * 64);
  const int first = reverse ? 1 : 0;
  // z segments of SZ planes: more workgroups in flight than one march per
  // column of rows, at the price of 3 extra planes read per segment
  const int SZ = N >= 32 ? 16 : N;
#define VC_MARCH(HX, HE)                                                                      \
  VC_COLS_DISPATCH(cols, {                                                                    \
    const dim3 g((unsigned)((N + TY - 1) / TY), (unsigned)((nb + C - 1) / C),                 \
                 (unsigned)((N + SZ - 1) / SZ));                                              \
    if (first)                                                                                \
      MLMC_LAUNCH((k_vc_march<T, C, RPW, HX, HE, 1>), g, blk, 0, s, xp, b, xout, ep, ws, kl,   \
                  dg, N, SZ, nb, active, timing_log());                                       \
    else                                                                                      \
      MLMC_LAUNCH((k_vc_march<T, C, RPW, HX, HE, 0>), g, blk, 0, s, xp, b, xout, ep, ws, kl,   \
                  dg, N, SZ, nb, active, timing_log());                                       \
  })
  if (xin && ec) {
    VC_MARCH(true, true);
  } else if (xin) {
    VC_MARCH(true, false);
  } else if (ec) {
    VC_MARCH(false, true);
  } else {
    VC_MARCH(false, false);
  }
#undef VC_MARCH
}

bool varcoef_march_ok(int N) { return N <= 128 && N % 2 == 0; }

template <typename T>
void varcoef_rbgs_march(const T* xin, const T* b, T* xout, const T* ec, double omega,
                        const typename Traits<T>::real* kl, const typename Traits<T>::real* dg,
                        int N, int nb, int cols, const int* active, bool reverse,
                        hipStream_t s) {
  if (!varcoef_march_ok(N)) throw Error(MLMC_EINVAL, "fused 3D sweep needs an even side <= 128");
  if (cols == 8) throw Error(MLMC_EINVAL, "fused 3D sweep takes 1, 2 or 4 columns per wave");
  // rows per wave: as many as fit 64 lane pairs (a row of N needs N/2 lanes)
  if (N <= 32)
    vc_march_launch<T, 4>(xin, b, xout, ec, omega, kl, dg, N, nb, cols, active, reverse, s);
  else if (N <= 64)
    vc_march_launch<T, 2>(xin, b, xout, ec, omega, kl, dg, N, nb, cols, active, reverse, s);
  else
    vc_march_launch<T, 1>(xin, b, xout, ec, omega, kl, dg, N, nb, cols, active, reverse, s);
}

template <typename T>
void varcoef_restrict(const T* b, const T* x, T* xc, const typename Traits<T>::real* kl,
                      const typename Traits<T>::real* dg, int N, bool residual, int nb, int cols,
                      const int* active, hipStream_t s) {
  const int64_t nc = (int64_t)(N / 2) * (N / 2) * (N / 2);
  const dim3 g((unsigned)((nc + kThreads - 1) / kThreads), (unsigned)((nb + cols - 1) / cols));
  if (residual) {
    VC_COLS_DISPATCH(cols, MLMC_LAUNCH((k_vc_res_restrict<T, C>), g, dim3(kThreads), 0, s, b, x,
                                       xc, kl, dg, N, nb, active, timing_log()));
  } else {
    VC_COLS_DISPATCH(cols, MLMC_LAUNCH((k_vc_restrict<T, C>), g, dim3(kThreads), 0, s, b, x, xc,
                                       kl, dg, N, 0, nb, active, timing_log()));
  }
}

template <typename T>
void varcoef_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                     const int* active, hipStream_t s) {
  const int64_t n = (int64_t)N * N * N;
  MLMC_LAUNCH(k_vc_prolong<T>, dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb),
              dim3(kThreads), 0, s, ec, x, N,
              (typename Traits<T>::real)(omega * 0.35355339059327373),
              (typename Traits<T>::real)beta, active, timing_log());
}

template <typename T>
void varcoef_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                          const typename Traits<T>::real* kl,
                          const typename Traits<T>::real* dg, int N, int nb, int cols,
                          const int* active, c64* partials, hipStream_t s) {
  const dim3 g((unsigned)varcoef_blocks(N), (unsigned)((nb + cols - 1) / cols));
  VC_COLS_DISPATCH(cols, MLMC_LAUNCH((k_vc_update_apply<T, C>), g, dim3(kThreads), 0, s, p_old,
                                     z, beta, p_new, q, kl, dg, N, nb, active, partials,
                                     timing_log()));
}

void varcoef_coarsen(const double* kf, double* kc, int N, hipStream_t s) {
  MLMC_LAUNCH(k_vc_coarsen, dim3(256), dim3(256), 0, s, kf, kc, N);
}

void varcoef_diag(const double* k, double shift, int N, double* d64, float* d32, double* kl64,
                  float* kl32, hipStream_t s) {
  MLMC_LAUNCH(k_vc_diag, dim3(512), dim3(256), 0, s, k, shift, N, d64, d32, kl64, kl32);
}

void varcoef_dense(const double* k, const double* diag, int N, double* aug, hipStream_t s) {
  MLMC_LAUNCH(k_vc_dense, dim3(N * N * N), dim3(256), 0, s, k, diag, N, aug);
}

#define VC_INST(T)                                                                          \
  template void varcoef_rbgs<T>(const T*, T*, const T*, const T*, int, int, int, const int*,  \
                                bool, bool, const T*, double, hipStream_t);                  \
  template void varcoef_rbgs_march<T>(const T*, const T*, T*, const T*, double, const T*,    \
                                      const T*, int, int, int, const int*, bool,             \
                                      hipStream_t);                                          \
  template void varcoef_restrict<T>(const T*, const T*, T*, const T*, const T*, int, bool,    \
                                    int, int, const int*, hipStream_t);                      \
  template void varcoef_prolong<T>(const T*, T*, int, double, double, int, const int*,        \
                                   hipStream_t);                                             \
  template void varcoef_update_apply<T>(const T*, const T*, const c64*, T*, T*, const T*,    \
                                        const T*, int, int, int, const int*, c64*,           \
                                        hipStream_t);
VC_INST(float)
VC_INST(double)
template void varcoef_residual<double, double, double>(const double*, const double*, double*,
                                                       const double*, const double*, int, int,
                                                       int, const int*, c64*, hipStream_t);
template void varcoef_residual<double, double, float>(const double*, const double*, float*,
                                                      const double*, const double*, int, int,
                                                      int, const int*, c64*, hipStream_t);
template void varcoef_residual<float, float, float>(const float*, const float*, float*,
                                                    const float*, const float*, int, int, int,
                                                    const int*, c64*, hipStream_t);

}  // namespace mlmc
