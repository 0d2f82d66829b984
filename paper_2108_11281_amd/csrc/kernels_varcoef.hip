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

template <typename T>
void varcoef_restrict(const T* b, const T* x, T* xc, const typename Traits<T>::real* kl,
                      const typename Traits<T>::real* dg, int N, bool residual, int nb, int cols,
                      const int* active, hipStream_t s) {
  const int64_t nc = (int64_t)(N / 2) * (N / 2) * (N / 2);
  const dim3 g((unsigned)((nc + kThreads - 1) / kThreads), (unsigned)((nb + cols - 1) / cols));
  VC_COLS_DISPATCH(cols, MLMC_LAUNCH((k_vc_restrict<T, C>), g, dim3(kThreads), 0, s, b, x, xc,
                                     kl, dg, N, residual ? 1 : 0, nb, active, timing_log()));
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
