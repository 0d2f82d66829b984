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
#include "vc_body.h"

namespace mlmc {
namespace {

using namespace vcb;

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

// r = b - A x (or r = A x when b is null); partials per column and block
template <typename Tb, typename T, typename Tr, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_residual(const Tb* __restrict__ b,
                                                          const T* __restrict__ x,
                                                          Tr* __restrict__ r,
                                                          const R_t<T>* __restrict__ kl,
                                                          const R_t<T>* __restrict__ dg, int N,
                                                          int nb, const int* active,
                                                          c64* partials, int* tlog) {
  __shared__ double red[16];
  vc_residual<Tb, T, Tr, COLS>(b, x, r, kl, dg, N, nb, active, partials, tlog, blockIdx.x,
                               blockIdx.y, gridDim.x, red);
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

// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q
template <typename T, int COLS>
__global__ __launch_bounds__(kThreads) void k_vc_update_apply(
    const T* __restrict__ p_old, const T* __restrict__ z, const c64* __restrict__ beta,
    T* __restrict__ p_new, T* __restrict__ q, const R_t<T>* __restrict__ kl,
    const R_t<T>* __restrict__ dg, int N, int nb, const int* active, c64* partials, int* tlog) {
  __shared__ double red[16];
  vc_update_apply<T, COLS>(p_old, z, beta, p_new, q, kl, dg, N, nb, active, partials, tlog,
                           blockIdx.x, blockIdx.y, gridDim.x, red);
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
  vc_res_restrict<T, COLS, kThreads>(b, x, rc, kl, dg, N, nb, active, tlog, blockIdx.x,
                                     blockIdx.y, threadIdx.x);
}

// one fused red-black sweep, out of place, marching along z (vc_march)
template <typename T, int COLS, int RPW, bool HX, bool HE, int F>
__global__ __launch_bounds__(kMarchWaves * 64) void k_vc_march(
    const T* __restrict__ xin, const T* __restrict__ b, T* __restrict__ xout,
    const T* __restrict__ ec, R_t<T> ws, const R_t<T>* __restrict__ kl,
    const R_t<T>* __restrict__ dg, int N, int SZ, int nb, const int* active, int* tlog) {
  __shared__ T lds[vc_march_lds<T, COLS, RPW>()];
  vc_march<T, COLS, RPW, HX, HE, F>(xin, b, xout, ec, ws, kl, dg, N, SZ, nb, active, tlog,
                                    blockIdx.x, blockIdx.y, blockIdx.z, lds);
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
