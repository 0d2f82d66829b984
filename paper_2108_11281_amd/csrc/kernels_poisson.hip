// 2D Poisson stencil kernels, matrix-free: A = d I - c (grid neighbours) on an
// N x N Dirichlet grid, unknown i = y*N + x, one grid plane per right-hand side.
// With 2x2 orthonormal aggregation the Galerkin operator of such a stencil is
// again one (d' = d - 2c, c' = c/2), so every level runs on these kernels.
//
// Launch shape: 1D grids of 256-thread blocks over (plane, tile) pairs with an
// XCD-aware order: the hardware deals consecutive block ids round-robin to the
// 8 XCDs, so block b is mapped to the logical tile range owned by XCD b % 8 and
// each XCD sweeps a contiguous run of tiles (neighbouring tiles share halo
// cache lines in that XCD's L2).
#include "kernels.h"
#include "lanes.h"

namespace mlmc {
namespace {

template <typename T> using R_t = typename Traits<T>::real;

constexpr int kXcds = 8;

// logical tile index of this block: a bijection that gives XCD x the
// contiguous range [x*q + min(x, r), ...) of the `total` tiles
__device__ __forceinline__ int xcd_tile_index(int total) {
  const int b = blockIdx.x;
  const int x = b % kXcds, local = b / kXcds;
  const int q = total / kXcds, r = total % kXcds;
  return x * q + (x < r ? x : r) + local;
}

// ---------------------------------------------------------------------------
// Fused red-black Gauss-Seidel sweep on a TX x TY tile staged in LDS.
//   x_out = S(x_in + omega/2 * P e_c ; b)   (one full sweep, first colour
//   `first`, then the other), Dirichlet zeros outside the grid.
// The tile is loaded with a 2-cell halo of x and a 1-cell halo of b; the first
// colour is updated on the tile plus a 1-cell ring (redundantly with the
// neighbouring tiles), so the second colour sees all its updated neighbours.
// x_in == nullptr means x_in = 0; ec == nullptr means no coarse correction.
// With partials, each block also writes its share of conj(b)^T x_out (the
// r^T z of the Krylov method when b = r and x_out = z).
// ---------------------------------------------------------------------------
constexpr int GTX = 128, GTY = 16;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_rbgs_tile(const T* __restrict__ xin,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ xout,
                                                        const T* __restrict__ ec,
                                                        R_t<T> wh, int N, R_t<T> dinv,
                                                        R_t<T> c, int first, int nbx, int nby,
                                                        int nb, const int* active,
                                                        c64* partials, int* tlog) {
  __shared__ T sx[GTY + 4][GTX + 4];
  __shared__ T sb[GTY + 2][GTX + 2];
  __shared__ double red[16];
  const int t = xcd_tile_index(nbx * nby * nb);
  const int k = t / (nbx * nby);
  const int rem = t - k * nbx * nby;
  const int by = rem / nbx, bx = rem - by * nbx;
  if (tlog && rem == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (k >= nb || (active && !active[k])) return;
  const int x0 = bx * GTX, y0 = by * GTY;
  const int64_t n = (int64_t)N * N;
  const int Nc = N >> 1;
  const T* xc = xin ? xin + (int64_t)k * n : nullptr;
  const T* bc = b + (int64_t)k * n;
  const T* ecc = ec ? ec + (int64_t)k * Nc * Nc : nullptr;
  const int tid = threadIdx.x;

  // all global loads are issued before the first LDS store, so that each
  // thread keeps ~20 loads in flight
  constexpr int NX = (GTY + 4) * (GTX + 4), NB = (GTY + 2) * (GTX + 2);
  constexpr int LX = (NX + kThreads - 1) / kThreads, LB = (NB + kThreads - 1) / kThreads;
  T vx[LX], vb[LB];
#pragma unroll
  for (int j = 0; j < LX; ++j) {
    const int idx = tid + j * kThreads;
    const int r = idx / (GTX + 4), cc = idx - r * (GTX + 4);
    const int gx = x0 - 2 + cc, gy = y0 - 2 + r;
    T v = zero_of(T());
    if (idx < NX && gx >= 0 && gx < N && gy >= 0 && gy < N) {
      if (xc) v = xc[gy * N + gx];
      if (ecc) v += wh * ecc[(gy >> 1) * Nc + (gx >> 1)];
    }
    vx[j] = v;
  }
#pragma unroll
  for (int j = 0; j < LB; ++j) {
    const int idx = tid + j * kThreads;
    const int r = idx / (GTX + 2), cc = idx - r * (GTX + 2);
    const int gx = x0 - 1 + cc, gy = y0 - 1 + r;
    vb[j] = (idx < NB && gx >= 0 && gx < N && gy >= 0 && gy < N) ? bc[gy * N + gx]
                                                                  : zero_of(T());
  }
#pragma unroll
  for (int j = 0; j < LX; ++j) {
    const int idx = tid + j * kThreads;
    if (idx < NX) (&sx[0][0])[idx] = vx[j];
  }
#pragma unroll
  for (int j = 0; j < LB; ++j) {
    const int idx = tid + j * kThreads;
    if (idx < NB) (&sb[0][0])[idx] = vb[j];
  }
  __syncthreads();
  // first colour on the tile and its 1-cell ring
  for (int idx = tid; idx < (GTY + 2) * (GTX + 2); idx += kThreads) {
    const int r = idx / (GTX + 2), cc = idx - r * (GTX + 2);
    const int gx = x0 - 1 + cc, gy = y0 - 1 + r;
    if (gx >= 0 && gx < N && gy >= 0 && gy < N && ((gx + gy) & 1) == first) {
      sx[r + 1][cc + 1] =
          dinv * (sb[r][cc] + c * (sx[r + 1][cc] + sx[r + 1][cc + 2] + sx[r][cc + 1] +
                                   sx[r + 2][cc + 1]));
    }
  }
  __syncthreads();
  // second colour on the tile; write the tile
  double dre = 0.0, dim = 0.0;
  T* xo = xout + (int64_t)k * n;
  for (int idx = tid; idx < GTY * GTX; idx += kThreads) {
    const int r = idx / GTX, cc = idx - r * GTX;
    const int gx = x0 + cc, gy = y0 + r;
    if (gx < N && gy < N) {
      T v;
      if (((gx + gy) & 1) != first)
        v = dinv * (sb[r + 1][cc + 1] + c * (sx[r + 2][cc + 1] + sx[r + 2][cc + 3] +
                                             sx[r + 1][cc + 2] + sx[r + 3][cc + 2]));
      else
        v = sx[r + 2][cc + 2];
      xo[gy * N + gx] = v;
      if (partials) cdot_acc(dre, dim, sb[r + 1][cc + 1], v);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (tid == 0) partials[(int64_t)k * (nbx * nby) + rem] = {dre, dim};
  }
}

// ---------------------------------------------------------------------------
// Fused red-black Gauss-Seidel sweep, column-marching form (no LDS):
//   x_out = S(x_in + omega/2 * P e_c ; b)
// A wave owns 62 consecutive columns (lanes 1..62; lanes 0 and 63 are halo
// lanes that redo the first colour of the neighbouring columns) and walks a
// segment of SR rows top to bottom.  At row yy it loads x_in(yy) and b(yy),
// updates the first colour on row yy-1 (its vertical neighbours yy-2 and yy
// are in registers, horizontal ones come from the neighbouring lanes) and then
// the second colour on row yy-2 from the updated first colour of rows
// yy-3..yy-1.  Every input value is read once and every output written once:
// 12 bytes per unknown for FP32 (plus 1/4 element for the folded coarse
// correction and 4 extra rows per segment of SR).
// ---------------------------------------------------------------------------
constexpr int SCOLS = 62;       // owned columns per wave

// rows per segment (SR): all loads of a segment are issued before its
// arithmetic, so the row count is bounded by registers (4 values per row and
// lane); chosen per level by the setup-time autotuner among gs_rows_options

// branch-free guarded load: the address is always valid (clamped to the base)
template <typename T>
__device__ __forceinline__ T ldz(const T* p, int idx, bool ok) {
  const T v = p[ok ? idx : 0];
  return ok ? v : zero_of(T());
}

template <typename T, bool HX, bool HE, int SR>
__global__ __launch_bounds__(kThreads) void k_rbgs_march(const T* __restrict__ xin,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ xout,
                                                         const T* __restrict__ ec, R_t<T> wh,
                                                         int N, R_t<T> dinv, R_t<T> c,
                                                         int first, int nb, const int* active,
                                                         c64* partials, int* tlog) {
  constexpr int NR = SR + 4;
  __shared__ double red[16];
  const int nwx = (N + SCOLS - 1) / SCOLS, nseg = (N + SR - 1) / SR;
  const int units_per_plane = nwx * nseg;
  const int blocks_per_plane = (units_per_plane + 3) / 4;
  const int t = xcd_tile_index(blocks_per_plane * nb);
  const int k = t / blocks_per_plane;
  const int bp = t - k * blocks_per_plane;
  if (tlog && bp == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (k >= nb || (active && !active[k])) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int unit = bp * 4 + w;                // unit = seg * nwx + wx within the plane
  const bool unit_ok = unit < units_per_plane;
  const int seg = unit / nwx, wx = unit - seg * nwx;
  const int x = wx * SCOLS - 1 + lane;
  const int ys = seg * SR;
  const int yend = ys + SR < N ? ys + SR : N;
  const bool col_in = unit_ok && x >= 0 && x < N;
  const bool owned = col_in && lane >= 1 && lane <= SCOLS;
  // the two halo lanes load their outer neighbour column (only they read E)
  const int xe = (lane == 0) ? x - 1 : (lane == 63 ? x + 1 : x);
  const bool edge_in = unit_ok && (lane == 0 || lane == 63) && xe >= 0 && xe < N;
  const int64_t n = (int64_t)N * N;
  const int Nc = N >> 1;
  const T* xc = xin + (HX ? (int64_t)k * n : 0);
  const T* bc = b + (int64_t)k * n;
  const T* ecc = ec + (HE ? (int64_t)k * Nc * Nc : 0);
  T* xo = xout + (int64_t)k * n;
  const T zero = zero_of(T());

  T X[NR], E[NR], B[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int yy = ys - 2 + r;
    const bool rok = yy >= 0 && yy < N;
    const bool okc = col_in && rok, oke = edge_in && rok;
    T xv = zero, ev = zero;
    if constexpr (HX) {
      xv = ldz(xc, yy * N + x, okc);
      ev = ldz(xc, yy * N + xe, oke);
    }
    if constexpr (HE) {
      xv += wh * ldz(ecc, (yy >> 1) * Nc + (x >> 1), okc);
      ev += wh * ldz(ecc, (yy >> 1) * Nc + (xe >> 1), oke);
    }
    X[r] = xv;
    E[r] = ev;
    B[r] = ldz(bc, yy * N + x, okc);
  }
  // first colour on rows ys-1 .. ys+SR (index r = row - (ys-2))
  T N1[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) N1[r] = zero;
#pragma unroll
  for (int r = 1; r < NR - 1; ++r) {
    const int y1 = ys - 2 + r;
    const T sl = wave_shr1(X[r]), sr = wave_shl1(X[r]);
    const T xl = (lane == 0) ? E[r] : sl;
    const T xr = (lane == 63) ? E[r] : sr;
    const bool ok = col_in && y1 >= 0 && y1 < N && ((x + y1) & 1) == first;
    const T v = dinv * (B[r] + c * (xl + xr + X[r - 1] + X[r + 1]));
    N1[r] = ok ? v : zero;
  }
  // second colour and output on rows ys .. yend-1 (r = 2 .. SR+1)
  double dre = 0.0, dim = 0.0;
#pragma unroll
  for (int r = 2; r < NR - 2; ++r) {
    const int y2 = ys - 2 + r;
    const T sl = wave_shr1(N1[r]), sr = wave_shl1(N1[r]);
    const T v2 = dinv * (B[r] + c * (sl + sr + N1[r - 1] + N1[r + 1]));
    const T v = (((x + y2) & 1) == first) ? N1[r] : v2;
    if (owned && y2 < yend) {
      xo[y2 * N + x] = v;
      if (partials) cdot_acc(dre, dim, B[r], v);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)k * blocks_per_plane + bp] = {dre, dim};
  }
}

// ---------------------------------------------------------------------------
// Two fused red-black sweeps (the march above blocked in time):
//   x_out = S(S(x_in + omega/2 * P e_c ; b) ; b)
// Each lane holds two adjacent columns (an even and an odd one), so in every
// row exactly one of its two cells has the colour being updated: a colour stage
// costs one update and one DPP lane shift per lane and row, and the loads are
// 2-element vectors.  The four colour stages (first, second, first, second)
// update the register rows in place (a colour's neighbours all have the other
// colour).  Each stage is valid one column and one row further in than the one
// before, so a wave owns lanes 2..61 (120 columns) and a segment of SR output
// rows loads SR + 8 rows.  HBM traffic is that of one sweep (x_in and b in,
// x_out out); every updated value is formed by the same operations, in the
// same order, as in two launches of the one-sweep kernel, so the results agree
// bit for bit.  Needs N even (every smoothed level has a coarser one).
// ---------------------------------------------------------------------------
// RS (the last pre-smoothing pass): the pass also writes the restricted
// residual rc = R (b - A x_out) of 2x2 aggregates (a lane's column pair is one
// aggregate column); the residual needs x_out one column and one row beyond
// the owned cells, so a wave then owns lanes 3..60 and loads SR + 10 rows.
template <bool RS> constexpr int rbgs2_first_lane() { return RS ? 3 : 2; }
template <bool RS> constexpr int rbgs2_cols() { return 2 * (64 - 2 * rbgs2_first_lane<RS>()); }
constexpr int SCOLS2 = rbgs2_cols<false>();  // 120 owned columns per wave

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T e0, e1;
};

template <typename T, bool HX, bool HE, int SR, int F, bool RS>
__global__ __launch_bounds__(kThreads) void k_rbgs2_march(const T* __restrict__ xin,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ xout,
                                                          const T* __restrict__ ec, R_t<T> wh,
                                                          int N, R_t<T> dinv, R_t<T> d, R_t<T> c,
                                                          int nb, const int* active,
                                                          c64* partials, T* __restrict__ rc,
                                                          int* tlog) {
  constexpr int HALO = RS ? 5 : 4;            // rows loaded above and below a segment
  constexpr int NR = SR + 2 * HALO;
  constexpr int LO = rbgs2_first_lane<RS>(), HI = 63 - LO;
  constexpr int COLS = rbgs2_cols<RS>();
  __shared__ double red[16];
  const int nwx = (N + COLS - 1) / COLS, nseg = (N + SR - 1) / SR;
  const int units_per_plane = nwx * nseg;
  const int blocks_per_plane = (units_per_plane + 3) / 4;
  const int t = xcd_tile_index(blocks_per_plane * nb);
  const int k = t / blocks_per_plane;
  const int bp = t - k * blocks_per_plane;
  if (tlog && bp == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (k >= nb || (active && !active[k])) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int unit = bp * 4 + w;                // unit = seg * nwx + wx within the plane
  const bool unit_ok = unit < units_per_plane;
  const int seg = unit / nwx, wx = unit - seg * nwx;
  const int x = wx * COLS - 2 * LO + 2 * lane;  // even column of the lane's pair
  const int ys = seg * SR;                    // even: row ys-HALO+r has the parity of r+HALO
  const int yend = ys + SR < N ? ys + SR : N;
  const bool col_in = unit_ok && x >= 0 && x < N;
  const bool owned = col_in && lane >= LO && lane <= HI;
  const int64_t n = (int64_t)N * N;
  const int Nc = N >> 1;
  const Pair<T>* xc = reinterpret_cast<const Pair<T>*>(xin + (HX ? (int64_t)k * n : 0));
  const Pair<T>* bc = reinterpret_cast<const Pair<T>*>(b + (int64_t)k * n);
  const T* ecc = ec + (HE ? (int64_t)k * Nc * Nc : 0);
  Pair<T>* xo = reinterpret_cast<Pair<T>*>(xout + (int64_t)k * n);
  const T zero = zero_of(T());
  const int half = N >> 1;                    // pairs per row
  const int px = x >> 1;

  // rows ys-HALO .. ys+SR+HALO-1 (index r = row - (ys-HALO)); b on rows 1..NR-2
  T S0[NR], S1[NR], B0[NR], B1[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int yy = ys - HALO + r;
    const bool ok = col_in && yy >= 0 && yy < N;
    T v0 = zero, v1 = zero;
    if constexpr (HX) {
      const Pair<T> p = xc[ok ? yy * half + px : 0];
      v0 = ok ? p.e0 : zero;
      v1 = ok ? p.e1 : zero;
    }
    if constexpr (HE) {
      // both columns of the pair lie in one 2x2 aggregate
      const T e = ldz(ecc, (yy >> 1) * Nc + px, ok);
      v0 += wh * e;
      v1 += wh * e;
    }
    S0[r] = v0;
    S1[r] = v1;
    if (r >= 1 && r <= NR - 2) {
      const Pair<T> q = bc[ok ? yy * half + px : 0];
      B0[r] = ok ? q.e0 : zero;
      B1[r] = ok ? q.e1 : zero;
    } else {
      B0[r] = zero;
      B1[r] = zero;
    }
  }
  auto in_grid = [&](int r) {
    const int yy = ys - HALO + r;
    return col_in && yy >= 0 && yy < N;
  };
  // one colour stage on rows lo..NR-1-lo: in row r the lane's cell of colour
  // C is its even column when C + r + HALO is even, else its odd column
  auto stage = [&](auto colour, int lo) {
    constexpr int C = decltype(colour)::value;
#pragma unroll
    for (int r = lo; r < NR - lo; ++r) {
      if (((C + r + HALO) & 1) == 0) {
        const T xl = wave_shr1(S1[r]), xr = S1[r];
        const T v = dinv * (B0[r] + c * (xl + xr + S0[r - 1] + S0[r + 1]));
        S0[r] = in_grid(r) ? v : zero;
      } else {
        const T xl = S0[r], xr = wave_shl1(S0[r]);
        const T v = dinv * (B1[r] + c * (xl + xr + S1[r - 1] + S1[r + 1]));
        S1[r] = in_grid(r) ? v : zero;
      }
    }
  };
  using First = std::integral_constant<int, F>;
  using Second = std::integral_constant<int, 1 - F>;
  stage(First(), 1);    // valid on columns 1..126 of the wave's 128
  stage(Second(), 2);   // 2..125
  stage(First(), 3);    // 3..124
  stage(Second(), 4);   // 4..123 (lanes 2..61)
  double dre = 0.0, dim = 0.0;
#pragma unroll
  for (int r = HALO; r < NR - HALO; ++r) {
    const int y2 = ys - HALO + r;
    if (owned && y2 < yend) {
      xo[y2 * half + px] = Pair<T>{S0[r], S1[r]};
      if (partials) {
        cdot_acc(dre, dim, B0[r], S0[r]);
        cdot_acc(dre, dim, B1[r], S1[r]);
      }
    }
  }
  if constexpr (RS) {
    // rc(px, Y) = 1/2 sum over the aggregate's 4 cells of (b - A x_out), in the
    // order of the stand-alone residual-restriction kernel
    T* rcc = rc + (int64_t)k * Nc * Nc;
#pragma unroll
    for (int r = HALO; r < NR - HALO; r += 2) {
      T acc = zero;
#pragma unroll
      for (int dy = 0; dy < 2; ++dy) {
        const int j = r + dy;
        const T xl = wave_shr1(S1[j]), xr = wave_shl1(S0[j]);
        acc += B0[j] - (d * S0[j] - c * (xl + S1[j] + S0[j - 1] + S0[j + 1]));
        acc += B1[j] - (d * S1[j] - c * (S0[j] + xr + S1[j - 1] + S1[j + 1]));
      }
      const int y2 = ys - HALO + r;
      if (owned && y2 < yend) rcc[(y2 >> 1) * Nc + px] = (R_t<T>)0.5 * acc;
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)k * blocks_per_plane + bp] = {dre, dim};
  }
}

// ---------------------------------------------------------------------------
// Row-marching stencil kernels: a block covers 64 consecutive x (one wave per
// row group) and 4 x MY rows; each thread walks MY rows keeping the vertical
// neighbours in registers.  Tile = 64 x (4*MY).
// ---------------------------------------------------------------------------
constexpr int MX = 64, MW = 4, MY = 8, MTY = MW * MY;

struct MarchTile {
  int k, rem, x, ybeg, yend;
  bool ok;
};

template <int RY = MY>
__device__ __forceinline__ MarchTile march_tile(int N, int nb, const int* active) {
  constexpr int TY = MW * RY;
  const int nbx = (N + MX - 1) / MX, nby = (N + TY - 1) / TY;
  const int t = xcd_tile_index(nbx * nby * nb);
  MarchTile m;
  m.k = t / (nbx * nby);
  m.rem = t - m.k * nbx * nby;
  const int by = m.rem / nbx, bx = m.rem - by * nbx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  m.x = bx * MX + lane;
  m.ybeg = by * TY + w * RY;
  m.yend = m.ybeg + RY < N ? m.ybeg + RY : N;
  m.ok = m.k < nb && !(active && !active[m.k]);
  return m;
}

template <typename T>
__device__ __forceinline__ T ld_or0(const T* p, int x, int y, int N) {
  return (x >= 0 && x < N && y >= 0 && y < N) ? p[y * N + x] : zero_of(T());
}

// y = A p (+ partials of conj(p)^T y).  With z and beta given, the product is
// taken of the updated Krylov direction p = z + beta * p_old, recomputed at the
// neighbours from (z, p_old) and written to p_new (a different buffer, so no
// block reads a value another block has already replaced).
template <typename T, bool UPD>
__global__ __launch_bounds__(kThreads) void k_apply_march(const T* __restrict__ x,
                                                          const T* __restrict__ z,
                                                          const c64* beta, T* __restrict__ xnew,
                                                          T* __restrict__ y, int N, R_t<T> d,
                                                          R_t<T> c, int nb, const int* active,
                                                          c64* partials, int* tlog) {
  __shared__ double red[16];
  const MarchTile m = march_tile(N, nb, active);
  if (tlog && m.rem == 0 && threadIdx.x == 0) tlog[m.k] = active ? active[m.k] : 1;
  if (!m.ok) return;
  const int64_t n = (int64_t)N * N;
  const T* xc = x + (int64_t)m.k * n;
  const T* zc = z + (UPD ? (int64_t)m.k * n : 0);
  T* xn = xnew + (UPD ? (int64_t)m.k * n : 0);
  T* yc = y + (int64_t)m.k * n;
  double dre = 0.0, dim = 0.0;
  c64 bt = {0.0, 0.0};
  if (UPD) bt = beta[m.k];
  const bool col_ok = m.x < N;
  const int xs = col_ok ? m.x : 0;
  const int lane = threadIdx.x & 63;  // a wave covers 64 consecutive columns
  // loads first (branch-free): the column (rows ybeg-1 .. ybeg+MY); the side
  // columns come from the neighbouring lanes (DPP), except for the two edge
  // lanes, which load the column beyond the wave
  T cz[MY + 2], cx[MY + 2], ez[MY], ex[MY];
#pragma unroll
  for (int j = 0; j < MY + 2; ++j) {
    const int yy = m.ybeg - 1 + j;
    const bool ok = col_ok && yy >= 0 && yy < N && yy <= m.yend;
    cx[j] = ldz(xc, yy * N + xs, ok);
    cz[j] = UPD ? ldz(zc, yy * N + xs, ok) : zero_of(T());
  }
  const int xe = lane == 0 ? m.x - 1 : m.x + 1;  // edge lanes' outer column
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < N;
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const bool ok = edge && yy < m.yend;
    ex[j] = ldz(xc, yy * N + xe, ok);
    ez[j] = UPD ? ldz(zc, yy * N + xe, ok) : zero_of(T());
  }
  auto P = [&](T zz, T xx) -> T { return UPD ? zz + scale_by(bt.re, bt.im, xx) : xx; };
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const T mid = P(cz[j + 1], cx[j + 1]);
    const T pe = P(ez[j], ex[j]);
    const T sl = wave_shr1(mid), sr = wave_shl1(mid);
    const T left = lane == 0 ? pe : sl;
    const T right = lane == 63 ? pe : sr;
    const T v = d * mid - c * (P(cz[j], cx[j]) + P(cz[j + 2], cx[j + 2]) + left + right);
    if (col_ok && yy < m.yend) {
      yc[yy * N + m.x] = v;
      if (UPD) xn[yy * N + m.x] = mid;
      cdot_acc(dre, dim, mid, v);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) {
      const int tiles = ((N + MX - 1) / MX) * ((N + MTY - 1) / MTY);
      partials[(int64_t)m.k * tiles + m.rem] = {dre, dim};
    }
  }
}

// r = b - A x (any precisions) with optional partials of |r|^2
template <typename Tb, typename Tx, typename Tr>
__global__ __launch_bounds__(kThreads) void k_residual_march(const Tb* __restrict__ b,
                                                             const Tx* __restrict__ x,
                                                             Tr* __restrict__ r, int N,
                                                             R_t<Tx> d, R_t<Tx> c, int nb,
                                                             const int* active,
                                                             c64* partials, int* tlog) {
  __shared__ double red[16];
  const MarchTile m = march_tile(N, nb, active);
  if (tlog && m.rem == 0 && threadIdx.x == 0) tlog[m.k] = active ? active[m.k] : 1;
  if (!m.ok) return;
  const int64_t n = (int64_t)N * N;
  const Tx* xc = x + (int64_t)m.k * n;
  const Tb* bc = b + (int64_t)m.k * n;
  Tr* rc = r + (int64_t)m.k * n;
  const bool col_ok = m.x < N;
  const int xs = col_ok ? m.x : 0;
  // the wave's 64 lanes hold 64 consecutive columns: left and right neighbours
  // come from lane shifts, and only lanes 0 and 63 load their outer neighbour
  const int lane = threadIdx.x & 63;
  const int xe = lane == 0 ? m.x - 1 : m.x + 1;
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < N;
  Tx cx[MY + 2], ex[MY];
  Tb bb[MY];
#pragma unroll
  for (int j = 0; j < MY + 2; ++j) {
    const int yy = m.ybeg - 1 + j;
    cx[j] = ldz(xc, yy * N + xs, col_ok && yy >= 0 && yy < N && yy <= m.yend);
  }
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const bool ok = col_ok && yy < m.yend;
    ex[j] = ldz(xc, yy * N + (edge ? xe : 0), ok && edge);
    bb[j] = ldz(bc, yy * N + xs, ok);
  }
  double dre = 0.0, dim = 0.0;
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    // columns at or beyond N hold zeros, as the Dirichlet boundary needs
    const Tx sl = wave_shr1(cx[j + 1]), sr = wave_shl1(cx[j + 1]);
    const Tx lxj = lane == 0 ? ex[j] : sl, rxj = lane == 63 ? ex[j] : sr;
    const Tx ax = d * cx[j + 1] - c * (cx[j] + cx[j + 2] + lxj + rxj);
    const Tx v = convert<Tx, Tb>(bb[j]) - ax;
    if (col_ok && yy < m.yend) {
      rc[yy * N + m.x] = convert<Tr, Tx>(v);
      cdot_acc(dre, dim, v, v);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) {
      const int tiles = ((N + MX - 1) / MX) * ((N + MTY - 1) / MTY);
      partials[(int64_t)m.k * tiles + m.rem] = {dre, dim};
    }
  }
}

// Column-pair forms of the two marches above for even N: a lane holds two
// adjacent columns (one 8-byte load per row and vector in FP32, 16 bytes in
// FP64), a wave 128 columns.  The neighbour across the pair is the lane's own
// other column, the ones across lanes come from lane shifts, and only lanes 0
// and 63 load the column beyond the wave.  Every entry is formed by the same
// operations in the same order as in the one-column forms; only the grouping
// of the partial sums differs (tiles of 128 x 4*MY).
constexpr int PX = 128;

__device__ __forceinline__ MarchTile pair_tile(int N, int nb, const int* active) {
  const int nbx = (N + PX - 1) / PX, nby = (N + MTY - 1) / MTY;
  const int t = xcd_tile_index(nbx * nby * nb);
  MarchTile m;
  m.k = t / (nbx * nby);
  m.rem = t - m.k * nbx * nby;
  const int by = m.rem / nbx, bx = m.rem - by * nbx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  m.x = bx * PX + 2 * lane;  // even column of the lane's pair
  m.ybeg = by * MTY + w * MY;
  m.yend = m.ybeg + MY < N ? m.ybeg + MY : N;
  m.ok = m.k < nb && !(active && !active[m.k]);
  return m;
}

template <typename T, bool UPD>
__global__ __launch_bounds__(kThreads) void k_apply_pair(const T* __restrict__ x,
                                                         const T* __restrict__ z,
                                                         const c64* beta, T* __restrict__ xnew,
                                                         T* __restrict__ y, int N, R_t<T> d,
                                                         R_t<T> c, int nb, const int* active,
                                                         c64* partials, int* tlog) {
  __shared__ double red[16];
  const MarchTile m = pair_tile(N, nb, active);
  if (tlog && m.rem == 0 && threadIdx.x == 0) tlog[m.k] = active ? active[m.k] : 1;
  if (!m.ok) return;
  const int64_t n = (int64_t)N * N;
  const int half = N >> 1;
  const T* xs = x + (int64_t)m.k * n;
  const T* zs = z + (UPD ? (int64_t)m.k * n : 0);
  const Pair<T>* xc = reinterpret_cast<const Pair<T>*>(xs);
  const Pair<T>* zc = reinterpret_cast<const Pair<T>*>(zs);
  Pair<T>* xn = reinterpret_cast<Pair<T>*>(xnew + (UPD ? (int64_t)m.k * n : 0));
  Pair<T>* yc = reinterpret_cast<Pair<T>*>(y + (int64_t)m.k * n);
  const T zero = zero_of(T());
  double dre = 0.0, dim = 0.0;
  c64 bt = {0.0, 0.0};
  if (UPD) bt = beta[m.k];
  const bool col_ok = m.x < N;
  const int px = col_ok ? (m.x >> 1) : 0;
  const int lane = threadIdx.x & 63;
  Pair<T> cz[MY + 2], cx[MY + 2];
  T ez[MY], ex[MY];
#pragma unroll
  for (int j = 0; j < MY + 2; ++j) {
    const int yy = m.ybeg - 1 + j;
    const bool ok = col_ok && yy >= 0 && yy < N && yy <= m.yend;
    const Pair<T> a = xc[ok ? yy * half + px : 0];
    cx[j] = ok ? a : Pair<T>{zero, zero};
    if (UPD) {
      const Pair<T> q = zc[ok ? yy * half + px : 0];
      cz[j] = ok ? q : Pair<T>{zero, zero};
    } else {
      cz[j] = Pair<T>{zero, zero};
    }
  }
  const int xe = lane == 0 ? m.x - 1 : m.x + 2;  // edge lanes' outer column
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < N;
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const bool ok = edge && yy < m.yend;
    ex[j] = ldz(xs, yy * N + xe, ok);
    ez[j] = UPD ? ldz(zs, yy * N + xe, ok) : zero;
  }
  auto P = [&](T zz, T xx) -> T { return UPD ? zz + scale_by(bt.re, bt.im, xx) : xx; };
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const T m0 = P(cz[j + 1].e0, cx[j + 1].e0), m1 = P(cz[j + 1].e1, cx[j + 1].e1);
    const T pe = P(ez[j], ex[j]);
    const T sl = wave_shr1(m1), sr = wave_shl1(m0);
    const T left = lane == 0 ? pe : sl;    // column x - 1
    const T right = lane == 63 ? pe : sr;  // column x + 2
    const T v0 = d * m0 - c * (P(cz[j].e0, cx[j].e0) + P(cz[j + 2].e0, cx[j + 2].e0) + left + m1);
    const T v1 = d * m1 - c * (P(cz[j].e1, cx[j].e1) + P(cz[j + 2].e1, cx[j + 2].e1) + m0 + right);
    if (col_ok && yy < m.yend) {
      yc[yy * half + px] = Pair<T>{v0, v1};
      if (UPD) xn[yy * half + px] = Pair<T>{m0, m1};
      cdot_acc(dre, dim, m0, v0);
      cdot_acc(dre, dim, m1, v1);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) {
      const int tiles = ((N + PX - 1) / PX) * ((N + MTY - 1) / MTY);
      partials[(int64_t)m.k * tiles + m.rem] = {dre, dim};
    }
  }
}

template <typename Tb, typename Tx, typename Tr>
__global__ __launch_bounds__(kThreads) void k_residual_pair(const Tb* __restrict__ b,
                                                            const Tx* __restrict__ x,
                                                            Tr* __restrict__ r, int N,
                                                            R_t<Tx> d, R_t<Tx> c, int nb,
                                                            const int* active, c64* partials,
                                                            int* tlog) {
  __shared__ double red[16];
  const MarchTile m = pair_tile(N, nb, active);
  if (tlog && m.rem == 0 && threadIdx.x == 0) tlog[m.k] = active ? active[m.k] : 1;
  if (!m.ok) return;
  const int64_t n = (int64_t)N * N;
  const int half = N >> 1;
  const Tx* xs = x + (int64_t)m.k * n;
  const Pair<Tx>* xc = reinterpret_cast<const Pair<Tx>*>(xs);
  const Pair<Tb>* bc = reinterpret_cast<const Pair<Tb>*>(b + (int64_t)m.k * n);
  Pair<Tr>* rc = reinterpret_cast<Pair<Tr>*>(r + (int64_t)m.k * n);
  const bool col_ok = m.x < N;
  const int px = col_ok ? (m.x >> 1) : 0;
  const int lane = threadIdx.x & 63;
  const int xe = lane == 0 ? m.x - 1 : m.x + 2;
  const bool edge = (lane == 0 || lane == 63) && xe >= 0 && xe < N;
  const Tx zx = zero_of(Tx());
  const Tb zb = zero_of(Tb());
  Pair<Tx> cx[MY + 2];
  Tx ex[MY];
  Pair<Tb> bb[MY];
#pragma unroll
  for (int j = 0; j < MY + 2; ++j) {
    const int yy = m.ybeg - 1 + j;
    const bool ok = col_ok && yy >= 0 && yy < N && yy <= m.yend;
    const Pair<Tx> a = xc[ok ? yy * half + px : 0];
    cx[j] = ok ? a : Pair<Tx>{zx, zx};
  }
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const bool ok = col_ok && yy < m.yend;
    ex[j] = ldz(xs, yy * N + (edge ? xe : 0), ok && edge);
    const Pair<Tb> q = bc[ok ? yy * half + px : 0];
    bb[j] = ok ? q : Pair<Tb>{zb, zb};
  }
  double dre = 0.0, dim = 0.0;
#pragma unroll
  for (int j = 0; j < MY; ++j) {
    const int yy = m.ybeg + j;
    const Tx sl = wave_shr1(cx[j + 1].e1), sr = wave_shl1(cx[j + 1].e0);
    const Tx l0 = lane == 0 ? ex[j] : sl, r1 = lane == 63 ? ex[j] : sr;
    const Tx a0 = d * cx[j + 1].e0 - c * (cx[j].e0 + cx[j + 2].e0 + l0 + cx[j + 1].e1);
    const Tx a1 = d * cx[j + 1].e1 - c * (cx[j].e1 + cx[j + 2].e1 + cx[j + 1].e0 + r1);
    const Tx v0 = convert<Tx, Tb>(bb[j].e0) - a0;
    const Tx v1 = convert<Tx, Tb>(bb[j].e1) - a1;
    if (col_ok && yy < m.yend) {
      rc[yy * half + px] = Pair<Tr>{convert<Tr, Tx>(v0), convert<Tr, Tx>(v1)};
      cdot_acc(dre, dim, v0, v0);
      cdot_acc(dre, dim, v1, v1);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) {
      const int tiles = ((N + PX - 1) / PX) * ((N + MTY - 1) / MTY);
      partials[(int64_t)m.k * tiles + m.rem] = {dre, dim};
    }
  }
}

// rc = R (b - A x): one thread per coarse column, RR coarse rows (2*RR fine
// rows); all loads of a thread are issued before the arithmetic
constexpr int RR = 4;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_res_restrict2(const T* __restrict__ b,
                                                            const T* __restrict__ x,
                                                            T* __restrict__ rc, int N,
                                                            R_t<T> d, R_t<T> c, int nb,
                                                            const int* active, int* tlog) {
  const int Nc = N >> 1;
  const MarchTile m = march_tile<RR>(Nc, nb, active);  // coarse-grid tiling
  if (tlog && m.rem == 0 && threadIdx.x == 0) tlog[m.k] = active ? active[m.k] : 1;
  if (!m.ok) return;
  const int64_t n = (int64_t)N * N, nc = (int64_t)Nc * Nc;
  const T* xc = x + (int64_t)m.k * n;
  const T* bc = b + (int64_t)m.k * n;
  T* out = rc + (int64_t)m.k * nc;
  // lanes of a wave are 64 consecutive coarse columns (128 fine columns); the
  // fine neighbours left of 2x and right of 2x+1 come from the neighbouring
  // lanes (DPP), the two edge lanes load the column beyond the wave.  No early
  // exit: every lane takes part in the lane shifts.
  const int lane = threadIdx.x & 63;
  const bool col_ok = m.x < Nc;
  const int fx = 2 * (col_ok ? m.x : 0);
  constexpr int FR = 2 * RR + 2;  // fine rows 2*ybeg-1 .. 2*ybeg+2*RR
  T x0[FR], x1[FR], xe[2 * RR], b0[2 * RR], b1[2 * RR];
  const int fy0 = 2 * m.ybeg - 1, fyend = 2 * m.yend;  // exclusive
#pragma unroll
  for (int j = 0; j < FR; ++j) {
    const int yy = fy0 + j;
    const bool ok = col_ok && yy >= 0 && yy < N && yy <= fyend;
    x0[j] = ldz(xc, yy * N + fx, ok);
    x1[j] = ldz(xc, yy * N + fx + 1, ok);
  }
  const int fe = lane == 0 ? fx - 1 : fx + 2;  // edge lanes' outer fine column
  const bool edge = col_ok && (lane == 0 || lane == 63) && fe >= 0 && fe < N;
#pragma unroll
  for (int j = 0; j < 2 * RR; ++j) {
    const int yy = 2 * m.ybeg + j;
    const bool ok = col_ok && yy < fyend;
    xe[j] = ldz(xc, yy * N + fe, ok && edge);
    b0[j] = ldz(bc, yy * N + fx, ok);
    b1[j] = ldz(bc, yy * N + fx + 1, ok);
  }
#pragma unroll
  for (int Yl = 0; Yl < RR; ++Yl) {
    T acc = zero_of(T());
#pragma unroll
    for (int dy = 0; dy < 2; ++dy) {
      const int j = 2 * Yl + dy;       // index into the 2*RR fine rows
      const int jc = j + 1;            // index into x0/x1 (offset by the upper row)
      const T sl = wave_shr1(x1[jc]), sr = wave_shl1(x0[jc]);
      const T xl = lane == 0 ? xe[j] : sl;    // fine column 2x-1
      const T xr = lane == 63 ? xe[j] : sr;   // fine column 2x+2
      // fine point (fx, row j): neighbours left xl, right x1, up/down x0
      acc += b0[j] - (d * x0[jc] - c * (xl + x1[jc] + x0[jc - 1] + x0[jc + 1]));
      // fine point (fx+1, row j): neighbours left x0, right xr, up/down x1
      acc += b1[j] - (d * x1[jc] - c * (x0[jc] + xr + x1[jc - 1] + x1[jc + 1]));
    }
    if (col_ok && m.ybeg + Yl < m.yend) out[(m.ybeg + Yl) * Nc + m.x] = (R_t<T>)0.5 * acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict2(const T* __restrict__ x,
                                                        T* __restrict__ xcoarse, int N, int nb,
                                                        const int* active) {
  const int Nc = N >> 1;
  const MarchTile m = march_tile(Nc, nb, active);
  if (!m.ok || m.x >= Nc) return;
  const int64_t n = (int64_t)N * N, nc = (int64_t)Nc * Nc;
  const T* xc = x + (int64_t)m.k * n;
  T* out = xcoarse + (int64_t)m.k * nc;
  for (int Y = m.ybeg; Y < m.yend; ++Y) {
    const int i0 = (2 * Y) * N + 2 * m.x;
    out[Y * Nc + m.x] = (R_t<T>)0.5 * (xc[i0] + xc[i0 + 1] + xc[i0 + N] + xc[i0 + N + 1]);
  }
}

// x = beta * x + (omega/2) e_c[aggregate]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_prolong2(const T* __restrict__ ec, T* __restrict__ x,
                                                       int N, R_t<T> wh, R_t<T> beta, int nb,
                                                       const int* active) {
  const MarchTile m = march_tile(N, nb, active);
  if (!m.ok || m.x >= N) return;
  const int Nc = N >> 1;
  const int64_t n = (int64_t)N * N, nc = (int64_t)Nc * Nc;
  const T* e = ec + (int64_t)m.k * nc;
  T* xcol = x + (int64_t)m.k * n;
  for (int yy = m.ybeg; yy < m.yend; ++yy) {
    const T v = wh * e[(yy >> 1) * Nc + (m.x >> 1)];
    const int i = yy * N + m.x;
    xcol[i] = (beta == (R_t<T>)0) ? v : beta * xcol[i] + v;
  }
}

template <typename T>
__global__ void k_dense_build(T* M, int N, R_t<T> d, R_t<T> c) {
  const int n = N * N;
  const int64_t ld = 2 * (int64_t)n;
  const int i = blockIdx.y;
  const int yy = i / N, xx = i - yy * N;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int jy = j / N, jx = j - jy * N;
    T v = zero_of(T());
    if (j == i)
      v = d;
    else if ((jy == yy && (jx == xx - 1 || jx == xx + 1)) ||
             (jx == xx && (jy == yy - 1 || jy == yy + 1)))
      v = -c;
    M[(int64_t)i * ld + j] = v;
  }
}

inline int march_blocks(int N, int nb, int ry = MY) {
  const int nbx = (N + MX - 1) / MX, nby = (N + MW * ry - 1) / (MW * ry);
  return nbx * nby * nb;
}

}  // namespace

// the column-pair forms serve every even side from 64 up
inline bool pair_march(int N) { return (N & 1) == 0 && N >= 64; }
int poisson_march_tiles(int N) {
  const int cols = pair_march(N) ? PX : MX;
  return ((N + cols - 1) / cols) * ((N + MTY - 1) / MTY);
}
inline int pair_blocks(int N, int nb) {
  return ((N + PX - 1) / PX) * ((N + MTY - 1) / MTY) * nb;
}
// partial sums per column of the fused sweep: blocks of 4 column-marching waves
// for N >= 64, LDS tiles below
template <typename T>
int poisson_gs_tiles(int N, int rows, int sweeps) {
  if (N >= 64) {
    const int cols = sweeps == 2 ? SCOLS2 : SCOLS;
    const int units = ((N + cols - 1) / cols) * ((N + rows - 1) / rows);
    return (units + 3) / 4;
  }
  return ((N + GTX - 1) / GTX) * ((N + GTY - 1) / GTY);
}
template int poisson_gs_tiles<float>(int, int, int);
template int poisson_gs_tiles<double>(int, int, int);

template <> void gs_rows_options<float>(int out[3]) { out[0] = 8; out[1] = 16; out[2] = 32; }
template <> void gs_rows_options<double>(int out[3]) { out[0] = 4; out[1] = 8; out[2] = 16; }

template <typename T>
void poisson_dense_build(T* aug, int N, double d, double c, hipStream_t s) {
  const int n = N * N;
  MLMC_LAUNCH(k_dense_build<T>, dim3((unsigned)((n + 255) / 256), (unsigned)n),
                     dim3(256), 0, s, aug, N, (R_t<T>)d, (R_t<T>)c);
}

template <typename T>
void poisson_apply(const T* x, T* y, int N, double d, double c, int nb, const int* active,
                   c64* partials, hipStream_t s) {
  if (pair_march(N))
    MLMC_LAUNCH((k_apply_pair<T, false>), dim3(pair_blocks(N, nb)), dim3(kThreads), 0, s, x, x,
                (const c64*)nullptr, y, y, N, (R_t<T>)d, (R_t<T>)c, nb, active, partials,
                timing_log());
  else
    MLMC_LAUNCH((k_apply_march<T, false>), dim3(march_blocks(N, nb)), dim3(kThreads), 0, s, x,
                x, (const c64*)nullptr, y, y, N, (R_t<T>)d, (R_t<T>)c, nb, active, partials,
                timing_log());
}

template <typename T>
void poisson_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q, int N,
                          double d, double c, int nb, const int* active, c64* partials,
                          hipStream_t s) {
  if (pair_march(N))
    MLMC_LAUNCH((k_apply_pair<T, true>), dim3(pair_blocks(N, nb)), dim3(kThreads), 0, s, p_old,
                z, beta, p_new, q, N, (R_t<T>)d, (R_t<T>)c, nb, active, partials, timing_log());
  else
    MLMC_LAUNCH((k_apply_march<T, true>), dim3(march_blocks(N, nb)), dim3(kThreads), 0, s,
                p_old, z, beta, p_new, q, N, (R_t<T>)d, (R_t<T>)c, nb, active, partials,
                timing_log());
}

template <typename Tb, typename Tx, typename Tr>
void poisson_residual(const Tb* b, const Tx* x, Tr* r, int N, double d, double c, int nb,
                      const int* active, c64* partials, hipStream_t s) {
  if (pair_march(N))
    MLMC_LAUNCH((k_residual_pair<Tb, Tx, Tr>), dim3(pair_blocks(N, nb)), dim3(kThreads), 0, s,
                b, x, r, N, (R_t<Tx>)d, (R_t<Tx>)c, nb, active, partials, timing_log());
  else
    MLMC_LAUNCH((k_residual_march<Tb, Tx, Tr>), dim3(march_blocks(N, nb)), dim3(kThreads), 0, s,
                b, x, r, N, (R_t<Tx>)d, (R_t<Tx>)c, nb, active, partials, timing_log());
}

template <typename T, int SR, int NSW>
static void rbgs_march_launch(const T* xin, const T* b, T* xout, const T* ec, double omega, int N,
                              double d, double c, int nb, const int* active, bool reverse,
                              c64* partials, T* rc, hipStream_t s) {
  const R_t<T> wh = (R_t<T>)(0.5 * omega), di = (R_t<T>)(1.0 / d), cc = (R_t<T>)c;
  const R_t<T> dd = (R_t<T>)d;
  const int f = reverse ? 1 : 0;
  // null pointers are replaced by b (valid, never read) for the templated forms
  const T* xp = xin ? xin : b;
  const T* ep = ec ? ec : b;
  const dim3 blk(kThreads);
  if constexpr (NSW == 2) {
    if (rc) {
      // last pre-smoothing pass: forward colour order, no coarse correction
      if (ec || reverse) throw Error(MLMC_EINVAL, "restricted residual only on a pre-pass");
      const int nwx = (N + rbgs2_cols<true>() - 1) / rbgs2_cols<true>();
      const dim3 g(((nwx * ((N + SR - 1) / SR) + 3) / 4) * nb);
      if (xin)
        MLMC_LAUNCH((k_rbgs2_march<T, true, false, SR, 0, true>), g, blk, 0, s, xp, b, xout, ep,
                    wh, N, di, dd, cc, nb, active, partials, rc, timing_log());
      else
        MLMC_LAUNCH((k_rbgs2_march<T, false, false, SR, 0, true>), g, blk, 0, s, xp, b, xout, ep,
                    wh, N, di, dd, cc, nb, active, partials, rc, timing_log());
      return;
    }
  }
  const dim3 g(poisson_gs_tiles<T>(N, SR, NSW) * nb);
#define MLMC_RBGS_LAUNCH(HX, HE)                                                            \
  do {                                                                                      \
    if constexpr (NSW == 2) {                                                               \
      if (f)                                                                                \
        MLMC_LAUNCH((k_rbgs2_march<T, HX, HE, SR, 1, false>), g, blk, 0, s, xp, b, xout, ep, \
                    wh, N, di, dd, cc, nb, active, partials, (T*)nullptr, timing_log());    \
      else                                                                                  \
        MLMC_LAUNCH((k_rbgs2_march<T, HX, HE, SR, 0, false>), g, blk, 0, s, xp, b, xout, ep, \
                    wh, N, di, dd, cc, nb, active, partials, (T*)nullptr, timing_log());    \
    } else                                                                                  \
      MLMC_LAUNCH((k_rbgs_march<T, HX, HE, SR>), g, blk, 0, s, xp, b, xout, ep, wh, N, di,   \
                  cc, f, nb, active, partials, timing_log());                               \
  } while (0)
  if (xin && ec)
    MLMC_RBGS_LAUNCH(true, true);
  else if (xin)
    MLMC_RBGS_LAUNCH(true, false);
  else if (ec)
    MLMC_RBGS_LAUNCH(false, true);
  else
    MLMC_RBGS_LAUNCH(false, false);
#undef MLMC_RBGS_LAUNCH
}

template <typename T, int NSW>
static void rbgs_march_rows(const T* xin, const T* b, T* xout, const T* ec, double omega, int N,
                            double d, double c, int nb, const int* active, bool reverse,
                            c64* partials, T* rc, int rows, hipStream_t s) {
  int opts[3];
  gs_rows_options<T>(opts);
  if (rows == opts[0])
    rbgs_march_launch<T, (sizeof(T) == 4 ? 8 : 4), NSW>(xin, b, xout, ec, omega, N, d, c, nb,
                                                        active, reverse, partials, rc, s);
  else if (rows == opts[1])
    rbgs_march_launch<T, (sizeof(T) == 4 ? 16 : 8), NSW>(xin, b, xout, ec, omega, N, d, c, nb,
                                                         active, reverse, partials, rc, s);
  else if (rows == opts[2])
    rbgs_march_launch<T, (sizeof(T) == 4 ? 32 : 16), NSW>(xin, b, xout, ec, omega, N, d, c, nb,
                                                          active, reverse, partials, rc, s);
  else
    throw Error(MLMC_EINVAL, "unsupported rows per Gauss-Seidel segment");
}

template <typename T>
void poisson_rbgs_fused(const T* xin, const T* b, T* xout, const T* ec, double omega, int N,
                        double d, double c, int nb, const int* active, bool reverse,
                        c64* partials, int rows, int sweeps, hipStream_t s) {
  if (sweeps != 1 && sweeps != 2) throw Error(MLMC_EINVAL, "a fused pass holds 1 or 2 sweeps");
  if (N >= 64) {
    if (sweeps == 2 && (N & 1)) throw Error(MLMC_EINVAL, "two fused sweeps need an even side");
    if (sweeps == 2)
      rbgs_march_rows<T, 2>(xin, b, xout, ec, omega, N, d, c, nb, active, reverse, partials,
                            (T*)nullptr, rows, s);
    else
      rbgs_march_rows<T, 1>(xin, b, xout, ec, omega, N, d, c, nb, active, reverse, partials,
                            (T*)nullptr, rows, s);
  } else {
    if (sweeps != 1) throw Error(MLMC_EINVAL, "two fused sweeps need a side of at least 64");
    const int nbx = (N + GTX - 1) / GTX, nby = (N + GTY - 1) / GTY;
    MLMC_LAUNCH(k_rbgs_tile<T>, dim3(nbx * nby * nb), dim3(kThreads), 0, s, xin, b,
                       xout, ec, (R_t<T>)(0.5 * omega), N, (R_t<T>)(1.0 / d), (R_t<T>)c,
                       reverse ? 1 : 0, nbx, nby, nb, active, partials, timing_log());
  }
}

template <typename T>
void poisson_rbgs_restrict(const T* xin, const T* b, T* xout, T* rc, int N, double d, double c,
                           int nb, const int* active, int rows, hipStream_t s) {
  if (N < 64 || (N & 1)) throw Error(MLMC_EINVAL, "fused pre-pass needs an even side >= 64");
  rbgs_march_rows<T, 2>(xin, b, xout, (const T*)nullptr, 0.0, N, d, c, nb, active, false,
                        (c64*)nullptr, rc, rows, s);
}

template <typename T>
void poisson_residual_restrict(const T* b, const T* x, T* rc, int N, double d, double c,
                               int nb, const int* active, hipStream_t s) {
  MLMC_LAUNCH(k_res_restrict2<T>, dim3(march_blocks(N / 2, nb, RR)), dim3(kThreads), 0, s,
                     b, x, rc, N, (R_t<T>)d, (R_t<T>)c, nb, active, timing_log());
}

template <typename T>
void agg2d_restrict(const T* x, T* xc, int N, int nb, const int* active, hipStream_t s) {
  MLMC_LAUNCH(k_restrict2<T>, dim3(march_blocks(N / 2, nb)), dim3(kThreads), 0, s, x,
                     xc, N, nb, active);
}

template <typename T>
void agg2d_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                   const int* active, hipStream_t s) {
  MLMC_LAUNCH(k_prolong2<T>, dim3(march_blocks(N, nb)), dim3(kThreads), 0, s, ec, x, N,
                     (R_t<T>)(0.5 * omega), (R_t<T>)beta, nb, active);
}

#define MLMC_INST_P(T)                                                                      \
  template void poisson_dense_build<T>(T*, int, double, double, hipStream_t);              \
  template void poisson_apply<T>(const T*, T*, int, double, double, int, const int*, c64*,  \
                                 hipStream_t);                                             \
  template void poisson_update_apply<T>(const T*, const T*, const c64*, T*, T*, int, double, \
                                        double, int, const int*, c64*, hipStream_t);       \
  template void poisson_rbgs_fused<T>(const T*, const T*, T*, const T*, double, int,       \
                                      double, double, int, const int*, bool, c64*, int,    \
                                      int, hipStream_t);                                   \
  template void poisson_rbgs_restrict<T>(const T*, const T*, T*, T*, int, double, double,  \
                                         int, const int*, int, hipStream_t);               \
  template void poisson_residual_restrict<T>(const T*, const T*, T*, int, double, double,  \
                                             int, const int*, hipStream_t);                \
  template void agg2d_restrict<T>(const T*, T*, int, int, const int*, hipStream_t);        \
  template void agg2d_prolong<T>(const T*, T*, int, double, double, int, const int*,       \
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
template void poisson_residual<float, double, float>(const float*, const double*, float*, int,
                                                     double, double, int, const int*, c64*,
                                                     hipStream_t);

}  // namespace mlmc
