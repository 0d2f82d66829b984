// Device bodies of the 3D 7-point variable-coefficient stencil kernels.  Each
// body takes its block index (and, where a workgroup runs more than one block,
// its thread index) as arguments, so that the one-problem launches and the
// grouped and persistent launches over several problems run the same
// operations in the same order and give identical results.
#pragma once

#include "common.h"
#include "lanes.h"

namespace mlmc {
namespace vcb {

template <typename T> using R_t = typename Traits<T>::real;
constexpr int kNT = 256;  // threads of a (virtual) block of the cell-parallel bodies

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

// wave sums, then the waves' sums in wave order by thread 0 (the kernels'
// block_sum2 for blocks of kNT threads)
__device__ __forceinline__ void bsum2(double& a, double& b, double* lds) {
  block_sum2<kNT>(a, b, lds);
}

// r = b - A x (or r = A x when b is null); partials: per column and block of
// |r|^2 (or conj(x)^T r).  Block (bx, by) of a grid with nblk blocks of kNT
// cells; COLS columns from by * COLS.
template <typename Tb, typename T, typename Tr, int COLS>
__device__ __forceinline__ void vc_residual(const Tb* __restrict__ b, const T* __restrict__ x,
                                            Tr* __restrict__ r, const R_t<T>* __restrict__ kl,
                                            const R_t<T>* __restrict__ dg, int N, int nb,
                                            const int* active, c64* partials, int* tlog, int bx,
                                            int by, int nblk, double* red) {
  const int col0 = by * COLS;
  if (tlog && bx == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int64_t n = (int64_t)N * N * N;
  const int64_t i = (int64_t)bx * kNT + threadIdx.x;
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
      bsum2(dre, dim, red);
      if (threadIdx.x == 0) partials[(int64_t)col * nblk + bx] = {dre, dim};
    }
  }
}

// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q.  The
// neighbours' p_new values are recomputed from z and p_old, so the update and
// the operator need a single pass.  Block (bx, by) as in vc_residual.
template <typename T, int COLS>
__device__ __forceinline__ void vc_update_apply(const T* __restrict__ p_old,
                                                const T* __restrict__ z,
                                                const c64* __restrict__ beta,
                                                T* __restrict__ p_new, T* __restrict__ q,
                                                const R_t<T>* __restrict__ kl,
                                                const R_t<T>* __restrict__ dg, int N, int nb,
                                                const int* active, c64* partials, int* tlog,
                                                int bx, int by, int nblk, double* red) {
  const int col0 = by * COLS;
  if (tlog && bx == 0 && threadIdx.x < COLS && col0 + (int)threadIdx.x < nb)
    tlog[col0 + threadIdx.x] = active ? active[col0 + threadIdx.x] : 1;
  const int64_t n = (int64_t)N * N * N;
  const int64_t i = (int64_t)bx * kNT + threadIdx.x;
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
    bsum2(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)col * nblk + bx] = {dre, dim};
  }
}

// rc = R (b - A x) for 2x2x2 aggregates (1/sqrt(8)): coarse cell
// I = bx * NT + tid (a thread per coarse cell, no barrier), COLS columns from
// by * COLS
template <typename T, int COLS, int NT>
__device__ __forceinline__ void vc_res_restrict(const T* __restrict__ b, const T* __restrict__ x,
                                                T* __restrict__ rc,
                                                const R_t<T>* __restrict__ kl,
                                                const R_t<T>* __restrict__ dg, int N, int nb,
                                                const int* active, int* tlog, int bx, int by,
                                                int tid) {
  using R = R_t<T>;
  const int col0 = by * COLS;
  if (tlog && bx == 0 && tid < COLS && col0 + tid < nb)
    tlog[col0 + tid] = active ? active[col0 + tid] : 1;
  const int Nc = N >> 1;
  const int nc = Nc * Nc * Nc;
  const int I = bx * NT + tid;
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

// LDS elements of vc_march<T, COLS, RPW, ...>
template <typename T, int COLS, int RPW>
__host__ __device__ constexpr int vc_march_lds() {
  return 2 * 2 * (kMarchWaves * RPW) * COLS * (64 / RPW);
}

template <typename T, int COLS, int RPW, bool HX, bool HE, int F>
__device__ __forceinline__ void vc_march(const T* __restrict__ xin, const T* __restrict__ b,
                                         T* __restrict__ xout, const T* __restrict__ ec,
                                         R_t<T> ws, const R_t<T>* __restrict__ kl,
                                         const R_t<T>* __restrict__ dg, int N, int SZ, int nb,
                                         const int* active, int* tlog, int bx, int by, int bz,
                                         T* lds) {
  using R = R_t<T>;
  constexpr int RW = kMarchWaves * RPW;  // rows held, incl. one halo row each side
  constexpr int TY = RW - 2;             // rows owned
  constexpr int LPR = 64 / RPW;          // lanes (pairs) per row
  // a row's second-colour cell at plane p (x_in) and first-colour cell at
  // plane p-1 (updated): vc_march_lds<T, COLS, RPW>() elements of LDS
  T (*xa)[RW][COLS][LPR] = reinterpret_cast<T (*)[RW][COLS][LPR]>(lds);
  T (*xb)[RW][COLS][LPR] = reinterpret_cast<T (*)[RW][COLS][LPR]>(lds + 2 * RW * COLS * LPR);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int col0 = by * COLS;
  if (tlog && bx == 0 && bz == 0 && threadIdx.x < COLS &&
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
  const int y = bx * TY - 1 + r;
  // a row of the wave's parity (uniform; y has this parity in every lane)
  const int ybase = __builtin_amdgcn_readfirstlane((int)(bx * TY - 1 + (w & 1)));
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
  const int zs = bz * SZ;
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

}  // namespace vcb
}  // namespace mlmc
