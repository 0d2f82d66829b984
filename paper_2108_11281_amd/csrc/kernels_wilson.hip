// Kernels of the complex lattice operators:
//  * the Wilson-like 2-spin U(1) operator on an N x N periodic lattice,
//      D = (m0+2) I - 1/2 sum_mu [(I - s_mu) U_mu(x) d_{x+mu} + (I + s_mu) U_mu(x-mu)^* d_{x-mu}]
//    with s_1 = [[0,1],[1,0]], s_2 = [[0,i],[-i,0]] (Example 4.3, halved, m0 = m/2),
//    site s = y*N + x, unknown 2*s + spin;
//  * coarse operators of test-vector aggregation: 5-point block stencils with
//    dof x dof complex blocks per site and direction (0 self, 1 +x, 2 -x,
//    3 +y, 4 -y), site S = Y*Nc + X, unknown S*dof + j;
//  * the aggregation transfers: P maps a coarse site's dof_c coefficients to
//    the b x b fine sites of its aggregate through per-unknown rows q[i][j].
// Vectors are RHS-major blocks (column k of length n at k*n).
#include "kernels.h"

namespace mlmc {
namespace {

template <typename T> using R_t = typename Traits<T>::real;

__host__ __device__ __forceinline__ c32 mk(float re, float im) { return {re, im}; }
__host__ __device__ __forceinline__ c64 mk(double re, double im) { return {re, im}; }
template <typename T> __device__ __forceinline__ T times_i(T a) { return mk(-a.im, a.re); }
template <typename T> __device__ __forceinline__ T cmul_conj(T u, T a) {  // conj(u) * a
  return mk(u.re * a.re + u.im * a.im, u.re * a.im - u.im * a.re);
}

// hop term H x at a site (the sum in D = (m0+2) I - H/2), 2 spins, from the
// links u (+x: U_0(s), -x: U_0(s-x), +y: U_1(s), -y: U_1(s-y)) and the
// neighbours' spin pairs xp (s+x), xm (s-x), yp (s+y), ym (s-y)
template <typename T>
__device__ __forceinline__ void wilson_hop_sum(T upx, T xp0, T xp1, T umx, T xm0, T xm1, T upy,
                                               T yp0, T yp1, T umy, T ym0, T ym1, T& h0,
                                               T& h1) {
  // +x: (I - s1) U_0(s) x_{s+x}
  {
    const T a0 = upx * xp0, a1 = upx * xp1;
    h0 = a0 - a1;
    h1 = a1 - a0;
  }
  // -x: (I + s1) conj(U_0(s-x)) x_{s-x}
  {
    const T a0 = cmul_conj(umx, xm0), a1 = cmul_conj(umx, xm1);
    h0 += a0 + a1;
    h1 += a1 + a0;
  }
  // +y: (I - s2) U_1(s) x_{s+y};  (I - s2) v = (v0 - i v1, v1 + i v0)
  {
    const T a0 = upy * yp0, a1 = upy * yp1;
    h0 += a0 - times_i(a1);
    h1 += a1 + times_i(a0);
  }
  // -y: (I + s2) conj(U_1(s-y)) x_{s-y};  (I + s2) v = (v0 + i v1, v1 - i v0)
  {
    const T a0 = cmul_conj(umy, ym0), a1 = cmul_conj(umy, ym1);
    h0 += a0 + times_i(a1);
    h1 += a1 - times_i(a0);
  }
}

// hop term at site (sx, sy) with x read from the column's global vector
template <typename T>
__device__ __forceinline__ void wilson_hop(const T* __restrict__ x, const T* __restrict__ U, int N,
                                           int sx, int sy, T& h0, T& h1) {
  const int n2 = N * N;
  const int xp = sx + 1 == N ? 0 : sx + 1, xm = sx == 0 ? N - 1 : sx - 1;
  const int yp = sy + 1 == N ? 0 : sy + 1, ym = sy == 0 ? N - 1 : sy - 1;
  const int s = sy * N + sx;
  const int tpx = sy * N + xp, tmx = sy * N + xm, tpy = yp * N + sx, tmy = ym * N + sx;
  wilson_hop_sum(U[s], x[2 * tpx], x[2 * tpx + 1], U[tmx], x[2 * tmx], x[2 * tmx + 1],
                 U[n2 + s], x[2 * tpy], x[2 * tpy + 1], U[n2 + tmy], x[2 * tmy], x[2 * tmy + 1],
                 h0, h1);
}

// r = b - D x (or y = D x when b == nullptr); one thread per (site, column);
// optional partials of |r|^2 (or conj(x)^T y)
template <typename Tb, typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_wilson_residual(const Tb* __restrict__ b,
                                                              const T* __restrict__ x,
                                                              Tr* __restrict__ r,
                                                              const T* __restrict__ U, int N,
                                                              R_t<T> diag, const int* active,
                                                              c64* partials) {
  __shared__ double red[16];
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int n2 = N * N;
  const int s = blockIdx.x * kThreads + threadIdx.x;
  const int64_t off = (int64_t)k * 2 * n2;
  double dre = 0.0, dim = 0.0;
  if (s < n2) {
    const int sy = s / N, sx = s - sy * N;
    T h0, h1;
    wilson_hop(x + off, U, N, sx, sy, h0, h1);
    const T x0 = x[off + 2 * s], x1 = x[off + 2 * s + 1];
    const R_t<T> half = (R_t<T>)0.5;
    T v0 = diag * x0 - half * h0, v1 = diag * x1 - half * h1;
    if (b) {
      v0 = convert<T, Tb>(b[off + 2 * s]) - v0;
      v1 = convert<T, Tb>(b[off + 2 * s + 1]) - v1;
      cdot_acc(dre, dim, v0, v0);
      cdot_acc(dre, dim, v1, v1);
    } else {
      cdot_acc(dre, dim, x0, v0);
      cdot_acc(dre, dim, x1, v1);
    }
    r[off + 2 * s] = convert<Tr, T>(v0);
    r[off + 2 * s + 1] = convert<Tr, T>(v1);
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {dre, dim};
  }
}

// one colour of a red-black site Gauss-Seidel sweep: x_s = (b_s + H x / 2)/diag
template <typename T>
__global__ __launch_bounds__(kThreads) void k_wilson_gs(const T* __restrict__ b, T* __restrict__ x,
                                                        const T* __restrict__ U, int N,
                                                        R_t<T> dinv, int colour, int zero_nbrs,
                                                        const int* active, int* tlog) {
  const int k = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (active && !active[k]) return;
  const int n2 = N * N, half = N >> 1;
  // thread t takes the t-th site of the colour in row-major order (N even):
  // row sy holds the colour at sx = 2j + ((colour + sy) & 1)
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= (n2 >> 1)) return;
  const int sy = t / half;
  const int sx = 2 * (t - sy * half) + ((colour + sy) & 1);
  const int s = sy * N + sx;
  const int64_t off = (int64_t)k * 2 * n2;
  T v0 = b[off + 2 * s], v1 = b[off + 2 * s + 1];
  if (!zero_nbrs) {
    T h0, h1;
    wilson_hop(x + off, U, N, sx, sy, h0, h1);
    const R_t<T> half = (R_t<T>)0.5;
    v0 += half * h0;
    v1 += half * h1;
  }
  x[off + 2 * s] = dinv * v0;
  x[off + 2 * s + 1] = dinv * v1;
}

// both colours of one red-black site Gauss-Seidel sweep in a single pass, out
// of place (xin is not read when zero_init; otherwise xout != xin).  A block
// takes a TS x TS tile of one column: the second-colour values of the tile
// and of a two-site periodic halo go to LDS, the first colour is updated on
// the tile and on its one-site halo ring (a ring site gets the value its own
// tile computes: same inputs, same arithmetic), then the second colour on the
// tile.  x is read and written once per sweep instead of once per colour.
template <typename T, int TS>
__global__ __launch_bounds__(kThreads) void k_wilson_gs2(const T* __restrict__ b,
                                                         const T* __restrict__ xin,
                                                         T* __restrict__ xout,
                                                         const T* __restrict__ U, int N,
                                                         R_t<T> dinv, int first, int zero_init,
                                                         const int* active, int* tlog) {
  constexpr int W = TS + 4;  // tile + two halo sites each side
  __shared__ T xs[W * W * 2];
  const int k = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (active && !active[k]) return;
  const int tiles = N / TS;
  const int ox = (int)(blockIdx.x % tiles) * TS - 2, oy = (int)(blockIdx.x / tiles) * TS - 2;
  const int n2 = N * N;
  const int64_t off = (int64_t)k * 2 * n2;
  const int second = 1 - first;
  const R_t<T> half = (R_t<T>)0.5;
  // W-space (lx, ly) -> lattice site; ox, oy and N are even, so the colour
  // (lx + ly) & 1 is the lattice colour
  auto gx_of = [&](int lx) { int g = ox + lx; return g < 0 ? g + N : (g >= N ? g - N : g); };
  auto gy_of = [&](int ly) { int g = oy + ly; return g < 0 ? g + N : (g >= N ? g - N : g); };
  auto update = [&](int lx, int ly, bool nbrs, T& v0, T& v1) {
    const int gx = gx_of(lx), gy = gy_of(ly);
    const int sidx = gy * N + gx;
    v0 = b[off + 2 * sidx];
    v1 = b[off + 2 * sidx + 1];
    if (nbrs) {
      const int gxm = gx == 0 ? N - 1 : gx - 1, gym = gy == 0 ? N - 1 : gy - 1;
      const T* c = xs + 2 * (ly * W + lx);
      T h0, h1;
      wilson_hop_sum(U[sidx], c[2], c[3], U[gy * N + gxm], c[-2], c[-1], U[n2 + sidx],
                     c[2 * W], c[2 * W + 1], U[n2 + gym * N + gx], c[-2 * W], c[-2 * W + 1],
                     h0, h1);
      v0 += half * h0;
      v1 += half * h1;
    }
    v0 = dinv * v0;
    v1 = dinv * v1;
    return sidx;
  };
  if (!zero_init) {
    // second-colour sites of the whole W x W window
    for (int q = threadIdx.x; q < W * W / 2; q += kThreads) {
      const int ly = q / (W / 2);
      const int lx = 2 * (q - ly * (W / 2)) + ((second + ly) & 1);
      const int sidx = gy_of(ly) * N + gx_of(lx);
      xs[2 * (ly * W + lx)] = xin[off + 2 * sidx];
      xs[2 * (ly * W + lx) + 1] = xin[off + 2 * sidx + 1];
    }
    __syncthreads();
  }
  // first colour on the tile and its one-site ring: rows and columns 1 .. TS+2
  constexpr int E = TS + 2;
  for (int q = threadIdx.x; q < E * E / 2; q += kThreads) {
    const int ly = 1 + q / (E / 2);
    const int lx = 1 + 2 * (q - (ly - 1) * (E / 2)) + ((first + ly + 1) & 1);
    T v0, v1;
    const int sidx = update(lx, ly, !zero_init, v0, v1);
    xs[2 * (ly * W + lx)] = v0;
    xs[2 * (ly * W + lx) + 1] = v1;
    if (lx >= 2 && lx < TS + 2 && ly >= 2 && ly < TS + 2) {
      xout[off + 2 * sidx] = v0;
      xout[off + 2 * sidx + 1] = v1;
    }
  }
  __syncthreads();
  // second colour on the tile: rows and columns 2 .. TS+1
  for (int q = threadIdx.x; q < TS * TS / 2; q += kThreads) {
    const int ly = 2 + q / (TS / 2);
    const int lx = 2 + 2 * (q - (ly - 2) * (TS / 2)) + ((second + ly) & 1);
    T v0, v1;
    const int sidx = update(lx, ly, true, v0, v1);
    xout[off + 2 * sidx] = v0;
    xout[off + 2 * sidx + 1] = v1;
  }
}

// ---- 5-point block stencils (coarse operators) ------------------------------
// Lanes along right-hand sides: a wave serves one site at a time for 64
// consecutive columns.  The site, hence every stencil block, inverted
// diagonal block and aggregate basis row it reads, is uniform over the wave
// (read through the scalar data cache, shared by the 64 columns); each lane
// reads its own column's DOF contiguous values of a site.
__device__ __forceinline__ int nbr_site(int S, int d, int Nc) {
  const int Y = S / Nc, X = S - Y * Nc;
  switch (d) {
    case 1: return Y * Nc + (X + 1 == Nc ? 0 : X + 1);
    case 2: return Y * Nc + (X == 0 ? Nc - 1 : X - 1);
    case 3: return (Y + 1 == Nc ? 0 : Y + 1) * Nc + X;
    case 4: return (Y == 0 ? Nc - 1 : Y - 1) * Nc + X;
    default: return S;
  }
}

// the wave's index within the grid (uniform: every lane computes the same)
__device__ __forceinline__ int wave_index() {
  return __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)));
}

// acc -= B x (DOF x DOF block, row-major) or acc += B x
template <int DOF, typename T>
__device__ __forceinline__ void block_mac(T* acc, const T* __restrict__ blk, const T* xv,
                                          bool subtract) {
#pragma unroll
  for (int i = 0; i < DOF; ++i) {
    T v = zero_of(T());
#pragma unroll
    for (int j = 0; j < DOF; ++j) v += blk[i * DOF + j] * xv[j];
    acc[i] = subtract ? acc[i] - v : acc[i] + v;
  }
}

// r = b - A x (b == nullptr: r = A x); blocks [site][5][DOF][DOF]; a wave per
// site and 64 columns
template <int DOF, typename Tb, typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_bsr_residual(const Tb* __restrict__ b,
                                                           const T* __restrict__ x,
                                                           Tr* __restrict__ r,
                                                           const T* __restrict__ B, int Nc,
                                                           int nb, const int* active) {
  const int lane = threadIdx.x & 63;
  const int S = wave_index();
  const int k = blockIdx.y * 64 + lane;
  const int ns = Nc * Nc;
  if (S >= ns) return;
  if (k >= nb || (active && !active[k])) return;
  const int64_t off = (int64_t)k * ns * DOF;
  T acc[DOF];
#pragma unroll
  for (int i = 0; i < DOF; ++i) acc[i] = zero_of(T());
  // one neighbour's values live at a time
#pragma unroll 1
  for (int d = 0; d < 5; ++d) {
    const int t = nbr_site(S, d, Nc);
    T xv[DOF];
#pragma unroll
    for (int j = 0; j < DOF; ++j) xv[j] = x[off + (int64_t)t * DOF + j];
    block_mac<DOF>(acc, B + ((int64_t)S * 5 + d) * DOF * DOF, xv, false);
  }
#pragma unroll
  for (int i = 0; i < DOF; ++i) {
    T v = acc[i];
    if (b) v = convert<T, Tb>(b[off + (int64_t)S * DOF + i]) - v;
    r[off + (int64_t)S * DOF + i] = convert<Tr, T>(v);
  }
}

// one colour of a red-black block Gauss-Seidel sweep, in place:
// x_S = Dinv_S (b_S - sum_{d != self} B[S][d] x_nbr); a wave per site of the
// colour (Nc even: the j-th site of colour c in row Y is X = 2j + ((c+Y) & 1))
template <int DOF, typename T>
__global__ __launch_bounds__(kThreads) void k_bsr_gs(const T* __restrict__ b, T* __restrict__ x,
                                                     const T* __restrict__ B,
                                                     const T* __restrict__ Dinv, int Nc,
                                                     int colour, int zero_nbrs, int nb,
                                                     const int* active, int* tlog) {
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.y * 64 + lane;
  if (tlog && blockIdx.x == 0 && threadIdx.x < 64 && k < nb) tlog[k] = active ? active[k] : 1;
  const int t = wave_index();
  const int hc = Nc >> 1;
  if (t >= Nc * hc) return;
  if (k >= nb || (active && !active[k])) return;
  const int Y = t / hc, j = t - Y * hc;
  const int S = Y * Nc + 2 * j + ((colour + Y) & 1);
  const int64_t off = (int64_t)k * Nc * Nc * DOF;
  T rhs[DOF];
#pragma unroll
  for (int i = 0; i < DOF; ++i) rhs[i] = b[off + (int64_t)S * DOF + i];
  if (!zero_nbrs) {
#pragma unroll
    for (int d = 1; d < 5; ++d) {
      const int tn = nbr_site(S, d, Nc);
      T xv[DOF];
#pragma unroll
      for (int jj = 0; jj < DOF; ++jj) xv[jj] = x[off + (int64_t)tn * DOF + jj];
      block_mac<DOF>(rhs, B + ((int64_t)S * 5 + d) * DOF * DOF, xv, true);
    }
  }
  T out[DOF];
#pragma unroll
  for (int i = 0; i < DOF; ++i) out[i] = zero_of(T());
  block_mac<DOF>(out, Dinv + (int64_t)S * DOF * DOF, rhs, false);
#pragma unroll
  for (int i = 0; i < DOF; ++i) x[off + (int64_t)S * DOF + i] = out[i];
}

// Thread-per-site forms: a thread serves one (site, column) and reads the
// site's blocks itself.  Which of the two forms is faster depends on the
// precision and the lattice (with complex128 blocks on large lattices the
// wave-uniform form waits on its scalar loads); the setup-time autotuner
// chooses per level.
// r = b - A x (b == nullptr: r = A x); one thread per (site, column) computing
// its DOF outputs; partial sums per column and block of kThreads sites
template <int DOF, typename Tb, typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_bsr_residual_sites(const Tb* __restrict__ b,
                                                           const T* __restrict__ x,
                                                           Tr* __restrict__ r,
                                                           const T* __restrict__ B, int Nc,
                                                           const int* active, c64* partials) {
  __shared__ double red[16];
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int ns = Nc * Nc;
  const int S = blockIdx.x * kThreads + threadIdx.x;
  const int64_t off = (int64_t)k * DOF * ns;
  double dre = 0.0, dim = 0.0;
  if (S < ns) {
    T acc[DOF];
#pragma unroll
    for (int i = 0; i < DOF; ++i) acc[i] = zero_of(T());
    for (int d = 0; d < 5; ++d) {
      const int t = nbr_site(S, d, Nc);
      const T* blk = B + ((int64_t)S * 5 + d) * DOF * DOF;
      T xv[DOF];
#pragma unroll
      for (int j = 0; j < DOF; ++j) xv[j] = x[off + (int64_t)t * DOF + j];
#pragma unroll
      for (int i = 0; i < DOF; ++i)
#pragma unroll
        for (int j = 0; j < DOF; ++j) acc[i] += blk[i * DOF + j] * xv[j];
    }
#pragma unroll
    for (int i = 0; i < DOF; ++i) {
      T v = acc[i];
      if (b) {
        v = convert<T, Tb>(b[off + (int64_t)S * DOF + i]) - v;
        cdot_acc(dre, dim, v, v);
      } else {
        cdot_acc(dre, dim, x[off + (int64_t)S * DOF + i], v);
      }
      r[off + (int64_t)S * DOF + i] = convert<Tr, T>(v);
    }
  }
  if (partials) {
    block_sum2<kThreads>(dre, dim, red);
    if (threadIdx.x == 0) partials[(int64_t)k * gridDim.x + blockIdx.x] = {dre, dim};
  }
}

// one colour of a red-black block Gauss-Seidel sweep:
// x_S = Dinv_S (b_S - sum_{d != self} B[S][d] x_nbr).  A group of G lanes
// (DOF rounded up to a power of two, so groups never straddle a wave) per
// site of the colour, lane i < DOF takes row i: its rows of the four
// neighbour blocks (contiguous across the group), then Dinv's row i against
// the group's right-hand sides gathered by lane shuffles
template <int DOF> constexpr int bsr_group() {
  return DOF <= 1 ? 1 : DOF <= 2 ? 2 : DOF <= 4 ? 4 : DOF <= 8 ? 8 : DOF <= 16 ? 16 : 32;
}
__device__ __forceinline__ c32 shfl_c(c32 v, int src) {
  return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}
__device__ __forceinline__ c64 shfl_c(c64 v, int src) {
  return {__shfl(v.re, src, 64), __shfl(v.im, src, 64)};
}

template <int DOF, typename T>
__global__ __launch_bounds__(kThreads) void k_bsr_gs_rows(const T* __restrict__ b, T* __restrict__ x,
                                                          const T* __restrict__ B,
                                                          const T* __restrict__ Dinv, int Nc,
                                                          int colour, int zero_nbrs,
                                                          const int* active, int* tlog) {
  constexpr int G = bsr_group<DOF>();
  const int k = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[k] = active ? active[k] : 1;
  if (active && !active[k]) return;
  const int ns = Nc * Nc, half = Nc >> 1;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  const int q = t / G, i = t % G;
  if (q >= (ns >> 1)) return;  // whole groups: G divides kThreads
  const int Y = q / half;
  const int S = Y * Nc + 2 * (q - Y * half) + ((colour + Y) & 1);
  const int64_t off = (int64_t)k * DOF * ns;
  const bool row = i < DOF;
  T rhs = zero_of(T());
  if (row) {
    rhs = b[off + (int64_t)S * DOF + i];
    if (!zero_nbrs) {
      for (int d = 1; d < 5; ++d) {
        const int tn = nbr_site(S, d, Nc);
        const T* blk = B + (((int64_t)S * 5 + d) * DOF + i) * DOF;
        const T* xv = x + off + (int64_t)tn * DOF;
#pragma unroll
        for (int j = 0; j < DOF; ++j) rhs -= blk[j] * xv[j];
      }
    }
  }
  const int lane0 = (int)(threadIdx.x & 63) - i;
  const T* di = Dinv + ((int64_t)S * DOF + (row ? i : 0)) * DOF;
  T v = zero_of(T());
#pragma unroll
  for (int j = 0; j < DOF; ++j) {
    const T rj = shfl_c(rhs, lane0 + j);
    if (row) v += di[j] * rj;
  }
  if (row) x[off + (int64_t)S * DOF + i] = v;
}

// r = b - A x (b == nullptr: r = A x) without partial sums: a group of lanes
// per site, one block row per lane, as in the sweep
template <int DOF, typename Tb, typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_bsr_residual_rows(const Tb* __restrict__ b,
                                                                const T* __restrict__ x,
                                                                Tr* __restrict__ r,
                                                                const T* __restrict__ B, int Nc,
                                                                const int* active) {
  constexpr int G = bsr_group<DOF>();
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int ns = Nc * Nc;
  const int t = blockIdx.x * kThreads + threadIdx.x;
  const int S = t / G, i = t % G;
  if (S >= ns || i >= DOF) return;
  const int64_t off = (int64_t)k * DOF * ns;
  T acc = zero_of(T());
  for (int d = 0; d < 5; ++d) {
    const int tn = nbr_site(S, d, Nc);
    const T* blk = B + (((int64_t)S * 5 + d) * DOF + i) * DOF;
    const T* xv = x + off + (int64_t)tn * DOF;
#pragma unroll
    for (int j = 0; j < DOF; ++j) acc += blk[j] * xv[j];
  }
  T v = acc;
  if (b) v = convert<T, Tb>(b[off + (int64_t)S * DOF + i]) - v;
  r[off + (int64_t)S * DOF + i] = convert<Tr, T>(v);
}

// ---- aggregation transfers --------------------------------------------------
// fine lattice Nf x Nf with dofF unknowns per site, aggregates of blk x blk
// sites, DOFC coarse unknowns per coarse site; q[i][j] (i fine unknown).

// xc = P^H x: a workgroup per (coarse site, 64 columns); its waves take the
// aggregate's rows in turn (the rows of q are uniform over a wave, each lane
// walks its column's blk*dofF contiguous fine values of a row), and the
// waves' shares are added in a fixed order through LDS
template <int DOFC, typename T>
__global__ __launch_bounds__(kThreads) void k_agg_restrict(const T* __restrict__ x,
                                                           T* __restrict__ xc,
                                                           const T* __restrict__ q, int Nf,
                                                           int dofF, int blk, int nb,
                                                           const int* active) {
  constexpr int W = kThreads / 64;
  __shared__ T part[W - 1][DOFC][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int k = blockIdx.y * 64 + lane;
  const int Nc = Nf / blk, nsc = Nc * Nc;
  const int S = blockIdx.x;
  const bool on = k < nb && (!active || active[k]);
  const int Y = S / Nc, X = S - Y * Nc;
  const int64_t nf = (int64_t)Nf * Nf * dofF;
  const T* xk = x + (int64_t)(on ? k : 0) * nf;
  const int wr = blk * dofF;  // contiguous fine unknowns per aggregate row
  T acc[DOFC];
#pragma unroll
  for (int j = 0; j < DOFC; ++j) acc[j] = zero_of(T());
  if (on) {
    for (int yy = w; yy < blk; yy += W) {
      const int64_t i0 = ((int64_t)(Y * blk + yy) * Nf + X * blk) * dofF;
      // unrolled so that several loads of x are in flight (same order of sums)
#pragma unroll 4
      for (int a = 0; a < wr; ++a) {
        const T v = xk[i0 + a];
        const T* qi = q + (i0 + a) * DOFC;
#pragma unroll
        for (int j = 0; j < DOFC; ++j) acc[j] += cmul_conj(qi[j], v);
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int j = 0; j < DOFC; ++j) part[w - 1][j][lane] = acc[j];
  }
  __syncthreads();
  if (w == 0 && on) {
#pragma unroll
    for (int v = 0; v < W - 1; ++v)
#pragma unroll
      for (int j = 0; j < DOFC; ++j) acc[j] += part[v][j][lane];
#pragma unroll
    for (int j = 0; j < DOFC; ++j) xc[(int64_t)k * nsc * DOFC + (int64_t)S * DOFC + j] = acc[j];
  }
}

// x = beta * x + omega * P xc ; one thread per (fine unknown, column): loads
// of x and of the rows of q are coalesced along the fine unknowns
template <int DOFC, typename T>
__global__ __launch_bounds__(kThreads) void k_agg_prolong(const T* __restrict__ xc, T* __restrict__ x,
                                                          const T* __restrict__ q, int Nf,
                                                          int dofF, int blk, R_t<T> omega,
                                                          R_t<T> beta, const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int Nc = Nf / blk;
  const int64_t nf = (int64_t)Nf * Nf * dofF;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nf) return;
  const int s = (int)(i / dofF);
  const int sy = s / Nf, sx = s - sy * Nf;
  const int S = (sy / blk) * Nc + (sx / blk);
  const T* e = xc + (int64_t)k * Nc * Nc * DOFC + (int64_t)S * DOFC;
  const T* qi = q + i * DOFC;
  T v = zero_of(T());
#pragma unroll
  for (int j = 0; j < DOFC; ++j) v += qi[j] * e[j];
  T* xk = x + (int64_t)k * nf;
  xk[i] = (beta == (R_t<T>)0) ? omega * v : beta * xk[i] + omega * v;
}

// ---- setup ---------------------------------------------------------------
__global__ void k_links(const double* theta, c64* U64, c32* U32, int n) {
  // n = 2 N^2 link phases
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double s, c;
    sincos(theta[i], &s, &c);
    U64[i] = {c, s};
    U32[i] = {(float)c, (float)s};
  }
}

// per-aggregate modified Gram-Schmidt of the nv test vectors restricted to the
// aggregate (FP64); V: [nv][n] (vector j at j*n), q out: [n][nq]; one block per
// aggregate, m = blk*blk*dofF rows.  split: the rows of each spin (a site's
// first dofF/2 unknowns carry spin 0) are orthonormalised on their own (the two
// row sets are disjoint, so both run in place in the same LDS copy); row r of
// spin p gets its basis in columns p*nv..p*nv+nv-1 and zeros in the others
// (nq = 2 nv); otherwise nq = nv.
__global__ __launch_bounds__(kThreads) void k_agg_orthonormalise(const c64* __restrict__ V,
                                                                 c64* __restrict__ q, int Nf,
                                                                 int dofF, int blk, int nv,
                                                                 int split) {
  extern __shared__ c64 sv[];  // m * nv
  __shared__ double red[16];
  const int Nc = Nf / blk;
  const int S = blockIdx.x;
  const int Y = S / Nc, X = S - Y * Nc;
  const int m = blk * blk * dofF;
  const int half = dofF / 2;
  const int64_t n = (int64_t)Nf * Nf * dofF;
  auto row_index = [&](int r) -> int64_t {
    const int site = r / dofF, a = r - site * dofF;
    const int yy = site / blk, xx = site - yy * blk;
    return (int64_t)((Y * blk + yy) * Nf + (X * blk + xx)) * dofF + a;
  };
  // spin of row r (0 for every row without the split)
  auto spin = [&](int r) { return split ? (r % dofF) / half : 0; };
  for (int idx = threadIdx.x; idx < m * nv; idx += kThreads) {
    const int r = idx / nv, j = idx - r * nv;
    sv[idx] = V[(int64_t)j * n + row_index(r)];
  }
  __syncthreads();
  for (int p = 0; p < (split ? 2 : 1); ++p) {
    for (int j = 0; j < nv; ++j) {
      // remove the components along the previous (already normalised) columns
      for (int i = 0; i < j; ++i) {
        double re = 0.0, im = 0.0;
        for (int r = threadIdx.x; r < m; r += kThreads)
          if (spin(r) == p) cdot_acc(re, im, sv[r * nv + i], sv[r * nv + j]);
        block_sum2<kThreads>(re, im, red);
        __shared__ double proj[2];
        if (threadIdx.x == 0) {
          proj[0] = re;
          proj[1] = im;
        }
        __syncthreads();
        const c64 h = {proj[0], proj[1]};
        for (int r = threadIdx.x; r < m; r += kThreads)
          if (spin(r) == p) sv[r * nv + j] -= h * sv[r * nv + i];
        __syncthreads();
      }
      double re = 0.0, im = 0.0;
      for (int r = threadIdx.x; r < m; r += kThreads)
        if (spin(r) == p) cdot_acc(re, im, sv[r * nv + j], sv[r * nv + j]);
      block_sum2<kThreads>(re, im, red);
      __shared__ double nrm;
      if (threadIdx.x == 0) nrm = sqrt(re);
      __syncthreads();
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int r = threadIdx.x; r < m; r += kThreads)
        if (spin(r) == p) sv[r * nv + j] = inv * sv[r * nv + j];
      __syncthreads();
    }
  }
  const int nq = split ? 2 * nv : nv;
  for (int idx = threadIdx.x; idx < m * nq; idx += kThreads) {
    const int r = idx / nq, c = idx - r * nq;
    const int p = c / nv, j = c - p * nv;  // p = 0 without the split
    q[row_index(r) * nq + c] = (spin(r) == p) ? sv[r * nv + j] : c64{0.0, 0.0};
  }
}

// gauge Laplacian (Example 4.2) as a 1 x 1 block stencil: B[s][0] = diag,
// B[s][1] = -U_0(s) (+x), B[s][2] = -conj(U_0(s-x)), B[s][3] = -U_1(s) (+y),
// B[s][4] = -conj(U_1(s-y)); U [2][N][N] (mu, y, x); a thread per site
__global__ __launch_bounds__(kThreads) void k_gauge_blocks(const c64* __restrict__ U, int N,
                                                           double diag, c64* __restrict__ B) {
  const int s = blockIdx.x * kThreads + threadIdx.x;
  if (s >= N * N) return;
  const int n2 = N * N;
  const int sy = s / N, sx = s - sy * N;
  const int tx = sy * N + (sx == 0 ? N - 1 : sx - 1);
  const int ty = (sy == 0 ? N - 1 : sy - 1) * N + sx;
  c64* b = B + (int64_t)s * 5;
  b[0] = {diag, 0.0};
  b[1] = {-U[s].re, -U[s].im};
  b[2] = {-U[tx].re, U[tx].im};
  b[3] = {-U[n2 + s].re, -U[n2 + s].im};
  b[4] = {-U[n2 + ty].re, U[n2 + ty].im};
}

// Galerkin blocks of the coarse operator, labelled by hop direction.
// Fine operator given as a block stencil (blocks Bf [site][5][dofF][dofF]) or,
// when Bf == nullptr, as the Wilson operator (links U, diagonal wdiag).
// One block per (coarse site S, direction d); output Bc[S][d][nv][nv].
// A fine hop from site s (in S) in direction d lands in the self block of S if
// the neighbour stays inside the aggregate without wrapping, otherwise in
// block d (whose coarse neighbour is nbr_site(S, d)).
__device__ __forceinline__ void fine_hop_target(int sx, int sy, int d, int Nf, int& tx, int& ty) {
  tx = sx;
  ty = sy;
  if (d == 1) tx = sx + 1 == Nf ? 0 : sx + 1;
  if (d == 2) tx = sx == 0 ? Nf - 1 : sx - 1;
  if (d == 3) ty = sy + 1 == Nf ? 0 : sy + 1;
  if (d == 4) ty = sy == 0 ? Nf - 1 : sy - 1;
}

// fine block (dofF x dofF) coupling site s to its neighbour in direction d
__device__ __forceinline__ c64 fine_coupling(const c64* Bf, const c64* U, double wdiag, int Nf,
                                             int dofF, int s, int d, int a, int bcol) {
  if (Bf) return Bf[((int64_t)s * 5 + d) * dofF * dofF + a * dofF + bcol];
  // Wilson: dofF = 2
  const int n2 = Nf * Nf;
  const int sy = s / Nf, sx = s - sy * Nf;
  if (d == 0) return {a == bcol ? wdiag : 0.0, 0.0};
  // -1/2 (I -+ s_mu) u with u the link factor of the hop
  c64 u;
  int t;
  if (d == 1) u = U[s];
  else if (d == 2) {
    t = sy * Nf + (sx == 0 ? Nf - 1 : sx - 1);
    u = {U[t].re, -U[t].im};
  } else if (d == 3) u = U[n2 + s];
  else {
    t = (sy == 0 ? Nf - 1 : sy - 1) * Nf + sx;
    u = {U[n2 + t].re, -U[n2 + t].im};
  }
  // spin matrices: d=1: I - s1 = [[1,-1],[-1,1]]; d=2: I + s1 = [[1,1],[1,1]];
  // d=3: I - s2 = [[1,-i],[i,1]]; d=4: I + s2 = [[1,i],[-i,1]]
  c64 m = {0.0, 0.0};
  if (a == bcol) m = {1.0, 0.0};
  else if (d == 1) m = {-1.0, 0.0};
  else if (d == 2) m = {1.0, 0.0};
  else if (d == 3) m = (a == 0) ? c64{0.0, -1.0} : c64{0.0, 1.0};
  else m = (a == 0) ? c64{0.0, 1.0} : c64{0.0, -1.0};
  return -0.5 * (m * u);
}

__global__ __launch_bounds__(kThreads) void k_galerkin(const c64* __restrict__ Bf,
                                                       const c64* __restrict__ U, double wdiag,
                                                       const c64* __restrict__ q, int Nf,
                                                       int dofF, int blk, int nv,
                                                       c64* __restrict__ Bc) {
  const int Nc = Nf / blk;
  const int S = blockIdx.x, dc = blockIdx.y;
  const int Y = S / Nc, X = S - Y * Nc;
  // each thread accumulates some (i, j) entries of the nv x nv output block
  for (int e = threadIdx.x; e < nv * nv; e += kThreads) {
    const int i = e / nv, j = e - i * nv;
    double re = 0.0, im = 0.0;
    for (int yy = 0; yy < blk; ++yy)
      for (int xx = 0; xx < blk; ++xx) {
        const int sx = X * blk + xx, sy = Y * blk + yy;
        const int s = sy * Nf + sx;
        for (int d = 0; d < 5; ++d) {
          int tx, ty;
          fine_hop_target(sx, sy, d, Nf, tx, ty);
          // which coarse block receives this hop
          int target;
          if (d == 0) target = 0;
          else {
            const bool inside = (d == 1 && xx + 1 < blk) || (d == 2 && xx > 0) ||
                                (d == 3 && yy + 1 < blk) || (d == 4 && yy > 0);
            target = inside ? 0 : d;
          }
          if (target != dc) continue;
          const int t = ty * Nf + tx;
          for (int a = 0; a < dofF; ++a) {
            const c64 qa = q[((int64_t)s * dofF + a) * nv + i];
            for (int bcol = 0; bcol < dofF; ++bcol) {
              const c64 f = fine_coupling(Bf, U, wdiag, Nf, dofF, s, d, a, bcol);
              const c64 qb = q[((int64_t)t * dofF + bcol) * nv + j];
              const c64 fq = f * qb;
              // conj(qa) * f * qb
              re += qa.re * fq.re + qa.im * fq.im;
              im += qa.re * fq.im - qa.im * fq.re;
            }
          }
        }
      }
    Bc[((int64_t)S * 5 + dc) * nv * nv + e] = {re, im};
  }
}

// dense n x n (left half of an n x 2n array) from a block stencil or the
// Wilson operator; one block per row
__global__ void k_dense_from_stencil(const c64* __restrict__ Bf, const c64* __restrict__ U,
                                     double wdiag, int Nf, int dof, c64* __restrict__ M) {
  const int64_t n = (int64_t)Nf * Nf * dof;
  const int64_t row = blockIdx.x;
  const int s = (int)(row / dof), a = (int)(row - (int64_t)s * dof);
  const int sy = s / Nf, sx = s - sy * Nf;
  c64* mrow = M + row * 2 * n;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) mrow[j] = {0.0, 0.0};
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int d = 0; d < 5; ++d) {
      int tx, ty;
      fine_hop_target(sx, sy, d, Nf, tx, ty);
      const int t = ty * Nf + tx;
      for (int bcol = 0; bcol < dof; ++bcol) {
        const c64 f = fine_coupling(Bf, U, wdiag, Nf, dof, s, d, a, bcol);
        mrow[(int64_t)t * dof + bcol] += f;
      }
    }
  }
}

// the 5 dof x dof blocks of row r = s * dof + a of a block stencil (or of the
// Wilson operator) as column indices and values, 5 * dof entries per row in
// direction-major order (repeated columns where a small periodic lattice wraps
// a hop onto the same site; the host sums them)
__global__ void k_stencil_entries(const c64* __restrict__ Bf, const c64* __restrict__ U,
                                  double wdiag, int Nf, int dof, int* __restrict__ cols,
                                  c64* __restrict__ vals) {
  const int64_t n = (int64_t)Nf * Nf * dof;
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  const int s = (int)(row / dof), a = (int)(row - (int64_t)s * dof);
  const int sy = s / Nf, sx = s - sy * Nf;
  int64_t e = row * 5 * dof;
  for (int d = 0; d < 5; ++d) {
    int tx, ty;
    fine_hop_target(sx, sy, d, Nf, tx, ty);
    const int t = ty * Nf + tx;
    for (int bcol = 0; bcol < dof; ++bcol, ++e) {
      cols[e] = t * dof + bcol;
      vals[e] = fine_coupling(Bf, U, wdiag, Nf, dof, s, d, a, bcol);
    }
  }
}

// Dinv[S] = (B[S][0])^{-1} by Gauss-Jordan with partial pivoting in registers
// of one thread per site (dof <= 16, FP64)
template <int DOF>
__global__ void k_block_diag_inverse(const c64* __restrict__ B, c64* __restrict__ Dinv64,
                                     c32* __restrict__ Dinv32, int ns) {
  const int S = blockIdx.x * blockDim.x + threadIdx.x;
  if (S >= ns) return;
  c64 a[DOF][2 * DOF];
  for (int i = 0; i < DOF; ++i)
    for (int j = 0; j < DOF; ++j) {
      a[i][j] = B[((int64_t)S * 5) * DOF * DOF + i * DOF + j];
      a[i][DOF + j] = {i == j ? 1.0 : 0.0, 0.0};
    }
  for (int c = 0; c < DOF; ++c) {
    int p = c;
    double best = abs2_of(a[c][c]);
    for (int i = c + 1; i < DOF; ++i)
      if (abs2_of(a[i][c]) > best) {
        best = abs2_of(a[i][c]);
        p = i;
      }
    if (p != c)
      for (int j = 0; j < 2 * DOF; ++j) {
        c64 t = a[c][j];
        a[c][j] = a[p][j];
        a[p][j] = t;
      }
    const double dd = abs2_of(a[c][c]);
    const c64 inv = {a[c][c].re / dd, -a[c][c].im / dd};
    for (int j = 0; j < 2 * DOF; ++j) a[c][j] = inv * a[c][j];
    for (int i = 0; i < DOF; ++i) {
      if (i == c) continue;
      const c64 f = a[i][c];
      for (int j = 0; j < 2 * DOF; ++j) a[i][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < DOF; ++i)
    for (int j = 0; j < DOF; ++j) {
      Dinv64[(int64_t)S * DOF * DOF + i * DOF + j] = a[i][DOF + j];
      Dinv32[(int64_t)S * DOF * DOF + i * DOF + j] = {(float)a[i][DOF + j].re,
                                                     (float)a[i][DOF + j].im};
    }
}

inline dim3 grid_sites(int64_t sites, int nb) {
  return dim3((unsigned)((sites + kThreads - 1) / kThreads), (unsigned)nb);
}

// a wave per item, 64 columns per wave: blocks of kThreads/64 waves
inline dim3 grid_waves(int64_t items, int nb) {
  constexpr int wpb = kThreads / 64;
  return dim3((unsigned)((items + wpb - 1) / wpb), (unsigned)((nb + 63) / 64));
}

}  // namespace

int wilson_residual_blocks(int N) { return (N * N + kThreads - 1) / kThreads; }
int bsr_residual_blocks(int Nc) { return (Nc * Nc + kThreads - 1) / kThreads; }

template <typename Tb, typename T, typename Tr>
void wilson_residual(const Tb* b, const T* x, Tr* r, const T* U, int N, double diag, int nb,
                     const int* active, c64* partials, hipStream_t s) {
  hipLaunchKernelGGL((k_wilson_residual<Tb, T, Tr>), grid_sites((int64_t)N * N, nb),
                     dim3(kThreads), 0, s, b, x, r, U, N, (R_t<T>)diag, active, partials);
}

template <typename T>
void wilson_rbgs(const T* b, T* x, const T* U, int N, double diag, int nb, const int* active,
                 bool zero_init, bool reverse, hipStream_t s) {
  MLMC_REQUIRE(N % 2 == 0, MLMC_EINVAL, "red-black sweep needs an even lattice side");
  const dim3 g = grid_sites((int64_t)N * N / 2, nb);
  const int first = reverse ? 1 : 0;
  MLMC_LAUNCH(k_wilson_gs<T>, g, dim3(kThreads), 0, s, b, x, U, N, (R_t<T>)(1.0 / diag), first,
              zero_init ? 1 : 0, active, timing_log());
  MLMC_LAUNCH(k_wilson_gs<T>, g, dim3(kThreads), 0, s, b, x, U, N, (R_t<T>)(1.0 / diag),
              1 - first, 0, active, (int*)nullptr);
}

bool wilson_rbgs_fused_ok(int N) { return N % 16 == 0; }

template <typename T>
void wilson_rbgs_fused(const T* b, const T* xin, T* xout, const T* U, int N, double diag, int nb,
                       const int* active, bool zero_init, bool reverse, hipStream_t s) {
  MLMC_REQUIRE(wilson_rbgs_fused_ok(N), MLMC_EINVAL, "fused sweep needs a side divisible by 16");
  MLMC_REQUIRE(zero_init || xin != xout, MLMC_EINVAL, "fused sweep is out of place");
  const int first = reverse ? 1 : 0;
  const R_t<T> dinv = (R_t<T>)(1.0 / diag);
  if (N % 32 == 0) {
    const dim3 g((unsigned)((N / 32) * (N / 32)), (unsigned)nb);
    MLMC_LAUNCH((k_wilson_gs2<T, 32>), g, dim3(kThreads), 0, s, b, xin, xout, U, N, dinv, first,
                zero_init ? 1 : 0, active, timing_log());
  } else {
    const dim3 g((unsigned)((N / 16) * (N / 16)), (unsigned)nb);
    MLMC_LAUNCH((k_wilson_gs2<T, 16>), g, dim3(kThreads), 0, s, b, xin, xout, U, N, dinv, first,
                zero_init ? 1 : 0, active, timing_log());
  }
}

#define BSR_DISPATCH(DOFV, ...)                                                         \
  switch (DOFV) {                                                                     \
    case 1: { constexpr int D = 1; __VA_ARGS__; break; }                              \
    case 2: { constexpr int D = 2; __VA_ARGS__; break; }                              \
    case 4: { constexpr int D = 4; __VA_ARGS__; break; }                              \
    case 8: { constexpr int D = 8; __VA_ARGS__; break; }                              \
    case 12: { constexpr int D = 12; __VA_ARGS__; break; }                            \
    case 16: { constexpr int D = 16; __VA_ARGS__; break; }                            \
    default: throw Error(MLMC_EUNSUPPORTED, "unsupported number of dofs per site");   \
  }

template <typename Tb, typename T, typename Tr>
void bsr_residual(const Tb* b, const T* x, Tr* r, const T* B, int Nc, int dof, int nb,
                  const int* active, c64* partials, int form, hipStream_t s) {
  // partial sums (the outer residual) come from the thread-per-site form
  if (form == 1 && !partials) {
    const dim3 g = grid_waves((int64_t)Nc * Nc, nb);
    BSR_DISPATCH(dof, hipLaunchKernelGGL((k_bsr_residual<D, Tb, T, Tr>), g, dim3(kThreads), 0, s,
                                          b, x, r, B, Nc, nb, active));
  } else if (!partials) {
    BSR_DISPATCH(dof, {
      const dim3 g = grid_sites((int64_t)Nc * Nc * bsr_group<D>(), nb);
      hipLaunchKernelGGL((k_bsr_residual_rows<D, Tb, T, Tr>), g, dim3(kThreads), 0, s, b, x, r,
                         B, Nc, active);
    });
  } else {
    const dim3 g = grid_sites((int64_t)Nc * Nc, nb);
    BSR_DISPATCH(dof, hipLaunchKernelGGL((k_bsr_residual_sites<D, Tb, T, Tr>), g, dim3(kThreads),
                                          0, s, b, x, r, B, Nc, active, partials));
  }
}

template <typename T>
void bsr_rbgs(const T* b, T* x, const T* B, const T* Dinv, int Nc, int dof, int nb,
              const int* active, bool zero_init, bool reverse, int form, hipStream_t s) {
  if (Nc & 1) throw Error(MLMC_EINVAL, "red-black block sweep needs an even lattice side");
  const int first = reverse ? 1 : 0;
  if (form == 1) {
    const dim3 g = grid_waves((int64_t)Nc * Nc / 2, nb);
    BSR_DISPATCH(dof, MLMC_LAUNCH((k_bsr_gs<D, T>), g, dim3(kThreads), 0, s, b, x, B, Dinv, Nc,
                                   first, zero_init ? 1 : 0, nb, active, timing_log()));
    BSR_DISPATCH(dof, MLMC_LAUNCH((k_bsr_gs<D, T>), g, dim3(kThreads), 0, s, b, x, B, Dinv, Nc,
                                   1 - first, 0, nb, active, (int*)nullptr));
  } else {
    BSR_DISPATCH(dof, {
      const dim3 g = grid_sites((int64_t)Nc * Nc / 2 * bsr_group<D>(), nb);
      MLMC_LAUNCH((k_bsr_gs_rows<D, T>), g, dim3(kThreads), 0, s, b, x, B, Dinv, Nc, first,
                  zero_init ? 1 : 0, active, timing_log());
      MLMC_LAUNCH((k_bsr_gs_rows<D, T>), g, dim3(kThreads), 0, s, b, x, B, Dinv, Nc, 1 - first,
                  0, active, (int*)nullptr);
    });
  }
}

template <typename T>
void agg_restrict(const T* x, T* xc, const T* q, int Nf, int dofF, int blk, int dofC, int nb,
                  const int* active, hipStream_t s) {
  const int Nc = Nf / blk;
  const dim3 g((unsigned)(Nc * Nc), (unsigned)((nb + 63) / 64));
  BSR_DISPATCH(dofC, hipLaunchKernelGGL((k_agg_restrict<D, T>), g, dim3(kThreads), 0, s, x, xc,
                                         q, Nf, dofF, blk, nb, active));
}

template <typename T>
void agg_prolong(const T* xc, T* x, const T* q, int Nf, int dofF, int blk, int dofC,
                 double omega, double beta, int nb, const int* active, hipStream_t s) {
  const dim3 g = grid_sites((int64_t)Nf * Nf * dofF, nb);
  BSR_DISPATCH(dofC, hipLaunchKernelGGL((k_agg_prolong<D, T>), g, dim3(kThreads), 0, s, xc, x, q,
                                         Nf, dofF, blk, (R_t<T>)omega, (R_t<T>)beta, active));
}

void gauge_blocks(const c64* U, int N, double diag, c64* B, hipStream_t s) {
  hipLaunchKernelGGL(k_gauge_blocks, dim3((N * N + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     s, U, N, diag, B);
}

void wilson_links(const double* theta, c64* U64, c32* U32, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_links, dim3(256), dim3(256), 0, s, theta, U64, U32, 2 * N * N);
}

void agg_orthonormalise(const c64* V, c64* q, int Nf, int dofF, int blk, int nv, bool split,
                        hipStream_t s) {
  const int Nc = Nf / blk;
  const size_t lds = sizeof(c64) * (size_t)blk * blk * dofF * nv;
  MLMC_REQUIRE(lds <= 60 * 1024, MLMC_EUNSUPPORTED,
               "aggregate too large for the LDS orthonormalisation");
  MLMC_REQUIRE(!split || dofF % 2 == 0, MLMC_EINVAL, "the spin split needs an even site size");
  hipLaunchKernelGGL(k_agg_orthonormalise, dim3(Nc * Nc), dim3(kThreads), lds, s, V, q, Nf,
                     dofF, blk, nv, split ? 1 : 0);
}

void galerkin_blocks(const c64* Bf, const c64* U, double wdiag, const c64* q, int Nf, int dofF,
                     int blk, int nv, c64* Bc, hipStream_t s) {
  const int Nc = Nf / blk;
  hipLaunchKernelGGL(k_galerkin, dim3(Nc * Nc, 5), dim3(kThreads), 0, s, Bf, U, wdiag, q, Nf,
                     dofF, blk, nv, Bc);
}

void dense_from_stencil(const c64* Bf, const c64* U, double wdiag, int Nf, int dof, c64* aug,
                        hipStream_t s) {
  const int64_t n = (int64_t)Nf * Nf * dof;
  hipLaunchKernelGGL(k_dense_from_stencil, dim3((unsigned)n), dim3(256), 0, s, Bf, U, wdiag, Nf,
                     dof, aug);
}

void stencil_entries(const c64* Bf, const c64* U, double wdiag, int Nf, int dof, int* cols,
                     c64* vals, hipStream_t s) {
  const int64_t n = (int64_t)Nf * Nf * dof;
  hipLaunchKernelGGL(k_stencil_entries, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Bf,
                     U, wdiag, Nf, dof, cols, vals);
}

void block_diag_inverse(const c64* B, c64* Dinv64, c32* Dinv32, int ns, int dof,
                        hipStream_t s) {
  const dim3 g((ns + 63) / 64), blk(64);
  BSR_DISPATCH(dof, hipLaunchKernelGGL((k_block_diag_inverse<D>), g, blk, 0, s, B, Dinv64,
                                        Dinv32, ns));
}

// ---- explicit instantiations ----------------------------------------------
template void wilson_residual<c64, c64, c64>(const c64*, const c64*, c64*, const c64*, int,
                                             double, int, const int*, c64*, hipStream_t);
template void wilson_residual<c64, c64, c32>(const c64*, const c64*, c32*, const c64*, int,
                                             double, int, const int*, c64*, hipStream_t);
template void wilson_residual<c32, c32, c32>(const c32*, const c32*, c32*, const c32*, int,
                                             double, int, const int*, c64*, hipStream_t);
template void wilson_rbgs_fused<c32>(const c32*, const c32*, c32*, const c32*, int, double, int,
                                     const int*, bool, bool, hipStream_t);
template void wilson_rbgs_fused<c64>(const c64*, const c64*, c64*, const c64*, int, double, int,
                                     const int*, bool, bool, hipStream_t);
template void wilson_rbgs<c32>(const c32*, c32*, const c32*, int, double, int, const int*, bool,
                               bool, hipStream_t);
template void wilson_rbgs<c64>(const c64*, c64*, const c64*, int, double, int, const int*, bool,
                               bool, hipStream_t);
template void bsr_residual<c64, c64, c64>(const c64*, const c64*, c64*, const c64*, int, int,
                                          int, const int*, c64*, int, hipStream_t);
template void bsr_residual<c64, c64, c32>(const c64*, const c64*, c32*, const c64*, int, int,
                                          int, const int*, c64*, int, hipStream_t);
template void bsr_residual<c32, c32, c32>(const c32*, const c32*, c32*, const c32*, int, int,
                                          int, const int*, c64*, int, hipStream_t);
template void bsr_rbgs<c32>(const c32*, c32*, const c32*, const c32*, int, int, int, const int*,
                            bool, bool, int, hipStream_t);
template void bsr_rbgs<c64>(const c64*, c64*, const c64*, const c64*, int, int, int, const int*,
                            bool, bool, int, hipStream_t);
template void agg_restrict<c32>(const c32*, c32*, const c32*, int, int, int, int, int,
                                const int*, hipStream_t);
template void agg_restrict<c64>(const c64*, c64*, const c64*, int, int, int, int, int,
                                const int*, hipStream_t);
template void agg_prolong<c32>(const c32*, c32*, const c32*, int, int, int, int, double, double,
                               int, const int*, hipStream_t);
template void agg_prolong<c64>(const c64*, c64*, const c64*, int, int, int, int, double, double,
                               int, const int*, hipStream_t);

}  // namespace mlmc
