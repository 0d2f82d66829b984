// Batched flexible GMRES building blocks: columns iterate in lockstep, each
// with its own Hessenberg matrix, Givens rotations and residual estimate
// (FP64 scalars on the device; vectors in the working precision).
// Krylov vectors of one basis are stored consecutively: vector i of column k
// at base + i*vstride + k*n.
#include "kernels.h"

namespace mlmc {
namespace {

constexpr int kMaxBasis = 33;  // restart length + 1

// partials[((k*nv + i) * nblk) + b] = sum over block b of conj(V_i) w  (column k);
// the basis is walked in groups of four vectors (register accumulators), w is
// re-read per group from cache
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mdot(const T* __restrict__ V, int64_t vstride,
                                                   int nv, const T* __restrict__ w, int64_t n,
                                                   const int* active, c64* partials) {
  __shared__ double red[16];
  const int k = blockIdx.y, nblk = gridDim.x;
  if (active && !active[k]) return;
  const int64_t chunk = (n + nblk - 1) / nblk;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  const T* wk = w + (int64_t)k * n;
  for (int i0 = 0; i0 < nv; i0 += 4) {
    double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    const int gcount = nv - i0 < 4 ? nv - i0 : 4;
    // two elements per step, their ten loads issued before the products, which
    // accumulate in element order as in a plain strided loop
    for (int64_t e0 = lo + threadIdx.x; e0 < hi; e0 += 2 * kThreads) {
      T we[2], ve[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int64_t e = e0 + (int64_t)q * kThreads;
        const int64_t ec = e < hi ? e : lo;
        we[q] = wk[ec];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          ve[q][u] = V[(i0 + (u < gcount ? u : 0)) * vstride + (int64_t)k * n + ec];
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (e0 + (int64_t)q * kThreads < hi) {
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (u < gcount) cdot_acc(re[u], im[u], ve[q][u], we[q]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < gcount) {
        double a = re[u], b = im[u];
        block_sum2<kThreads>(a, b, red);
        if (threadIdx.x == 0) partials[((int64_t)k * nv + i0 + u) * nblk + blockIdx.x] = {a, b};
      }
    }
  }
}

// w -= sum_i h[k*nv + i] V_i
template <typename T>
__global__ __launch_bounds__(kThreads) void k_maxpy(const T* __restrict__ V, int64_t vstride,
                                                    int nv, const c64* __restrict__ h,
                                                    T* __restrict__ w, int64_t n,
                                                    const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  T acc = w[(int64_t)k * n + e];
#pragma unroll 4
  for (int i = 0; i < nv; ++i) {
    const c64 c = h[(int64_t)k * nv + i];
    acc -= scale_by(c.re, c.im, V[i * vstride + (int64_t)k * n + e]);
  }
  w[(int64_t)k * n + e] = acc;
}

// d = sum_{i < dims[k]} y[k*ldy + i] Z_i for columns with start[k]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_combine(const T* __restrict__ Z, int64_t vstride,
                                                      const c64* __restrict__ y, int ldy,
                                                      const int* __restrict__ dims,
                                                      T* __restrict__ d, int64_t n,
                                                      const int* start) {
  const int k = blockIdx.y;
  if (!start[k]) return;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  T acc = zero_of(T());
  const int m = dims[k];
#pragma unroll 4
  for (int i = 0; i < m; ++i) {
    const c64 c = y[(int64_t)k * ldy + i];
    acc += scale_by(c.re, c.im, Z[i * vstride + (int64_t)k * n + e]);
  }
  d[(int64_t)k * n + e] = acc;
}

// dst = src / sqrt(nrm2[k])
template <typename T>
__global__ void k_scale_inv_norm(T* dst, const T* src, const c64* nrm2, int64_t n,
                                 const int* active) {
  const int k = blockIdx.y;
  if (active && !active[k]) return;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  const double s = nrm2[k].re > 0.0 ? 1.0 / sqrt(nrm2[k].re) : 0.0;
  dst[(int64_t)k * n + e] = scale_by(s, 0.0, src[(int64_t)k * n + e]);
}

struct GState {
  c64* H;     // [nb][m+1][m]  Hessenberg (rotated in place: upper triangle R)
  c64* cs;    // [nb][m]       rotation cosines (real part used)
  c64* sn;    // [nb][m]       rotation sines
  c64* g;     // [nb][m+1]     rotated right-hand side
  int* dims;  // [nb]          basis size used by the column
};

__global__ void k_givens_init(GState st, const c64* beta2, const int* active, int m, int nb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb) return;
  st.dims[k] = 0;
  for (int i = 0; i <= m; ++i) st.g[(int64_t)k * (m + 1) + i] = {0.0, 0.0};
  if (active[k]) st.g[(int64_t)k * (m + 1)] = {sqrt(beta2[k].re), 0.0};
}

// Column j of the Hessenberg matrix: h[k*(j+1) + i] (i <= j) and |w|^2 (h_{j+1,j}^2).
// Applies the previous rotations, forms the new one, updates g; columns whose
// residual estimate |g_{j+1}| <= tol * beta stop (active = 0, dims = j+1).
__global__ void k_givens_step(GState st, const c64* h, const c64* wn2, const c64* beta2,
                              double tol, int j, int m, int* active, int nb, int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    if (!active[k]) continue;
    c64* Hk = st.H + (int64_t)k * (m + 1) * m;
    const c64* hk = h + (int64_t)k * (j + 1);
    // rotation i acts on entries i (already rotated by rotation i - 1) and i + 1
    // (still as formed): the column streams through `a`, and entry i is final
    // after rotation i (no indexed local array, which would live in scratch)
    c64 a = hk[0];
    for (int i = 0; i < j; ++i) {
      const double c = st.cs[(int64_t)k * m + i].re;
      const c64 s = st.sn[(int64_t)k * m + i];
      const c64 b = hk[i + 1];
      // [a; b] <- [c a + s b; -conj(s) a + c b]
      Hk[(int64_t)i * m + j] = c * a + s * b;
      const c64 sc = {s.re, -s.im};
      a = c * b - sc * a;
    }
    const c64 b = {sqrt(wn2[k].re), 0.0};
    const double na = sqrt(a.re * a.re + a.im * a.im), nbv = sqrt(b.re * b.re + b.im * b.im);
    const double r = sqrt(na * na + nbv * nbv);
    double c;
    c64 s;
    if (r == 0.0) {
      c = 1.0;
      s = {0.0, 0.0};
    } else if (na == 0.0) {
      c = 0.0;
      s = {b.re / nbv, -b.im / nbv};  // conj(b)/|b|
    } else {
      c = na / r;
      const c64 ph = {a.re / na, a.im / na};
      const c64 bc = {b.re / r, -b.im / r};  // conj(b)/r
      s = ph * bc;
    }
    st.cs[(int64_t)k * m + j] = {c, 0.0};
    st.sn[(int64_t)k * m + j] = s;
    Hk[(int64_t)j * m + j] = c * a + s * b;
    c64* gk = st.g + (int64_t)k * (m + 1);
    const c64 gj = gk[j];
    const c64 sc = {s.re, -s.im};
    gk[j] = c * gj;
    gk[j + 1] = -1.0 * (sc * gj);
    const double res = sqrt(gk[j + 1].re * gk[j + 1].re + gk[j + 1].im * gk[j + 1].im);
    st.dims[k] = j + 1;
    const double bn = sqrt(beta2[k].re);
    if (res <= tol * bn || !(res == res) || j + 1 == m)
      active[k] = 0;
    else
      atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

// y = R^{-1} g (back substitution on the rotated Hessenberg), per column
__global__ void k_givens_solve(GState st, c64* y, const int* start, int m, int nb) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nb || !start[k]) return;
  const c64* Hk = st.H + (int64_t)k * (m + 1) * m;
  const c64* gk = st.g + (int64_t)k * (m + 1);
  c64* yk = y + (int64_t)k * m;
  const int d = st.dims[k];
  for (int i = d - 1; i >= 0; --i) {
    c64 acc = gk[i];
    for (int j = i + 1; j < d; ++j) acc -= Hk[(int64_t)i * m + j] * yk[j];
    const c64 rii = Hk[(int64_t)i * m + i];
    const double dd = rii.re * rii.re + rii.im * rii.im;
    const c64 inv = dd > 0.0 ? c64{rii.re / dd, -rii.im / dd} : c64{0.0, 0.0};
    yk[i] = inv * acc;
  }
}

inline dim3 grid_n(int64_t n, int nb) {
  return dim3((unsigned)((n + kThreads - 1) / kThreads), (unsigned)nb);
}

}  // namespace

template <typename T>
void krylov_mdot(const T* V, int64_t vstride, int nv, const T* w, int64_t n, int nb,
                 const int* active, c64* partials, int* nblk_out, hipStream_t s) {
  MLMC_REQUIRE(nv <= kMaxBasis, MLMC_EUNSUPPORTED, "Krylov basis too large");
  // enough parallelism but few partials: nv*nb*nblk entries
  int nblk = reduce_blocks(n);
  if (nblk > 256) nblk = 256;
  *nblk_out = nblk;
  hipLaunchKernelGGL(k_mdot<T>, dim3(nblk, nb), dim3(kThreads), 0, s, V, vstride, nv, w, n,
                     active, partials);
}

template <typename T>
void krylov_maxpy(const T* V, int64_t vstride, int nv, const c64* h, T* w, int64_t n, int nb,
                  const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_maxpy<T>, grid_n(n, nb), dim3(kThreads), 0, s, V, vstride, nv, h, w, n,
                     active);
}

template <typename T>
void krylov_combine(const T* Z, int64_t vstride, const c64* y, int ldy, const int* dims, T* d,
                    int64_t n, int nb, const int* start, hipStream_t s) {
  hipLaunchKernelGGL(k_combine<T>, grid_n(n, nb), dim3(kThreads), 0, s, Z, vstride, y, ldy,
                     dims, d, n, start);
}

template <typename T>
void vec_scale_inv_norm(T* dst, const T* src, const c64* nrm2, int64_t n, int nb,
                        const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inv_norm<T>, grid_n(n, nb), dim3(kThreads), 0, s, dst, src, nrm2,
                     n, active);
}

void givens_init(c64* H, c64* cs, c64* sn, c64* g, int* dims, const c64* beta2,
                 const int* active, int m, int nb, hipStream_t s) {
  GState st{H, cs, sn, g, dims};
  hipLaunchKernelGGL(k_givens_init, dim3((nb + 255) / 256), dim3(256), 0, s, st, beta2, active,
                     m, nb);
}

void givens_step(c64* H, c64* cs, c64* sn, c64* g, int* dims, const c64* h, const c64* wn2,
                 const c64* beta2, double tol, int j, int m, int* active, int nb, int* count,
                 hipStream_t s) {
  GState st{H, cs, sn, g, dims};
  hipLaunchKernelGGL(k_givens_step, dim3(1), dim3(256), 0, s, st, h, wn2, beta2, tol, j, m,
                     active, nb, count);
}

void givens_solve(c64* H, c64* cs, c64* sn, c64* g, int* dims, c64* y, const int* start, int m,
                  int nb, hipStream_t s) {
  GState st{H, cs, sn, g, dims};
  hipLaunchKernelGGL(k_givens_solve, dim3((nb + 255) / 256), dim3(256), 0, s, st, y, start, m,
                     nb);
}

#define MLMC_INST_K(T)                                                                      \
  template void krylov_mdot<T>(const T*, int64_t, int, const T*, int64_t, int, const int*,  \
                               c64*, int*, hipStream_t);                                    \
  template void krylov_maxpy<T>(const T*, int64_t, int, const c64*, T*, int64_t, int,       \
                                const int*, hipStream_t);                                   \
  template void krylov_combine<T>(const T*, int64_t, const c64*, int, const int*, T*,       \
                                  int64_t, int, const int*, hipStream_t);                   \
  template void vec_scale_inv_norm<T>(T*, const T*, const c64*, int64_t, int, const int*,   \
                                      hipStream_t);

MLMC_INST_K(c32)
MLMC_INST_K(c64)
MLMC_INST_K(float)
MLMC_INST_K(double)

}  // namespace mlmc
