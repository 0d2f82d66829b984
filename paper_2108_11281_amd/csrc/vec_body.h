// Device bodies of the reduction, Krylov and dense kernels.  Each body takes
// its block index (and, where a workgroup runs more than one block, its thread
// index within the block) as arguments, so that the one-problem launches and
// the grouped launches over several problems run the same operations in the
// same order and give identical results.
#pragma once

#include "common.h"

namespace mlmc {
namespace body {

constexpr int kNT = 256;  // threads of a (virtual) block

// block_sum2 for a block of NT threads that starts at thread `base` of its
// workgroup: wave sums, then the waves' sums added in wave order by thread
// tid == 0.  The barriers are the workgroup's: every thread of the workgroup
// must call it the same number of times.  lds: 2 NT / 64 doubles per block.
template <int NT>
__device__ __forceinline__ void vsum2(double& a, double& b, double* lds, int tid) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = tid & 63, wid = tid >> 6;
  __syncthreads();
  if (lane == 0) {
    lds[2 * wid] = a;
    lds[2 * wid + 1] = b;
  }
  __syncthreads();
  if (tid == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      sa += lds[2 * w];
      sb += lds[2 * w + 1];
    }
    a = sa;
    b = sb;
  }
}

// chunk [lo, hi) of block bx of nblk over n elements
__device__ __forceinline__ void chunk_of(int64_t n, int nblk, int bx, int64_t& lo, int64_t& hi) {
  const int64_t chunk = (n + nblk - 1) / nblk;
  lo = (int64_t)bx * chunk;
  hi = lo + chunk < n ? lo + chunk : n;
}

// partials[k*nblk + bx] = sum over chunk bx of conj(x) y (column k); `live`
// false: the block takes part in the barriers only
template <typename T>
__device__ __forceinline__ void dot(const T* x, const T* y, int64_t n, int nblk, int bx, int k,
                                    bool live, c64* partials, double* lds, int tid) {
  int64_t lo = 0, hi = 0;
  chunk_of(n, nblk, bx, lo, hi);
  if (!live) hi = lo;
  const T* xc = x + (int64_t)k * n;
  const T* yc = y + (int64_t)k * n;
  double re = 0.0, im = 0.0;
  for (int64_t i = lo + tid; i < hi; i += kNT) cdot_acc(re, im, xc[i], yc[i]);
  vsum2<kNT>(re, im, lds, tid);
  if (live && tid == 0) partials[(int64_t)k * nblk + bx] = {re, im};
}

// fixed-order sum of column k's nblk partials
__device__ __forceinline__ c64 finish(const c64* partials, int nblk, int k, double* lds) {
  double re = 0.0, im = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kNT) {
    c64 v = partials[(int64_t)k * nblk + b];
    re += v.re;
    im += v.im;
  }
  vsum2<kNT>(re, im, lds, threadIdx.x);
  return {re, im};
}

// the CG step length of column k from pq (thread 0 of the block)
__device__ __forceinline__ void alpha_rule(c64 pq, const c64* rz, const int* active, int k,
                                           c64* alpha) {
  double a = 0.0;
  if ((!active || active[k]) && pq.re != 0.0 && isfinite(pq.re)) a = rz[k].re / pq.re;
  alpha[k] = {a, 0.0};
}

// the CG direction coefficient of column k from rz_new; rz = rz_new
__device__ __forceinline__ void beta_rule(c64 rzn, c64* rz, const int* active, int k,
                                          c64* beta) {
  double b = 0.0;
  if ((!active || active[k]) && rz[k].re != 0.0) b = rzn.re / rz[k].re;
  beta[k] = {b, 0.0};
  rz[k] = rzn;
}

// x += alpha p ; r -= alpha q ; partials of |r|^2 (column k, block bx of nblk).
// x_zero: x holds no values yet and is taken as zero (not read): x = 0 + alpha p
template <typename T>
__device__ __forceinline__ void cg_xr(T* x, T* r, const T* p, const T* q, c64 a, int64_t n,
                                      int nblk, int bx, int k, c64* partials, double* lds,
                                      bool x_zero = false) {
  int64_t lo = 0, hi = 0;
  chunk_of(n, nblk, bx, lo, hi);
  const int64_t off = (int64_t)k * n;
  double re = 0.0, im = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kNT) {
    const T x0 = x_zero ? zero_of(T()) : x[off + i];
    T xi = x0 + scale_by(a.re, a.im, p[off + i]);
    T ri = r[off + i] - scale_by(a.re, a.im, q[off + i]);
    x[off + i] = xi;
    r[off + i] = ri;
    cdot_acc(re, im, ri, ri);
  }
  vsum2<kNT>(re, im, lds, threadIdx.x);
  if (threadIdx.x == 0) partials[(int64_t)k * nblk + bx] = {re, im};
}

// The FP64 refinement's fold of the FP32 correction, one pass: y += d,
// partials of b^T d (the stated-error share, same blocks and order as the
// dot), d = 0.  Column k, block bx of nblk.  y_zero: y holds no values yet and
// is taken as zero (not read): y = 0 + d
template <typename Tb>
__device__ __forceinline__ void ir_fold(double* y, float* d, const Tb* b, int64_t n, int nblk,
                                        int bx, int k, c64* partials, double* lds,
                                        bool y_zero = false) {
  int64_t lo = 0, hi = 0;
  chunk_of(n, nblk, bx, lo, hi);
  const int64_t off = (int64_t)k * n;
  double re = 0.0, im = 0.0;
  // groups of four elements per thread with every load issued before the
  // arithmetic (twelve loads in flight); the dot accumulates in the order of a
  // plain strided loop
  constexpr int U = 4;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += U * kNT) {
    float dv[U];
    double yv[U], bv[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t i = i0 + (int64_t)j * kNT;
      const bool ok = i < hi;
      dv[j] = ok ? d[off + i] : 0.0f;
      yv[j] = ok && !y_zero ? y[off + i] : 0.0;
      bv[j] = ok ? (double)b[off + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int64_t i = i0 + (int64_t)j * kNT;
      if (i < hi) {
        const double di = (double)dv[j];
        y[off + i] = yv[j] + di;
        cdot_acc(re, im, bv[j], di);
        d[off + i] = 0.0f;
      }
    }
  }
  vsum2<kNT>(re, im, lds, threadIdx.x);
  if (threadIdx.x == 0) partials[(int64_t)k * nblk + bx] = {re, im};
}

// per-column rules of the refinement (one column each)
__device__ __forceinline__ int mark_rule(const c64* rr, const c64* ref, double tol2, int* active,
                                         int k) {
  int a = active[k];
  if (a && rr[k].re <= tol2 * ref[k].re) a = 0;
  if (a && !isfinite(rr[k].re)) a = 0;  // reported by the host as non-converged
  active[k] = a;
  return a;
}
__device__ __forceinline__ bool due_rule(const c64* rr, const c64* rr_upd, const c64* bb,
                                         double delta2, double tol2, int k) {
  const double v = rr[k].re;
  return v <= delta2 * rr_upd[k].re || v <= tol2 * bb[k].re || !isfinite(v);
}
__device__ __forceinline__ void ir_err_rule(const c64* bd, const c64* rr_old, const c64* rr_new,
                                            c64* err, int k) {
  const double mag = sqrt(bd[k].re * bd[k].re + bd[k].im * bd[k].im);
  const double ratio = rr_old[k].re > 0.0 ? sqrt(rr_new[k].re / rr_old[k].re) : 1.0;
  err[k] = {mag * ratio, 0.0};
}
__device__ __forceinline__ void restart_rule(const c64* rr_new, const c64* rr_rec, c64* rz,
                                             double factor, int k) {
  if (!(rr_new[k].re <= factor * rr_rec[k].re)) rz[k] = {0.0, 0.0};
}

// ---- coarsest solve as an MFMA GEMM: Z = B At (real types, n % 16 == 0) ----
// One wave computes a 16 (RHS) x 16 (unknowns) tile of Z with
// v_mfma_{f32,f64}_16x16x4.  Operand layout of these instructions (one block):
// A (16x4): lane l holds A[l % 16][l / 16]; B (4x16): lane l holds
// B[l / 16][l % 16]; D (16x16): lane l, register r holds D[row][l % 16] with
// row = 4*(l/16) + r for the f32 form and row = 4*r + l/16 for the f64 form.
// The reduction index is permuted inside each chunk of 16 (lane group g supplies
// k = 4g + s at step s for both operands), which leaves the sum unchanged and
// lets each lane load its A values as one vector.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc_t = f32x4;
  __device__ static acc_t step(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int g, int r) { return 4 * g + r; }
};
template <> struct Mfma<double> {
  using acc_t = f64x4;
  __device__ static acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int g, int r) { return 4 * r + g; }
};

// The 16 x 16 tile (bx, by) of Z.  The reduction index, in chunks of 16, is
// split into kDenseParts consecutive ranges; each range's partial tile is
// accumulated in chunk order (UNR chunks of loads in flight), and the partial
// tiles are summed in range order in LDS (wave r sums accumulator row r).  W
// waves per tile (W >= 4 divides
// kDenseParts): wave w computes its kDenseParts / W ranges one after another,
// so the sums do not depend on W.  Pk is the transposed inverse in the packed
// MFMA layout of dense_pack4 (leading dimension ld, a multiple of 16; rows and
// columns n..ld-1 zero): the four reduction indices a lane supplies to one
// chunk's four MFMA steps are 16 contiguous bytes (32 for FP64), as are its
// four right-hand-side entries when n is a multiple of 4.  B and Z columns
// have length n, so the tail of the last tile reads zeros and writes nothing.
// part: kDenseParts x 4 x 64 T of LDS per tile; tid: thread within the tile's
// W waves; `live` false: barriers only.  [klo, khi): the right-hand sides
// computed and stored (the others of the tile are read as zero); the sums of
// the computed ones do not depend on it.
constexpr int kDenseParts = 16;
template <typename T> struct Vec4 {
  typedef T type __attribute__((ext_vector_type(4)));
};
template <typename T, int W = 4>
__device__ __forceinline__ void dense_apply_mfma(const T* __restrict__ Pk, const T* __restrict__ B,
                                                 T* __restrict__ Z, int n, int ld, int nb,
                                                 const int* active, int bx, int by, bool live,
                                                 T* part, int tid, int klo = 0,
                                                 int khi = 1 << 30) {
  static_assert(kDenseParts % W == 0 && W >= 4, "waves must divide the ranges (at least 4)");
  using V4 = typename Vec4<T>::type;
  constexpr int UNR = 4, PPW = kDenseParts / W;
  const int wave = tid >> 6, lane = tid & 63;
  const int i0 = bx * 16;       // unknown tile
  const int m0 = by * 16;       // RHS tile
  const int g = lane >> 4, c = lane & 15;
  const int row = m0 + c;       // RHS whose A-operand this lane supplies
  const bool row_ok = row < nb && row >= klo && row < khi;
  const T* brow = B + (int64_t)(row_ok ? row : 0) * n;
  const bool bvec = (n & 3) == 0;  // B rows 16-byte aligned in groups of four
  const int chunks = live ? ld / 16 : 0;
  // the four reduction indices 16 ch + 4 g + s (s = 0..3) of chunk ch
  auto load = [&](int ch, T* a, T* bv) {
    const int j = ch * 16 + 4 * g;
    const V4 p = *reinterpret_cast<const V4*>(Pk + ((int64_t)(ch * 4 + g) * ld + i0 + c) * 4);
    if (bvec) {
      V4 q = {0, 0, 0, 0};
      if (row_ok && j < n) q = *reinterpret_cast<const V4*>(brow + j);
#pragma unroll
      for (int s = 0; s < 4; ++s) a[s] = q[s];
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) a[s] = (row_ok && j + s < n) ? brow[j + s] : (T)0;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) bv[s] = p[s];
  };
  for (int q = 0; q < PPW; ++q) {
    const int p = wave * PPW + q;
    const int cbeg = p * chunks / kDenseParts, cend = (p + 1) * chunks / kDenseParts;
    typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
    int ch = cbeg;
    for (; ch + UNR <= cend; ch += UNR) {
      T a[UNR][4], bv[UNR][4];
#pragma unroll
      for (int u = 0; u < UNR; ++u) load(ch + u, a[u], bv[u]);
#pragma unroll
      for (int u = 0; u < UNR; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc = Mfma<T>::step(a[u][s], bv[u][s], acc);
    }
    for (; ch < cend; ++ch) {
      T a[4], bv[4];
      load(ch, a, bv);
#pragma unroll
      for (int s = 0; s < 4; ++s) acc = Mfma<T>::step(a[s], bv[s], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part[(p * 4 + r) * 64 + lane] = acc[r];
  }
  __syncthreads();
  if (wave < 4 && live) {  // wave r sums accumulator row r of the partial tiles
    const int r = wave;
    T v = part[r * 64 + lane];
#pragma unroll
    for (int p = 1; p < kDenseParts; ++p) v = v + part[(p * 4 + r) * 64 + lane];
    const int k = m0 + Mfma<T>::row(g, r);
    if (k < nb && k >= klo && k < khi && (!active || active[k]) && i0 + c < n)
      Z[(int64_t)k * n + i0 + c] = v;
  }
}

}  // namespace body
}  // namespace mlmc
