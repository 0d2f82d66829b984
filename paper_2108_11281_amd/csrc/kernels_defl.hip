// Block-vector kernels of deflated Hutchinson (Sec. 4.2 eqs. orth_proj / defl,
// the comparison method of Sec. 5) and of the subspace eigensolver that finds
// the deflated eigenvectors: the Gram product C = A^T B of two blocks of
// vectors (a reduction over the n unknowns, split over row chunks and summed in
// a fixed order) and the combination Out = beta X + alpha U C.  Blocks are
// RHS-major: vector j of a block is contiguous, element r at [j * n + r].
// FP64 throughout (the projection feeds the FP64 right-hand side of the refined
// solve); the FP64 vector FMA rate equals the FP64 matrix-core rate on gfx950,
// so these run on plain FMA tiles.
#include "kernels.h"

namespace mlmc {
namespace {

constexpr int kGT = 64;  // Gram output tile (64 x 64 per block, 4 x 4 per thread)
constexpr int kGK = 32;  // unknowns per LDS step

// part[c][i][j] = sum over rows r of chunk c of A[i][r] * B[j][r]
__global__ __launch_bounds__(kThreads) void k_gram_partials(const double* __restrict__ A, int ma,
                                                            const double* __restrict__ B, int mb,
                                                            int64_t n, int64_t chunk,
                                                            double* __restrict__ part) {
  __shared__ double sA[kGK][kGT + 1];
  __shared__ double sB[kGK][kGT + 1];
  const int c = blockIdx.x;
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  const int64_t r0 = (int64_t)c * chunk;
  const int64_t r1 = r0 + chunk < n ? r0 + chunk : n;
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tj = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += kGK) {
    // 64 vectors x 32 consecutive unknowns of each operand; a wave reads two
    // vectors' 32-element runs (coalesced)
#pragma unroll
    for (int e = 0; e < (kGT * kGK) / kThreads; ++e) {
      const int idx = tid + e * kThreads;
      const int ii = idx / kGK, kk = idx - ii * kGK;
      const int64_t r = rb + kk;
      const bool okr = r < r1;
      sA[kk][ii] = (okr && i0 + ii < ma) ? A[(int64_t)(i0 + ii) * n + r] : 0.0;
      sB[kk][ii] = (okr && j0 + ii < mb) ? B[(int64_t)(j0 + ii) * n + r] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kGK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        a[p] = sA[kk][ti * 4 + p];
        b[p] = sB[kk][tj * 4 + p];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
  double* pc = part + (int64_t)c * ma * mb;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int i = i0 + ti * 4 + p;
    if (i >= ma) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tj * 4 + q;
      if (j < mb) pc[(int64_t)i * mb + j] = acc[p][q];
    }
  }
}

// C[i][j] = sum_c part[c][i][j], chunks in ascending order (run to run identical)
__global__ void k_gram_finish(const double* __restrict__ part, int nchunks, int64_t mm,
                              double* __restrict__ C) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= mm) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(int64_t)c * mm + t];
  C[t] = s;
}

constexpr int kCJ = 32;  // output vectors per block of the combination
constexpr int kCM = 64;  // coefficient rows staged in LDS per step

// Out[j][r] = beta X[j][r] + alpha sum_m U[m][r] C[m * ldc + j]; Out may be X
// (each element is read and written by the same thread)
__global__ __launch_bounds__(kThreads) void k_combine(const double* __restrict__ U, int kk,
                                                      const double* __restrict__ C, int ldc,
                                                      const double* X, double* Out, int nc,
                                                      int64_t n, double alpha, double beta) {
  __shared__ double sC[kCM][kCJ];
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int j0 = blockIdx.y * kCJ;
  const int jn = nc - j0 < kCJ ? nc - j0 : kCJ;
  double acc[kCJ];
#pragma unroll
  for (int j = 0; j < kCJ; ++j) acc[j] = 0.0;
  for (int m0 = 0; m0 < kk; m0 += kCM) {
    const int mn = kk - m0 < kCM ? kk - m0 : kCM;
#pragma unroll
    for (int e = 0; e < (kCM * kCJ) / kThreads; ++e) {
      const int idx = threadIdx.x + e * kThreads;
      const int mm = idx / kCJ, jj = idx - mm * kCJ;
      sC[mm][jj] = (mm < mn && jj < jn) ? C[(int64_t)(m0 + mm) * ldc + j0 + jj] : 0.0;
    }
    __syncthreads();
    if (r < n) {
      for (int mm = 0; mm < mn; ++mm) {
        const double u = U[(int64_t)(m0 + mm) * n + r];
#pragma unroll
        for (int j = 0; j < kCJ; ++j) acc[j] = fma(u, sC[mm][j], acc[j]);
      }
    }
    __syncthreads();
  }
  if (r >= n) return;
#pragma unroll
  for (int j = 0; j < kCJ; ++j) {
    if (j < jn) {
      const int64_t o = (int64_t)(j0 + j) * n + r;
      const double base = beta != 0.0 ? beta * X[o] : 0.0;
      Out[o] = base + alpha * acc[j];
    }
  }
}

}  // namespace

int gram_chunks(int64_t n, int ma, int mb) {
  // enough blocks to fill the chip (>= 2048), chunks of at least 1024 unknowns
  const int tiles = ((ma + kGT - 1) / kGT) * ((mb + kGT - 1) / kGT);
  int64_t c = (2048 + tiles - 1) / tiles;
  const int64_t cmax = (n + 1023) / 1024;
  if (c > cmax) c = cmax;
  if (c < 1) c = 1;
  return (int)c;
}

void gram_partials(const double* A, int ma, const double* B, int mb, int64_t n, int nchunks,
                   double* part, hipStream_t s) {
  const int64_t chunk = (n + nchunks - 1) / nchunks;
  dim3 grid(nchunks, (ma + kGT - 1) / kGT, (mb + kGT - 1) / kGT);
  hipLaunchKernelGGL(k_gram_partials, grid, dim3(kThreads), 0, s, A, ma, B, mb, n, chunk, part);
}

void gram_finish(const double* part, int nchunks, int ma, int mb, double* C, hipStream_t s) {
  const int64_t mm = (int64_t)ma * mb;
  hipLaunchKernelGGL(k_gram_finish, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, part,
                     nchunks, mm, C);
}

void block_combine(const double* U, int kk, const double* C, int ldc, const double* X,
                   double* Out, int nc, int64_t n, double alpha, double beta, hipStream_t s) {
  dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (nc + kCJ - 1) / kCJ);
  hipLaunchKernelGGL(k_combine, grid, dim3(kThreads), 0, s, U, kk, C, ldc, X, Out, nc, n, alpha,
                     beta);
}

}  // namespace mlmc
