// Learned smoother for the 2-spin lattice operator: a 3-layer 3x3 convolutional
// network (8 -> 16 -> 16 -> 4 channels, ReLU, no bias) that maps the RMS-scaled
// residual and the link phases of each site to a correction of the iterate.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation): rows = 16 lattice sites of a region, columns =
// 16 output channels, K = (tap, input channel) in chunks of 32.  Lane layout of
// that instruction (one wave): lane l supplies A[row l%16][k 8(l/16)..+7] and
// B[k 8(l/16)..+7][col l%16], and receives D[rows 4(l/16)..+3][col l%16].
//
// Inference (k_nn_apply): one workgroup per 16 x 16 output tile and right-hand
// side; the 22 x 22 input region (halo 3, periodic wrap) and both hidden layers
// stay in LDS, the correction s * net(r / s) is added to x in place.
// Training (k_nn_train): one workgroup per 22 x 22 crop; forward, loss, and the
// backward pass (weight gradients and data gradients through both ReLUs) all in
// LDS; per-crop weight gradients are reduced in a fixed order afterwards.
#include "kernels.h"

namespace mlmc {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTo = 16;          // output tile side
constexpr int kT2 = kTo + 2;     // second hidden layer region side (18)
constexpr int kT1 = kTo + 4;     // first hidden layer region side (20)
constexpr int kT0 = kTo + 6;     // input region side (22)
constexpr int kC0 = 8, kC1 = 16, kC2 = 16, kC3 = 4;
constexpr int kOffW1 = 0, kOffW2 = 16 * 8 * 9, kOffW3 = kOffW2 + 16 * 16 * 9;
constexpr int kNumW = kOffW3 + 4 * 16 * 9;   // 4032
// packed forward B fragments: chunks per layer (K padded to multiples of 32)
constexpr int kCh1 = 3, kCh2 = 5, kCh3 = 5;
constexpr int kFragL1 = 0, kFragL2 = kCh1, kFragL3 = kCh1 + kCh2, kFrags = kCh1 + kCh2 + kCh3;

__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf8 bf8_zero() {
  bf8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
  return z;
}

// One forward convolution layer of a workgroup (4 waves): out region Ho x Wo
// from the input region (Ho+2) x (Wo+2) in LDS ([site][CIN] BF16, or with PIN
// two planes [CIN/8][site][8] of in_plane sites).  Output either BF16
// [site][16] (ReLU applied; POUT: planes [2][site][8] of out_plane sites) or
// FP32 [site][4] (last layer).  The planar form keeps the 16-byte operand
// loads of 16 consecutive sites on consecutive LDS addresses (with [site][16]
// they are 32 bytes apart and two of every eight lanes share banks).
template <int CIN, int COUT, int NCH, bool RELU, bool F32OUT, bool PIN = false, bool POUT = false>
__device__ void conv_fwd(const __bf16* __restrict__ in, int Wi, void* out, int Wo, int Ho,
                         const bf8* __restrict__ frag, int wave, int lane, int in_plane = 0,
                         int out_plane = 0) {
  bf8 b[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) b[c] = frag[c * 64 + lane];
  const int nsites = Wo * Ho;
  const int mtiles = (nsites + 15) / 16;
  const int g = lane >> 4, r16 = lane & 15;
  for (int m = wave; m < mtiles; m += 4) {
    const int p = 16 * m + r16;
    const bool pv = p < nsites;
    const int py = pv ? p / Wo : 0, px = pv ? p - (p / Wo) * Wo : 0;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int k0 = 32 * c + 8 * g;
      const int tap = k0 / CIN, ci0 = k0 - tap * CIN;
      bf8 a = bf8_zero();
      if (pv && tap < 9) {
        const int ay = py + tap / 3, ax = px + tap % 3;
        if constexpr (PIN)
          a = *reinterpret_cast<const bf8*>(in + ((ci0 >> 3) * in_plane + ay * Wi + ax) * 8);
        else
          a = *reinterpret_cast<const bf8*>(in + (ay * Wi + ax) * CIN + ci0);
      }
      acc = mfma(a, b[c], acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = 16 * m + 4 * g + i;
      if (q < nsites && r16 < COUT) {
        float v = acc[i];
        if (RELU) v = fmaxf(v, 0.f);
        if (F32OUT)
          static_cast<float*>(out)[q * COUT + r16] = v;
        else if (POUT)
          static_cast<__bf16*>(out)[((r16 >> 3) * out_plane + q) * 8 + (r16 & 7)] = (__bf16)v;
        else
          static_cast<__bf16*>(out)[q * 16 + r16] = (__bf16)v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// inference
// ---------------------------------------------------------------------------
// the input region is dead once the first hidden layer is formed, and that
// layer once the second is: each pair shares its LDS (two barriers between)
struct NnApplyLds {
  union {
    __bf16 x0[kT0 * kT0 * kC0];
    __bf16 h2[2 * kT2 * kT2 * 8];  // planes [2][site][8]
  };
  union {
    __bf16 h1[2 * kT1 * kT1 * 8];  // planes [2][site][8]
    float o[kTo * kTo * kC3];
  };
};

__global__ __launch_bounds__(256) void k_nn_apply(const c32* __restrict__ r, c32* __restrict__ x,
                                                  const c64* __restrict__ rr, double inv_n,
                                                  const __bf16* __restrict__ links,
                                                  const bf8* __restrict__ frag, int N, int tiles_x,
                                                  const int* active, int* tlog) {
  __shared__ __attribute__((aligned(16))) NnApplyLds sm;
  const int col = blockIdx.y;
  if (tlog && blockIdx.x == 0 && threadIdx.x == 0) tlog[col] = active ? active[col] : 1;
  if (active && !active[col]) return;
  const double s2 = rr[col].re * inv_n;
  if (!(s2 > 0.0)) return;  // zero residual: no correction
  const float s = (float)sqrt(s2), inv_s = (float)(1.0 / sqrt(s2));
  const int ty0 = (blockIdx.x / tiles_x) * kTo, tx0 = (blockIdx.x % tiles_x) * kTo;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t off = (int64_t)col * N * N * 2;
  for (int idx = tid; idx < kT0 * kT0; idx += 256) {
    const int ry = idx / kT0, rx = idx - ry * kT0;
    const int gy = (ty0 + ry - 3 + N) % N, gx = (tx0 + rx - 3 + N) % N;
    const int site = gy * N + gx;
    const c32 r0 = r[off + 2 * site], r1 = r[off + 2 * site + 1];
    __bf16* d = sm.x0 + idx * kC0;
    d[0] = (__bf16)(r0.re * inv_s);
    d[1] = (__bf16)(r0.im * inv_s);
    d[2] = (__bf16)(r1.re * inv_s);
    d[3] = (__bf16)(r1.im * inv_s);
    d[4] = links[site * 4 + 0];
    d[5] = links[site * 4 + 1];
    d[6] = links[site * 4 + 2];
    d[7] = links[site * 4 + 3];
  }
  __syncthreads();
  conv_fwd<kC0, kC1, kCh1, true, false, false, true>(sm.x0, kT0, sm.h1, kT1, kT1,
                                                     frag + kFragL1 * 64, wave, lane, 0,
                                                     kT1 * kT1);
  __syncthreads();
  conv_fwd<kC1, kC2, kCh2, true, false, true, true>(sm.h1, kT1, sm.h2, kT2, kT2,
                                                    frag + kFragL2 * 64, wave, lane, kT1 * kT1,
                                                    kT2 * kT2);
  __syncthreads();
  conv_fwd<kC2, kC3, kCh3, false, true, true, false>(sm.h2, kT2, sm.o, kTo, kTo,
                                                     frag + kFragL3 * 64, wave, lane, kT2 * kT2);
  __syncthreads();
  {
    const int ly = tid / kTo, lx = tid - ly * kTo;
    const int site = (ty0 + ly) * N + (tx0 + lx);
    const float* o = sm.o + tid * kC3;
    c32* xs = x + off + 2 * site;
    c32 a = xs[0], b = xs[1];
    a.re += s * o[0];
    a.im += s * o[1];
    b.re += s * o[2];
    b.im += s * o[3];
    xs[0] = a;
    xs[1] = b;
  }
}

// link features (cos, sin of theta_0 and theta_1 per site) in BF16
__global__ void k_nn_links(const double* __restrict__ theta, __bf16* __restrict__ links, int N) {
  const int n = N * N;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    links[4 * i + 0] = (__bf16)(float)cos(theta[i]);
    links[4 * i + 1] = (__bf16)(float)sin(theta[i]);
    links[4 * i + 2] = (__bf16)(float)cos(theta[n + i]);
    links[4 * i + 3] = (__bf16)(float)sin(theta[n + i]);
  }
}

// forward B fragments from the FP32 master weights W[co][ci][tap]
__global__ void k_nn_pack(const float* __restrict__ w, bf8* __restrict__ frag) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kFrags * 64) return;
  const int chunk = t / 64, lane = t % 64;
  int layer, c, cin, cout, off;
  if (chunk < kFragL2) {
    layer = 0; c = chunk; cin = kC0; cout = kC1; off = kOffW1;
  } else if (chunk < kFragL3) {
    layer = 1; c = chunk - kFragL2; cin = kC1; cout = kC2; off = kOffW2;
  } else {
    layer = 2; c = chunk - kFragL3; cin = kC2; cout = kC3; off = kOffW3;
  }
  (void)layer;
  const int n = lane & 15;
  bf8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int k = 32 * c + 8 * (lane >> 4) + j;
    const int tap = k / cin, ci = k - tap * cin;
    const float val = (tap < 9 && n < cout) ? w[off + (n * cin + ci) * 9 + tap] : 0.f;
    v[j] = (__bf16)val;
  }
  frag[t] = v;
}

// ---------------------------------------------------------------------------
// training: forward + backward of one 22 x 22 crop per workgroup
// ---------------------------------------------------------------------------
struct NnTrainLds {
  __bf16 x0[kT0 * kT0 * kC0];   // input
  __bf16 h1[kT1 * kT1 * 16];    // ReLU(z1)
  __bf16 h2[kT2 * kT2 * 16];    // ReLU(z2)
  float o[kTo * kTo * kC3];     // output
  __bf16 dout[kTo * kTo * 8];   // dL/d out, channels padded to 8
  __bf16 dz2[kT2 * kT2 * 16];   // dL/d z2
  __bf16 dz1[kT1 * kT1 * 16];   // dL/d z1
  double red[8];
};

// weight gradient of one layer: dW[co][ci][tap] = sum_p dY[p][co] X[p + tap][ci]
// over the Ho x Wo output region; dY [site][DYS] (BF16), X [site][CIN].  Work
// items: (tap group), each a 16 x 16 block over (co, n); CIN = 16: one tap per
// item (n = ci); CIN = 8: two taps per item (n = 8 * (tap - 2T) + ci).
template <int CIN, int COUT, int DYS>
__device__ void conv_wgrad(const __bf16* __restrict__ dy, const __bf16* __restrict__ X, int Wi,
                           int Wo, int Ho, float* __restrict__ gout, int wave, int lane) {
  const int nsites = Wo * Ho;
  const int nch = (nsites + 31) / 32;
  const int items = CIN == 16 ? 9 : 5;
  const int g = lane >> 4, r16 = lane & 15;
  for (int it = wave; it < items; it += 4) {
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    // B column n = r16 -> (tap, ci)
    const int tapB = CIN == 16 ? it : 2 * it + (r16 >> 3);
    const int ciB = CIN == 16 ? r16 : (r16 & 7);
    const bool bv = tapB < 9;
    const int ta = bv ? tapB / 3 : 0, tb = bv ? tapB % 3 : 0;
    for (int c = 0; c < nch; ++c) {
      bf8 a, b;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int p = 32 * c + 8 * g + j;
        const bool pv = p < nsites;
        const int py = pv ? p / Wo : 0, px = pv ? p - (p / Wo) * Wo : 0;
        a[j] = (pv && r16 < COUT) ? dy[p * DYS + r16] : (__bf16)0.0f;
        b[j] = (pv && bv) ? X[((py + ta) * Wi + px + tb) * CIN + ciB] : (__bf16)0.0f;
      }
      acc = mfma(a, b, acc);
    }
    // D rows co = 4g + i, column n = r16
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int co = 4 * g + i;
      if (co < COUT && bv) gout[(co * CIN + ciB) * 9 + tapB] = acc[i];
    }
  }
}

// data gradient through a convolution, times the ReLU mask of the input
// activation: dX[q][ci] = [X[q] > 0] * sum_{tap, co} W[co][ci][tap] dY[q - tap][co]
// over the Hi x Wi input region; dY [site][DYS] on the (Hi-2) x (Wi-2) output
// region (DYS = padded channel count, 8 or 16), W FP32 master weights of the
// layer; result BF16 [site][16].
template <int CIN, int COUT, int DYS>
__device__ void conv_dgrad(const __bf16* __restrict__ dy, const __bf16* __restrict__ X, int Wi,
                           int Hi, const float* __restrict__ W, __bf16* __restrict__ dx, int wave,
                           int lane) {
  constexpr int K = 9 * DYS;
  constexpr int NCH = (K + 31) / 32;
  const int Wo = Wi - 2, Ho = Hi - 2;
  const int g = lane >> 4, r16 = lane & 15;
  // B fragments: k = tap * DYS + co, column ci = r16
  bf8 b[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 32 * c + 8 * g + j;
      const int tap = k / DYS, co = k - tap * DYS;
      b[c][j] = (tap < 9 && co < COUT && r16 < CIN) ? (__bf16)W[(co * CIN + r16) * 9 + tap]
                                                   : (__bf16)0.0f;
    }
  }
  const int nsites = Wi * Hi;
  const int mtiles = (nsites + 15) / 16;
  for (int m = wave; m < mtiles; m += 4) {
    const int q = 16 * m + r16;
    const bool qv = q < nsites;
    const int qy = qv ? q / Wi : 0, qx = qv ? q - (q / Wi) * Wi : 0;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      const int k0 = 32 * c + 8 * g;
      const int tap = k0 / DYS, co0 = k0 - tap * DYS;
      bf8 a = bf8_zero();
      if (qv && tap < 9) {
        const int oy = qy - tap / 3, ox = qx - tap % 3;
        if (oy >= 0 && oy < Ho && ox >= 0 && ox < Wo)
          a = *reinterpret_cast<const bf8*>(dy + (oy * Wo + ox) * DYS + co0);
      }
      acc = mfma(a, b[c], acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int qq = 16 * m + 4 * g + i;
      if (qq < nsites && r16 < CIN) {
        const float mask = (float)X[qq * 16 + r16] > 0.f ? 1.f : 0.f;
        dx[qq * 16 + r16] = (__bf16)(acc[i] * mask);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_nn_train(const __bf16* __restrict__ in,
                                                  const float* __restrict__ tgt,
                                                  const int* __restrict__ order,
                                                  const bf8* __restrict__ frag,
                                                  const float* __restrict__ w,
                                                  float* __restrict__ gpart,
                                                  double* __restrict__ lpart, float dscale) {
  __shared__ __attribute__((aligned(16))) NnTrainLds sm;
  const int item = blockIdx.x;                       // slot of this crop in the step
  const int crop = order ? order[item] : item;       // crop in the data set
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  {
    const bf8* src = reinterpret_cast<const bf8*>(in + (int64_t)crop * kT0 * kT0 * kC0);
    bf8* dst = reinterpret_cast<bf8*>(sm.x0);
    for (int i = tid; i < kT0 * kT0; i += 256) dst[i] = src[i];
  }
  __syncthreads();
  conv_fwd<kC0, kC1, kCh1, true, false>(sm.x0, kT0, sm.h1, kT1, kT1, frag + kFragL1 * 64, wave,
                                        lane);
  __syncthreads();
  conv_fwd<kC1, kC2, kCh2, true, false>(sm.h1, kT1, sm.h2, kT2, kT2, frag + kFragL2 * 64, wave,
                                        lane);
  __syncthreads();
  conv_fwd<kC2, kC3, kCh3, false, true>(sm.h2, kT2, sm.o, kTo, kTo, frag + kFragL3 * 64, wave,
                                        lane);
  __syncthreads();
  // loss and dL/d out (one site per thread)
  double l2 = 0.0;
  {
    const float* t = tgt + ((int64_t)crop * kTo * kTo + tid) * kC3;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      float d = 0.f;
      if (c < kC3) {
        d = sm.o[tid * kC3 + c] - t[c];
        l2 += (double)d * d;
      }
      sm.dout[tid * 8 + c] = (__bf16)(dscale * d);
    }
  }
  double dummy = 0.0;
  block_sum2<256>(l2, dummy, sm.red);
  if (tid == 0) lpart[item] = l2;
  __syncthreads();
  float* gw = gpart + (int64_t)item * kNumW;
  conv_wgrad<kC2, kC3, 8>(sm.dout, sm.h2, kT2, kTo, kTo, gw + kOffW3, wave, lane);
  conv_dgrad<kC2, kC3, 8>(sm.dout, sm.h2, kT2, kT2, w + kOffW3, sm.dz2, wave, lane);
  __syncthreads();
  conv_wgrad<kC1, kC2, 16>(sm.dz2, sm.h1, kT1, kT2, kT2, gw + kOffW2, wave, lane);
  conv_dgrad<kC1, kC2, 16>(sm.dz2, sm.h1, kT1, kT1, w + kOffW2, sm.dz1, wave, lane);
  __syncthreads();
  conv_wgrad<kC0, kC1, 16>(sm.dz1, sm.x0, kT0, kT1, kT1, gw + kOffW1, wave, lane);
}

// grad[i] = sum over crops of gpart (fixed order); loss = sum lpart * lscale
__global__ void k_nn_reduce(const float* __restrict__ gpart, const double* __restrict__ lpart,
                            int ncrops, float* __restrict__ grad, double* __restrict__ loss,
                            double lscale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNumW) {
    float s = 0.f;
    for (int c = 0; c < ncrops; ++c) s += gpart[(int64_t)c * kNumW + i];
    grad[i] = s;
  }
  if (i == 0) {
    double l = 0.0;
    for (int c = 0; c < ncrops; ++c) l += lpart[c];
    *loss = l * lscale;
  }
}

__global__ void k_nn_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                          const float* __restrict__ g, float lr, float b1, float b2, float eps,
                          float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kNumW) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// training crops: input [crop][22*22][8] BF16 from the residual r (scaled by the
// column's RMS) and the link features; target [crop][16*16][4] = e / s on the
// crop's interior.  origin[crop] = (column, y0, x0) of the crop's input corner.
__global__ void k_nn_crops(const c64* __restrict__ r, const c64* __restrict__ e,
                           const c64* __restrict__ rr, double inv_n,
                           const __bf16* __restrict__ links, const int* __restrict__ origin,
                           int N, __bf16* __restrict__ in, float* __restrict__ tgt) {
  const int crop = blockIdx.x;
  const int col = origin[3 * crop], y0 = origin[3 * crop + 1], x0 = origin[3 * crop + 2];
  const double s2 = rr[col].re * inv_n;
  const double inv_s = s2 > 0.0 ? 1.0 / sqrt(s2) : 0.0;
  const int64_t off = (int64_t)col * N * N * 2;
  for (int idx = threadIdx.x; idx < kT0 * kT0; idx += blockDim.x) {
    const int ry = idx / kT0, rx = idx - ry * kT0;
    const int site = ((y0 + ry) % N) * N + (x0 + rx) % N;
    const c64 r0 = r[off + 2 * site], r1 = r[off + 2 * site + 1];
    __bf16* d = in + ((int64_t)crop * kT0 * kT0 + idx) * kC0;
    d[0] = (__bf16)(float)(r0.re * inv_s);
    d[1] = (__bf16)(float)(r0.im * inv_s);
    d[2] = (__bf16)(float)(r1.re * inv_s);
    d[3] = (__bf16)(float)(r1.im * inv_s);
    d[4] = links[site * 4 + 0];
    d[5] = links[site * 4 + 1];
    d[6] = links[site * 4 + 2];
    d[7] = links[site * 4 + 3];
    if (ry >= 3 && ry < 3 + kTo && rx >= 3 && rx < 3 + kTo) {
      const c64 e0 = e[off + 2 * site], e1 = e[off + 2 * site + 1];
      float* t = tgt + ((int64_t)crop * kTo * kTo + (ry - 3) * kTo + (rx - 3)) * kC3;
      t[0] = (float)(e0.re * inv_s);
      t[1] = (float)(e0.im * inv_s);
      t[2] = (float)(e1.re * inv_s);
      t[3] = (float)(e1.im * inv_s);
    }
  }
}

// FP32 crops (tests) -> BF16 inputs
__global__ void k_nn_round_inputs(const float* __restrict__ src, __bf16* __restrict__ dst,
                                  int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (__bf16)src[i];
}

}  // namespace

int nn_num_weights() { return kNumW; }
int nn_frag_count() { return kFrags * 64; }
int nn_crop_in_elems() { return kT0 * kT0 * kC0; }
int nn_crop_out_elems() { return kTo * kTo * kC3; }
int nn_crop_side() { return kT0; }

void nn_links(const double* theta, void* links, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_links, dim3(256), dim3(256), 0, s, theta, static_cast<__bf16*>(links),
                     N);
}

void nn_pack(const float* w, void* frag, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_pack, dim3((kFrags * 64 + 255) / 256), dim3(256), 0, s, w,
                     static_cast<bf8*>(frag));
}

void nn_apply(const c32* r, c32* x, const c64* rr, double inv_n, const void* links,
              const void* frag, int N, int nb, const int* active, hipStream_t s) {
  const int tiles_x = N / kTo;
  MLMC_LAUNCH(k_nn_apply, dim3(tiles_x * tiles_x, nb), dim3(256), 0, s, r, x, rr, inv_n,
              static_cast<const __bf16*>(links), static_cast<const bf8*>(frag), N, tiles_x,
              active, timing_log());
}

void nn_train_step(const void* in, const float* tgt, const int* order, int ncrops,
                   const void* frag, const float* w, float* gpart, double* lpart, float* grad,
                   double* loss, hipStream_t s) {
  const double count = (double)ncrops * kTo * kTo * kC3;
  MLMC_LAUNCH(k_nn_train, dim3(ncrops), dim3(256), 0, s, static_cast<const __bf16*>(in), tgt,
              order, static_cast<const bf8*>(frag), w, gpart, lpart, (float)(2.0 / count));
  hipLaunchKernelGGL(k_nn_reduce, dim3((kNumW + 255) / 256), dim3(256), 0, s, gpart, lpart,
                     ncrops, grad, loss, 1.0 / count);
}

void nn_adam(float* w, float* m, float* v, const float* g, double lr, double b1, double b2,
             double eps, int t, hipStream_t s) {
  const double c1 = 1.0 - std::pow(b1, t), c2 = 1.0 - std::pow(b2, t);
  hipLaunchKernelGGL(k_nn_adam, dim3((kNumW + 255) / 256), dim3(256), 0, s, w, m, v, g, (float)lr,
                     (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
}

void nn_crops(const c64* r, const c64* e, const c64* rr, double inv_n, const void* links,
              const int* origin, int ncrops, int N, void* in, float* tgt, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_crops, dim3(ncrops), dim3(256), 0, s, r, e, rr, inv_n,
                     static_cast<const __bf16*>(links), origin, N, static_cast<__bf16*>(in), tgt);
}

void nn_round_inputs(const float* src, void* dst, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_round_inputs, dim3(256), dim3(256), 0, s, src,
                     static_cast<__bf16*>(dst), count);
}

}  // namespace mlmc
