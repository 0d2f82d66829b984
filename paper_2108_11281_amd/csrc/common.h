// Shared device/host helpers: error handling, scalar types, Philox4x64-10,
// wave64 reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "../../include/mlmc.h"

namespace mlmc {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MLMC_HIP(call)                                                          \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::mlmc::Error(MLMC_EDEVICE, std::string(#call) + " failed: " +      \
                                            hipGetErrorString(e_));             \
  } while (0)

#define MLMC_REQUIRE(cond, code, msg)                                           \
  do {                                                                          \
    if (!(cond)) throw ::mlmc::Error((code), (msg));                            \
  } while (0)

// ---------------------------------------------------------------------------
// Scalars.  Real: float, double.  Complex: c32, c64 (interleaved re, im).
// ---------------------------------------------------------------------------
struct c32 {
  float re, im;
};
struct c64 {
  double re, im;
};

template <typename T> struct Traits;
template <> struct Traits<float> {
  using real = float;
  static constexpr bool is_complex = false;
};
template <> struct Traits<double> {
  using real = double;
  static constexpr bool is_complex = false;
};
template <> struct Traits<c32> {
  using real = float;
  static constexpr bool is_complex = true;
};
template <> struct Traits<c64> {
  using real = double;
  static constexpr bool is_complex = true;
};

#define HD __host__ __device__ __forceinline__

HD float zero_of(float) { return 0.f; }
HD double zero_of(double) { return 0.0; }
HD c32 zero_of(c32) { return {0.f, 0.f}; }
HD c64 zero_of(c64) { return {0.0, 0.0}; }

HD c32 operator+(c32 a, c32 b) { return {a.re + b.re, a.im + b.im}; }
HD c64 operator+(c64 a, c64 b) { return {a.re + b.re, a.im + b.im}; }
HD c32 operator-(c32 a, c32 b) { return {a.re - b.re, a.im - b.im}; }
HD c64 operator-(c64 a, c64 b) { return {a.re - b.re, a.im - b.im}; }
HD c32 operator-(c32 a) { return {-a.re, -a.im}; }
HD c64 operator-(c64 a) { return {-a.re, -a.im}; }
HD c32 operator*(c32 a, c32 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
HD c64 operator*(c64 a, c64 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
HD c32 operator*(float s, c32 a) { return {s * a.re, s * a.im}; }
HD c64 operator*(double s, c64 a) { return {s * a.re, s * a.im}; }
HD c32& operator+=(c32& a, c32 b) { a = a + b; return a; }
HD c64& operator+=(c64& a, c64 b) { a = a + b; return a; }
HD c32& operator-=(c32& a, c32 b) { a = a - b; return a; }
HD c64& operator-=(c64& a, c64 b) { a = a - b; return a; }

HD float conj_of(float a) { return a; }
HD double conj_of(double a) { return a; }
HD c32 conj_of(c32 a) { return {a.re, -a.im}; }
HD c64 conj_of(c64 a) { return {a.re, -a.im}; }

HD double abs2_of(float a) { return (double)a * a; }
HD double abs2_of(double a) { return a * a; }
HD double abs2_of(c32 a) { return (double)a.re * a.re + (double)a.im * a.im; }
HD double abs2_of(c64 a) { return a.re * a.re + a.im * a.im; }

// conj(a) * b accumulated in FP64, as (re, im)
HD void cdot_acc(double& re, double& im, float a, float b) { re += (double)a * b; }
HD void cdot_acc(double& re, double& im, double a, double b) { re += a * b; }
HD void cdot_acc(double& re, double& im, c32 a, c32 b) {
  re += (double)a.re * b.re + (double)a.im * b.im;
  im += (double)a.re * b.im - (double)a.im * b.re;
}
HD void cdot_acc(double& re, double& im, c64 a, c64 b) {
  re += a.re * b.re + a.im * b.im;
  im += a.re * b.im - a.im * b.re;
}

// scalar (given as FP64 re, im) times vector element, in T's precision
HD float scale_by(double re, double im, float a) { return (float)re * a; }
HD double scale_by(double re, double im, double a) { return re * a; }
HD c32 scale_by(double re, double im, c32 a) {
  c32 s = {(float)re, (float)im};
  return s * a;
}
HD c64 scale_by(double re, double im, c64 a) {
  c64 s = {re, im};
  return s * a;
}

// conversions between precisions
template <typename To, typename From> HD To convert(From a);
template <> HD float convert<float, double>(double a) { return (float)a; }
template <> HD double convert<double, float>(float a) { return (double)a; }
template <> HD double convert<double, double>(double a) { return a; }
template <> HD float convert<float, float>(float a) { return a; }
template <> HD c32 convert<c32, c64>(c64 a) { return {(float)a.re, (float)a.im}; }
template <> HD c64 convert<c64, c32>(c32 a) { return {(double)a.re, (double)a.im}; }
template <> HD c64 convert<c64, c64>(c64 a) { return a; }
template <> HD c32 convert<c32, c32>(c32 a) { return a; }
// real part (used for constants such as 1 given as c64)
template <> HD float convert<float, c64>(c64 a) { return (float)a.re; }
template <> HD double convert<double, c64>(c64 a) { return a.re; }
template <> HD c32 convert<c32, double>(double a) { return {(float)a, 0.f}; }
template <> HD c64 convert<c64, double>(double a) { return {a, 0.0}; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// key = (seed, problem); counter = (block, sample, level, stream).
// ---------------------------------------------------------------------------
struct u64x4 {
  uint64_t v[4];
};

HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

HD u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                       uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = mulhi64(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = mulhi64(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  u64x4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

struct ProbeKey {
  uint64_t seed, problem, sample, level, stream;
};

// Rademacher entry i: bit (i & 63) of word ((i >> 6) & 3) of block i >> 8.
HD double rademacher_entry(const ProbeKey& k, uint64_t i) {
  u64x4 w = philox4x64_10(i >> 8, k.sample, k.level, k.stream, k.seed, k.problem);
  uint64_t word = w.v[(i >> 6) & 3];
  return ((word >> (i & 63)) & 1ull) ? -1.0 : 1.0;
}
// Z4 entry i: 2-bit field 2*(i & 31) of word ((i >> 5) & 3) of block i >> 7;
// 0, 1, 2, 3 -> 1, i, -1, -i.
HD c64 z4_entry(const ProbeKey& k, uint64_t i) {
  u64x4 w = philox4x64_10(i >> 7, k.sample, k.level, k.stream, k.seed, k.problem);
  uint64_t word = w.v[(i >> 5) & 3];
  int f = (int)((word >> (2 * (i & 31))) & 3ull);
  c64 r;
  r.re = (f == 0) ? 1.0 : (f == 2 ? -1.0 : 0.0);
  r.im = (f == 1) ? 1.0 : (f == 3 ? -1.0 : 0.0);
  return r;
}

template <typename T> HD T probe_entry(const ProbeKey& k, uint64_t i);
template <> HD double probe_entry<double>(const ProbeKey& k, uint64_t i) {
  return rademacher_entry(k, i);
}
template <> HD float probe_entry<float>(const ProbeKey& k, uint64_t i) {
  return (float)rademacher_entry(k, i);
}
template <> HD c64 probe_entry<c64>(const ProbeKey& k, uint64_t i) { return z4_entry(k, i); }
template <> HD c32 probe_entry<c32>(const ProbeKey& k, uint64_t i) {
  c64 z = z4_entry(k, i);
  return {(float)z.re, (float)z.im};
}

// ---------------------------------------------------------------------------
// Block reduction of FP64 pairs for 256-thread blocks (4 waves of 64).
// Fixed order: lanes by xor-butterfly, then waves 0..3 in order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* lds) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    lds[2 * wid] = a;
    lds[2 * wid + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      sa += lds[2 * w];
      sb += lds[2 * w + 1];
    }
    a = sa;
    b = sb;
  }
}

}  // namespace mlmc
