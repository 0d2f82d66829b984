// Allocation-free entry point (mlmc_smooth_noalloc): the smoother's working
// copies live in a fixed device array instead of memory allocated per call, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
#include <mutex>
#include <string>

#include "context.h"

namespace {

// One copy per device, held until the process ends.  Host code never takes its
// address directly: the array's name is a host-side stand-in, so the device
// address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)MLMC_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
bool g_done[kMaxDevices] = {};
void* g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};

}  // namespace

namespace mlmc {

void noalloc_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[dev]) return;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
  void* p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
  g_ptr[dev] = (e == hipSuccess) ? p : nullptr;
  g_err[dev] = e;
  g_done[dev] = true;
}

}  // namespace mlmc

extern "C" int mlmc_smooth_noalloc(mlmc_ctx* c, int level, int nrhs, int sweeps, int flags,
                                   const double* b_dev, double* x_dev, double* rc_dev) {
  mlmc::Context* ctx = reinterpret_cast<mlmc::Context*>(c);
  if (!ctx || !b_dev || !x_dev) return MLMC_EINVAL;
  try {
    const int dev = ctx->device();
    MLMC_REQUIRE(dev >= 0 && dev < kMaxDevices, MLMC_EDEVICE, "device index out of range");
    mlmc::noalloc_init(dev);  // normally done by mlmc_setup already
    void* ws = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      MLMC_REQUIRE(g_ptr[dev] != nullptr, MLMC_EDEVICE,
                   std::string("no device address of the fixed workspace: ") +
                       hipGetErrorString(g_err[dev]));
      ws = g_ptr[dev];
    }
    MLMC_REQUIRE(mlmc::smooth_flags_valid(flags), MLMC_EINVAL, "unknown smoother flags");
    ctx->smooth_fp64(level, nrhs, sweeps, (flags & MLMC_SMOOTH_REVERSE) != 0,
                     (flags & MLMC_SMOOTH_ZERO_START) != 0, b_dev, x_dev, rc_dev, ws,
                     kScratchBytes, mlmc::smooth_csr_tail(flags));
    ctx->last_error.clear();
    return MLMC_OK;
  } catch (const mlmc::Error& e) {
    ctx->last_error = e.what();
    return e.code;
  } catch (const std::exception& e) {
    ctx->last_error = e.what();
    return MLMC_EINVAL;
  }
}
