// The C ABI (include/mlmc.h): argument checks, exception-to-status mapping.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <new>
#include <vector>
#include <string>

#include "context.h"

using mlmc::Context;
using mlmc::Error;

namespace {

thread_local std::string g_setup_error;

template <typename F>
int guarded(Context* ctx, F&& f) {
  try {
    f();
    if (ctx) ctx->last_error.clear();
    return MLMC_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.what();
    else g_setup_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "host allocation failed";
    else g_setup_error = "host allocation failed";
    return MLMC_ENOMEM;
  } catch (const std::exception& e) {
    if (ctx) ctx->last_error = e.what();
    else g_setup_error = e.what();
    return MLMC_EINVAL;
  }
}

// the opaque handle of the C ABI is the context object itself
Context* as_ctx(mlmc_ctx* p) { return reinterpret_cast<Context*>(p); }
mlmc_ctx* as_handle(Context* p) { return reinterpret_cast<mlmc_ctx*>(p); }

}  // namespace

extern "C" {

int mlmc_default_options(mlmc_options* opt) {
  if (!opt) return MLMC_EINVAL;
  std::memset(opt, 0, sizeof(*opt));
  opt->precision = MLMC_FP32_IR64;
  opt->nb = 128;
  opt->nu_pre = 1;
  opt->nu_post = 1;
  opt->omega = 1.8;
  opt->alloc = MLMC_ALLOC_EQUAL;
  opt->rho_weights = nullptr;
  opt->solve_tol = 1e-10;
  opt->inner_tol = 0.0;  // automatic per operator kind
  opt->max_iter = 200;
  opt->max_refine = 8;
  opt->krylov_restart = 16;
  opt->min_samples = 5;
  opt->max_samples = (int64_t)1 << 22;
  opt->tau = 0.0;
  opt->learned = 0;
  opt->graphs = 0;
  opt->narrow_fp64 = 0;
  opt->top_cycles = 0;
  return MLMC_OK;
}

int mlmc_setup(const mlmc_operator* A, const mlmc_hierarchy* h, const mlmc_options* opt,
               void* hip_stream, mlmc_ctx** out_ctx) {
  if (!out_ctx) return MLMC_EINVAL;
  *out_ctx = nullptr;
  if (!A || !h) {
    g_setup_error = "null operator or hierarchy";
    return MLMC_EINVAL;
  }
  mlmc_options o;
  if (opt) o = *opt;
  else mlmc_default_options(&o);
  Context* ctx = nullptr;
  int rc = guarded(nullptr, [&] {
    ctx = new Context(*A, *h, o, static_cast<hipStream_t>(hip_stream));
    // the device's copy of the fixed workspace of the allocation-free entry
    // points, looked up once per device while it is current
    mlmc::noalloc_init(ctx->device());
  });
  if (rc == MLMC_OK) *out_ctx = as_handle(ctx);
  return rc;
}

int mlmc_trace(mlmc_ctx* c, double tol, uint64_t seed, mlmc_result* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->trace(tol, seed, out); });
}

int mlmc_hutchinson(mlmc_ctx* c, double tol, uint64_t seed, mlmc_result* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->hutchinson(tol, seed, out); });
}

int mlmc_sample_level(mlmc_ctx* c, int level, uint64_t seed, int64_t first, int64_t nsamples,
                      double* out, double* out_err) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->sample_level(level, seed, first, nsamples, out, out_err); });
}

int mlmc_coarse_trace(mlmc_ctx* c, double* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  out[0] = ctx->coarse_trace_re();
  out[1] = ctx->coarse_trace_im();
  return MLMC_OK;
}

int mlmc_level_size(mlmc_ctx* c, int level, int64_t* n) {
  Context* ctx = as_ctx(c);
  if (!ctx || !n) return MLMC_EINVAL;
  if (level < 1 || level > ctx->levels_solver()) {
    ctx->last_error = "level out of range";
    return MLMC_EINVAL;
  }
  *n = ctx->level_size(level);
  return MLMC_OK;
}

int mlmc_solve(mlmc_ctx* c, int level, int nrhs, const double* b_dev, double* y_dev,
               double* relres) {
  Context* ctx = as_ctx(c);
  if (!ctx || !b_dev || !y_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->solve_fp64(level, nrhs, b_dev, y_dev, relres, true); });
}

int mlmc_apply(mlmc_ctx* c, int level, int nrhs, const double* x_dev, double* y_dev) {
  Context* ctx = as_ctx(c);
  if (!ctx || !x_dev || !y_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->apply_fp64(level, nrhs, x_dev, y_dev); });
}

int mlmc_smooth(mlmc_ctx* c, int level, int nrhs, int sweeps, int flags, const double* b_dev,
                double* x_dev, double* rc_dev) {
  Context* ctx = as_ctx(c);
  if (!ctx || !b_dev || !x_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] {
    MLMC_REQUIRE(mlmc::smooth_flags_valid(flags), MLMC_EINVAL, "unknown smoother flags");
    ctx->smooth_fp64(level, nrhs, sweeps, (flags & MLMC_SMOOTH_REVERSE) != 0,
                     (flags & MLMC_SMOOTH_ZERO_START) != 0, b_dev, x_dev, rc_dev, nullptr, 0,
                     mlmc::smooth_csr_tail(flags));
  });
}

int mlmc_restrict(mlmc_ctx* c, int level, int nrhs, const double* x_dev, double* xc_dev) {
  Context* ctx = as_ctx(c);
  if (!ctx || !x_dev || !xc_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->restrict_fp64(level, nrhs, x_dev, xc_dev); });
}

int mlmc_prolong(mlmc_ctx* c, int level, int nrhs, const double* xc_dev, double* x_dev) {
  Context* ctx = as_ctx(c);
  if (!ctx || !x_dev || !xc_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->prolong_fp64(level, nrhs, xc_dev, x_dev); });
}

int mlmc_probes(mlmc_ctx* c, int level, uint64_t seed, int stream, int64_t first, int nrhs,
                double* out_dev) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out_dev) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->probes_fp64(level, seed, stream, first, nrhs, out_dev); });
}

int mlmc_export_coarse(mlmc_ctx* c, int which, double* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->export_coarse(which, out); });
}

int mlmc_export_prolongation(mlmc_ctx* c, int level, double* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->export_prolongation(level, out); });
}

int mlmc_export_csr(mlmc_ctx* c, int level, int64_t* nnz, int64_t* row_ptr, int32_t* col_idx,
                    double* vals, int32_t* agg, int32_t* colour) {
  Context* ctx = as_ctx(c);
  if (!ctx || !nnz) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->export_csr(level, nnz, row_ptr, col_idx, vals, agg, colour); });
}

int mlmc_export_level(mlmc_ctx* c, int level, int which, int64_t* rows, int64_t* cols,
                      int64_t* nnz, int64_t* row_ptr, int32_t* col_idx, double* vals) {
  Context* ctx = as_ctx(c);
  if (!ctx) return MLMC_EINVAL;
  return guarded(ctx, [&] {
    ctx->export_level(level, which, rows, cols, nnz, row_ptr, col_idx, vals);
  });
}

int mlmc_run_estimator(int levels, mlmc_sample_fn sample, mlmc_pilot_fn pilot, void* user,
                       const double* coarse, const double* cost, const mlmc_options* opt,
                       double tol, mlmc_result* out) {
  if (!sample || !opt || !out || levels < 2 || levels > MLMC_MAX_LEVELS) {
    g_setup_error = "invalid estimator arguments";
    return MLMC_EINVAL;
  }
  return guarded(nullptr, [&] {
    MLMC_REQUIRE(opt->nb >= 1, MLMC_EINVAL, "nb must be >= 1");
    MLMC_REQUIRE(opt->min_samples >= 2, MLMC_EINVAL, "min_samples must be >= 2");
    MLMC_REQUIRE(opt->max_samples >= opt->min_samples, MLMC_EINVAL,
                 "max_samples below min_samples");
    mlmc::SamplerIface smp;
    smp.sample = [&](int level, int64_t first, int64_t count, mlmc::c64* o) {
      int rc = sample(user, level, first, count, reinterpret_cast<double*>(o));
      MLMC_REQUIRE(rc == 0, rc < 0 ? rc : MLMC_EINVAL, "sampler callback failed");
      for (int64_t k = 0; k < count; ++k)
        MLMC_REQUIRE(std::isfinite(o[k].re) && std::isfinite(o[k].im), MLMC_ENOCONV,
                     "sampler returned a non-finite sample on level " +
                         std::to_string(level));
    };
    if (pilot) {
      smp.pilot = [&](int64_t count, mlmc::c64* o) {
        int rc = pilot(user, count, reinterpret_cast<double*>(o));
        MLMC_REQUIRE(rc == 0, rc < 0 ? rc : MLMC_EINVAL, "pilot callback failed");
      };
    }
    std::vector<double> cv(levels - 1, 1.0);
    if (cost)
      for (int l = 0; l < levels - 1; ++l) cv[l] = cost[l];
    mlmc::c64 cz = {coarse ? coarse[0] : 0.0, coarse ? coarse[1] : 0.0};
    mlmc::run_estimator(levels, smp, cz, cv, *opt, tol, out);
  });
}

int mlmc_set_allocator(mlmc_alloc_fn alloc, mlmc_free_fn free_fn, void* user) {
  if ((alloc == nullptr) != (free_fn == nullptr)) return MLMC_EINVAL;
  mlmc::alloc_hooks().alloc = alloc;
  mlmc::alloc_hooks().free_fn = free_fn;
  mlmc::alloc_hooks().user = user;
  return MLMC_OK;
}

int mlmc_learned_train(mlmc_ctx* c, const float* w_init, const mlmc_train_options* opt,
                       mlmc_train_report* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !w_init || !opt) return MLMC_EINVAL;
  return guarded(ctx, [&] {
    for (int i = 0; i < MLMC_NN_WEIGHTS; ++i)
      MLMC_REQUIRE(std::isfinite(w_init[i]), MLMC_EINVAL, "initial weights must be finite");
    ctx->nn_train(w_init, *opt, out);
  });
}

int mlmc_learned_set_weights(mlmc_ctx* c, const float* w) {
  Context* ctx = as_ctx(c);
  if (!ctx || !w) return MLMC_EINVAL;
  return guarded(ctx, [&] {
    for (int i = 0; i < MLMC_NN_WEIGHTS; ++i)
      MLMC_REQUIRE(std::isfinite(w[i]), MLMC_EINVAL, "weights must be finite");
    ctx->nn_set_weights(w);
  });
}

int mlmc_learned_get_weights(mlmc_ctx* c, float* w) {
  Context* ctx = as_ctx(c);
  if (!ctx || !w) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->nn_get_weights(w); });
}

int mlmc_learned_stats(mlmc_ctx* c, int64_t* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  out[0] = ctx->nn_stats[0];
  out[1] = ctx->nn_stats[1];
  return MLMC_OK;
}

int mlmc_nn_apply(mlmc_ctx* c, int nrhs, const double* r, double* e) {
  Context* ctx = as_ctx(c);
  if (!ctx || !r || !e) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->nn_apply_fp64(nrhs, r, e); });
}

int mlmc_nn_loss_grad(mlmc_ctx* c, int ncrops, const float* in, const float* target, double* loss,
                      float* grad) {
  Context* ctx = as_ctx(c);
  if (!ctx || !in || !target || !loss || !grad) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->nn_loss_grad(ncrops, in, target, loss, grad); });
}

int mlmc_nn_crops(mlmc_ctx* c, int nrhs, const double* r, const double* e, int ncrops,
                  const int32_t* origin, float* in, float* target) {
  Context* ctx = as_ctx(c);
  if (!ctx || !r || !e || !origin || !in || !target) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->nn_crops_fp64(nrhs, r, e, ncrops, origin, in, target); });
}

int mlmc_nn_adam_step(mlmc_ctx* c, const float* grad, double lr, int t) {
  Context* ctx = as_ctx(c);
  if (!ctx || !grad) return MLMC_EINVAL;
  return guarded(ctx, [&] {
    for (int i = 0; i < MLMC_NN_WEIGHTS; ++i)
      MLMC_REQUIRE(std::isfinite(grad[i]), MLMC_EINVAL, "gradient must be finite");
    ctx->nn_adam_step(grad, lr, t);
  });
}

int mlmc_deflation_setup(mlmc_ctx* c, const mlmc_deflation_options* opt,
                         mlmc_deflation_report* report) {
  Context* ctx = as_ctx(c);
  if (!ctx || !opt) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->deflation_setup(*opt, report); });
}

int mlmc_deflated_sample(mlmc_ctx* c, uint64_t seed, int64_t first, int64_t nsamples, double* out,
                         double* out_err) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->deflated_sample(seed, first, nsamples, out, out_err); });
}

int mlmc_deflated_hutchinson(mlmc_ctx* c, double tol, uint64_t seed, mlmc_result* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->deflated_hutchinson(tol, seed, out); });
}

int mlmc_deflation_export(mlmc_ctx* c, double* eigenvalues, double* vectors_dev, double* direct) {
  Context* ctx = as_ctx(c);
  if (!ctx) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->deflation_export(eigenvalues, vectors_dev, direct); });
}

int mlmc_batch_sample(mlmc_ctx* const* ctxs, int count, int level, const uint64_t* seeds,
                      int64_t first, int64_t nsamples, int workers, double* out,
                      double* seconds) {
  if (!ctxs || count < 1 || !seeds || !out || nsamples < 1 || first < 0 || workers < 1)
    return MLMC_EINVAL;
  std::vector<Context*> cs(count);
  for (int i = 0; i < count; ++i) {
    cs[i] = as_ctx(ctxs[i]);
    if (!cs[i]) return MLMC_EINVAL;
    for (int j = 0; j < i; ++j)
      if (cs[j] == cs[i]) return MLMC_EINVAL;  // a context serves one worker at a time
    if (level < 1 || level >= cs[i]->levels_mlmc()) return MLMC_EINVAL;
  }
  // longest first: order by the level's unknowns (the solve cost grows with it)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return cs[a]->level_size(level) > cs[b]->level_size(level);
  });
  std::vector<int> status(count, MLMC_OK);
  std::atomic<int> next{0};
  auto work = [&] {
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= count) return;
      const int i = order[t];
      Context* ctx = cs[i];
      const auto t0 = std::chrono::steady_clock::now();
      status[i] = guarded(ctx, [&] {
        MLMC_HIP(hipSetDevice(ctx->device()));
        ctx->sample_level(level, seeds[i], first, nsamples, out + (size_t)i * nsamples * 2,
                          nullptr);
      });
      if (seconds)
        seconds[i] =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
  };
  const int nw = std::min(workers, count);
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(work);
  work();
  for (auto& th : pool) th.join();
  for (int i = 0; i < count; ++i)
    if (status[i] != MLMC_OK) return status[i];
  return MLMC_OK;
}

int mlmc_batch_sample_grouped(mlmc_ctx* const* ctxs, int count, int level,
                              const uint64_t* seeds, int64_t first, int64_t nsamples, int mode,
                              double* out, int* status) {
  if (!ctxs || count < 1 || !seeds || !out || !status || nsamples < 1 || first < 0 ||
      (mode != 1 && mode != 2))
    return MLMC_EINVAL;
  std::vector<Context*> cs(count);
  for (int i = 0; i < count; ++i) {
    cs[i] = as_ctx(ctxs[i]);
    if (!cs[i]) return MLMC_EINVAL;
    for (int j = 0; j < i; ++j)
      if (cs[j] == cs[i]) return MLMC_EINVAL;
    status[i] = MLMC_OK;
  }
  const int rc = guarded(cs[0], [&] {
    MLMC_HIP(hipSetDevice(cs[0]->device()));
    mlmc::group_batch_sample(cs, level, seeds, first, nsamples, mode, out, status);
  });
  if (rc != MLMC_OK) return rc;
  for (int i = 0; i < count; ++i)
    if (status[i] != MLMC_OK) return status[i];
  return MLMC_OK;
}

int mlmc_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream) {
  if (!src_dev || !dst_dev || bytes % 16 != 0 || ((uintptr_t)src_dev | (uintptr_t)dst_dev) % 16)
    return MLMC_EINVAL;
  return guarded(nullptr, [&] {
    mlmc::stream_copy(src_dev, dst_dev, bytes, static_cast<hipStream_t>(hip_stream));
    MLMC_HIP(hipGetLastError());
  });
}

int mlmc_counters(mlmc_ctx* c, int64_t* out, int n) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out || n < 0 || n > 4) return MLMC_EINVAL;
  for (int i = 0; i < n; ++i) out[i] = ctx->counters[i];
  return MLMC_OK;
}

int mlmc_set_timing(mlmc_ctx* c, int mask, int stride) {
  Context* ctx = as_ctx(c);
  if (!ctx || stride < 1) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->set_timing((unsigned)mask, stride); });
}

int mlmc_kernel_stats(mlmc_ctx* c, int kernel, int fp64, double* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->kernel_stats(kernel, fp64, out); });
}

int mlmc_kernel_stats_level(mlmc_ctx* c, int kernel, int fp64, int level, double* out) {
  Context* ctx = as_ctx(c);
  if (!ctx || !out) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->kernel_stats(kernel, fp64, out, level); });
}

int mlmc_reset_kernel_stats(mlmc_ctx* c) {
  Context* ctx = as_ctx(c);
  if (!ctx) return MLMC_EINVAL;
  return guarded(ctx, [&] { ctx->reset_kernel_stats(); });
}

const char* mlmc_last_error(const mlmc_ctx* c) {
  const Context* ctx = reinterpret_cast<const Context*>(c);
  if (!ctx) return g_setup_error.c_str();
  return ctx->last_error.c_str();
}

const char* mlmc_status_string(int status) {
  switch (status) {
    case MLMC_OK: return "ok";
    case MLMC_EINVAL: return "invalid argument";
    case MLMC_ENOMEM: return "out of memory";
    case MLMC_EDEVICE: return "device error";
    case MLMC_ENOCONV: return "not converged";
    case MLMC_ESTATE: return "invalid state";
    case MLMC_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

void mlmc_destroy(mlmc_ctx* c) {
  try {
    delete as_ctx(c);
  } catch (...) {
  }
}

}  // extern "C"
