// Hierarchy setup, V-cycle, Krylov solvers with FP64 iterative refinement, and
// the level-difference samples of the MLMC trace estimator.
#include "context.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace mlmc {

AllocHooks& alloc_hooks() {
  static AllocHooks h;
  return h;
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------
Context::Context(const mlmc_operator& A, const mlmc_hierarchy& h, const mlmc_options& o,
                 hipStream_t s)
    : kind_(A.kind), op_(A), h_(h), opt_(o), s_(s) {
  hooks_ = alloc_hooks();
  MLMC_HIP(hipGetDevice(&device_));
  op_.field = nullptr;  // caller memory is not kept
  op_.row_ptr = nullptr;
  op_.col_idx = nullptr;
  op_.vals = nullptr;
  h_.agg = nullptr;
  h_.P = nullptr;
  Ls_ = h.levels_solver;
  L_ = h.levels_mlmc;
  nb_ = o.nb;
  MLMC_REQUIRE(Ls_ >= 2 && Ls_ <= MLMC_MAX_LEVELS, MLMC_EINVAL,
               "levels_solver must be in [2, 16]");
  MLMC_REQUIRE(L_ >= 2 && L_ <= Ls_, MLMC_EINVAL, "levels_mlmc must be in [2, levels_solver]");
  MLMC_REQUIRE(nb_ >= 1 && nb_ <= 1024, MLMC_EINVAL, "nb must be in [1, 1024]");
  MLMC_REQUIRE(o.precision == MLMC_FP64 || o.precision == MLMC_FP32_IR64, MLMC_EINVAL,
               "unknown precision");
  MLMC_REQUIRE(o.solve_tol > 0 && o.inner_tol >= 0, MLMC_EINVAL,
               "solve_tol must be > 0 and inner_tol >= 0");
  // inner_tol 0: the measured best per solver -- 1e-3 for the refined CG of the
  // real operators, 1e-2 for the complex FGMRES restart cycles
  if (opt_.inner_tol == 0.0)
    opt_.inner_tol = (A.kind == MLMC_WILSON2D || A.kind == MLMC_GAUGE2D) ? 1e-2 : 1e-3;
  MLMC_REQUIRE(o.top_cycles >= 0 && o.top_cycles <= 2, MLMC_EINVAL, "top_cycles must be 0, 1 or 2");
  // top_cycles 0: two coarse-grid cycles below the top level for the 2D Poisson
  // operator with at least two pre- and post-smoothing sweeps (measured faster),
  // one elsewhere.  The second cycle gives the coarse solve M2 = 2M - M A M, and
  // M2 A = I - (I - M A)^2 is positive definite only while every eigenvalue of
  // M A stays below 2: with one sweep on each side and over-correction 1.8 the
  // 2D V-cycle's largest eigenvalue of M A is about 2.4 on hierarchies of five
  // and more levels (1.45 with two sweeps), so CG would then run with an
  // indefinite preconditioner and some columns stall
  const bool two_sweeps = o.nu_pre >= 2 && o.nu_post >= 2;
  top_cycles_ = o.top_cycles > 0 ? o.top_cycles
                                 : (A.kind == MLMC_POISSON2D && two_sweeps ? 2 : 1);
  MLMC_REQUIRE(o.max_iter >= 1 && o.max_refine >= 1, MLMC_EINVAL, "iteration limits < 1");
  MLMC_REQUIRE(o.nu_pre >= 0 && o.nu_post >= 0, MLMC_EINVAL, "negative sweep count");
  MLMC_REQUIRE(o.min_samples >= 2, MLMC_EINVAL, "min_samples must be >= 2");
  MLMC_REQUIRE(o.alloc >= 0 && o.alloc <= 2, MLMC_EINVAL, "unknown allocation rule");
  MLMC_REQUIRE(!o.learned || (A.kind == MLMC_WILSON2D && o.precision == MLMC_FP32_IR64 &&
                              A.n_side % 16 == 0),
               MLMC_EUNSUPPORTED,
               "the learned smoother needs WILSON2D, MLMC_FP32_IR64 and a side divisible by 16");
  try {
    switch (kind_) {
      case MLMC_POISSON2D:
        omega_ = opt_.omega > 0 ? opt_.omega : 1.8;
        build_poisson();
        break;
      case MLMC_VARCOEF3D:
        varcoef_ = true;
        omega_ = opt_.omega > 0 ? opt_.omega : 1.8;
        build_varcoef(A.field);
        break;
      case MLMC_CSR:
        csr_ = true;
        omega_ = opt_.omega > 0 ? opt_.omega : 1.0;
        build_csr(A, h.agg, h.P);
        break;
      case MLMC_WILSON2D:
      case MLMC_GAUGE2D:
        complex_ = true;
        omega_ = opt_.omega > 0 ? opt_.omega : 1.0;
        build_wilson(A.field);
        break;
      default:
        throw Error(MLMC_EUNSUPPORTED, "operator kind not supported");
    }
  } catch (...) {
    for (void* p : allocs_) {
      if (hooks_.free_fn) hooks_.free_fn(p, hooks_.user);
      else (void)hipFree(p);
    }
    allocs_.clear();
    if (count_host_) (void)hipHostFree(count_host_);
    if (host_c64_) (void)hipHostFree(host_c64_);
    count_host_ = nullptr;
    host_c64_ = nullptr;
    throw;
  }
}

Context::~Context() {
  (void)hipStreamSynchronize(s_);
  for (auto& kv : graphs_) (void)hipGraphExecDestroy(kv.second.ex);
  if (cap_s_) (void)hipStreamDestroy(cap_s_);
  for (const Pending& p : pending_) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
  for (hipEvent_t e : fg_ev_)
    if (e) (void)hipEventDestroy(e);
  for (void* p : allocs_) {
    if (hooks_.free_fn) hooks_.free_fn(p, hooks_.user);
    else (void)hipFree(p);
  }
  if (count_host_) (void)hipHostFree(count_host_);
  if (host_c64_) (void)hipHostFree(host_c64_);
}

void* Context::dalloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (hooks_.alloc) {
    p = hooks_.alloc(bytes, hooks_.user);
    MLMC_REQUIRE(p != nullptr, MLMC_ENOMEM, "device allocation failed");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    MLMC_REQUIRE(e == hipSuccess, MLMC_ENOMEM,
                 std::string("hipMalloc failed: ") + hipGetErrorString(e));
  }
  allocs_.push_back(p);
  return p;
}

void Context::dfree(void* p) {
  if (!p) return;
  auto it = std::find(allocs_.begin(), allocs_.end(), p);
  if (it == allocs_.end()) return;
  MLMC_HIP(hipStreamSynchronize(s_));
  allocs_.erase(it);
  if (hooks_.free_fn) hooks_.free_fn(p, hooks_.user);
  else (void)hipFree(p);
}

template <> Work<float>& Context::work<float>() {
  MLMC_REQUIRE(w32_.x != nullptr, MLMC_ESTATE, "FP32 work vectors exist in MLMC_FP32_IR64 mode only");
  return w32_;
}
template <> Work<double>& Context::work<double>() {
  MLMC_REQUIRE(w64_.x != nullptr, MLMC_ESTATE, "FP64 work vectors exist in MLMC_FP64 mode only");
  return w64_;
}

// work vectors for batches of up to `width` columns (0: nb)
template <typename T>
void Context::alloc_work(Work<T>& w, int width) {
  const int cols = width > 0 ? std::min(width, nb_) : nb_;
  const int64_t n1 = lv_[0].n * cols;
  w.x = dalloc_n<T>(n1);
  w.r = dalloc_n<T>(n1);
  w.z = dalloc_n<T>(n1);
  w.p = dalloc_n<T>(n1);
  w.p2 = dalloc_n<T>(n1);
  w.q = dalloc_n<T>(n1);
  w.vb.assign(Ls_, nullptr);
  w.vx.assign(Ls_, nullptr);
  w.vt.assign(Ls_, nullptr);
  w.vr2.assign(Ls_, nullptr);
  w.ve2.assign(Ls_, nullptr);
  for (int m = 0; m < Ls_; ++m) {
    if (m > 0) {
      w.vb[m] = dalloc_n<T>(lv_[m].n * cols);
      w.vx[m] = dalloc_n<T>(lv_[m].n * cols);
    }
    if (m < Ls_ - 1) w.vt[m] = dalloc_n<T>(lv_[m].n * cols);
    if (top_cycles_ == 2 && m > 0 && m < Ls_ - 1 && (varcoef_ || csr_)) {
      w.vr2[m] = dalloc_n<T>(lv_[m].n * cols);
      w.ve2[m] = dalloc_n<T>(lv_[m].n * cols);
    }
  }
}

// Invert A_level densely in FP64 (Gauss-Jordan with partial pivoting on the
// device).  Returns the row-major inverse and its trace.
void Context::invert_coarse(int level, double** inv_out, c64* trace_out) {
  const Level& L = lv_[level - 1];
  MLMC_REQUIRE(L.n <= 16384, MLMC_EINVAL,
               "coarsest level too large for a dense inverse (n > 16384)");
  const int n = (int)L.n;
  double* aug = dalloc_n<double>(2 * (int64_t)n * n);  // the builders' layout: n x 2n
  switch (kind_) {
    case MLMC_POISSON2D:
      poisson_dense_build<double>(aug, L.side, L.d, L.c, s_);
      break;
    case MLMC_VARCOEF3D:
      varcoef_dense(L.kf64, L.dg64, L.side, aug, s_);
      break;
    case MLMC_CSR:
      csr_dense(L.A64, aug, s_);
      break;
    default:
      throw Error(MLMC_EUNSUPPORTED, "dense build");
  }
  double* inv = dalloc_n<double>((int64_t)n * n);
  dense_invert_checked<double>(aug, n, inv);
  dense_trace<double>(inv, n, scal_[kTmp], s_);
  MLMC_HIP(hipMemcpyAsync(host_c64_, scal_[kTmp], sizeof(c64), hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  *trace_out = host_c64_[0];
  *inv_out = inv;
  dfree(aug);
}

// out = A^{-1} for the n x n matrix in the left half of aug (n x 2n, row-major;
// overwritten); a singular A is an error
template <typename T>
void Context::dense_invert_checked(T* aug, int n, T* out) {
  T* rowbuf = dalloc_n<T>(kGjPanel + 1);
  T* colbuf = dalloc_n<T>(n);
  T* tbuf = dalloc_n<T>((int64_t)kGjPanel * n);
  int* ipiv = dalloc_n<int>(2 * (int64_t)n + 1);
  dense_inverse<T>(aug, n, 2 * (int64_t)n, out, rowbuf, colbuf, tbuf, ipiv, s_);
  int singular = 0;
  MLMC_HIP(hipMemcpyAsync(&singular, ipiv + 2 * (int64_t)n, sizeof(int), hipMemcpyDeviceToHost,
                          s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  dfree(ipiv);
  dfree(tbuf);
  dfree(colbuf);
  dfree(rowbuf);
  MLMC_REQUIRE(!singular, MLMC_EINVAL, "coarsest-level matrix is singular (zero pivot)");
}
template void Context::dense_invert_checked<double>(double*, int, double*);
template void Context::dense_invert_checked<c64>(c64*, int, c64*);

// device/pinned buffers shared by every operator kind: reduction partials,
// per-column scalars, flags and the FP64 sample-batch vectors (complex: two
// doubles per unknown)
void Context::alloc_common() {
  const int64_t n1 = lv_[0].n;
  const int64_t elem = complex_ ? 2 : 1;
  // per-column partial sums: enough for one partial per 256-thread block of
  // the finest level (stencil kernels with fused dots) or kMaxPartials
  const int64_t per_col = std::max<int64_t>(kMaxPartials, (n1 + kThreads - 1) / kThreads);
  // complex operators: the FGMRES multi-dot writes up to 256 partials for each
  // of the m+1 basis vectors of every column
  const int64_t cap = std::max<int64_t>(per_col * nb_, complex_ ? 256LL * nb_ * (m_ + 1) : 0);
  partials_ = dalloc_n<c64>(cap);
  partials_cap_ = cap;
  c64* sc = dalloc_n<c64>((int64_t)kNumScalars * nb_);
  for (int i = 0; i < kNumScalars; ++i) scal_[i] = sc + (int64_t)i * nb_;
  act_outer_ = dalloc_n<int>(nb_);
  act_inner_ = dalloc_n<int>(nb_);
  count_dev_ = dalloc_n<int>(8);
  MLMC_HIP(hipHostMalloc((void**)&count_host_, 8 * sizeof(int), hipHostMallocMapped));
  MLMC_HIP(hipHostGetDevicePointer((void**)&count_map_, count_host_, 0));
  MLMC_HIP(hipHostMalloc((void**)&host_c64_, 8 * (size_t)nb_ * sizeof(c64)));
  b1_ = dalloc_n<double>(n1 * nb_ * elem);
  y1_ = dalloc_n<double>(n1 * nb_ * elem);
  b2_ = dalloc_n<double>(lv_[1].n * nb_ * elem);
  y2_ = dalloc_n<double>(lv_[1].n * nb_ * elem);
  r64_ = dalloc_n<double>(n1 * nb_ * elem);
}

void Context::build_poisson() {
  MLMC_REQUIRE(op_.n_side >= 2, MLMC_EINVAL, "n_side must be >= 2");
  MLMC_REQUIRE(op_.diag > 0 && op_.off >= 0 && op_.diag >= 4 * op_.off, MLMC_EINVAL,
               "POISSON2D needs diag >= 4*off >= 0 (positive definite)");
  lv_.resize(Ls_);
  int side = op_.n_side;
  double d = op_.diag, c = op_.off;
  for (int l = 0; l < Ls_; ++l) {
    if (l > 0) {
      MLMC_REQUIRE(side % 2 == 0, MLMC_EINVAL,
                   "grid side not divisible by 2 at level " + std::to_string(l));
      side /= 2;
      // Galerkin of the 5-point stencil with orthonormal 2x2 aggregation:
      // diagonal block sum (4d - 8c)/4, coupling across an edge 2(-c)/4.
      const double dn = d - 2.0 * c, cn = 0.5 * c;
      d = dn;
      c = cn;
    }
    Level& L = lv_[l];
    L.index = l + 1;
    L.side = side;
    L.dof = 1;
    L.n = (int64_t)side * side;
    L.d = d;
    L.c = c;
  }
  MLMC_REQUIRE(lv_[Ls_ - 1].n <= 16384, MLMC_EINVAL, "coarsest solver level larger than 128^2");
  finish_real_build();
  tune_poisson();
}

// Autotuner of the fused Poisson sweep: per smoothed level with N >= 64, time
// the heaviest form (input iterate, folded coarse correction, as many fused
// sweeps as the post-smoother's first pass) over all nb columns for each
// compiled segment length and keep the fastest.  The swept
// values do not depend on the choice; the fused r^T z partial sums are grouped
// by segment, so the FP32 recursion can differ in its last bits (the FP64
// judged solution still meets solve_tol).  Runs once at setup on the library's
// work vectors.
void Context::tune_poisson() {
  hipEvent_t a = event(), b = event();
  auto tune = [&](auto tag, Level& L, int slot, int l) {
    using T = decltype(tag);
    Work<T>& w = work<T>();
    int opts[3];
    gs_rows_options<T>(opts);
    // the pass the post-smoother starts with (the heaviest form)
    const int sw = std::min(sweeps_per_pass(l), std::max(1, opt_.nu_post));
    // the default segment length is kept unless another is at least 10% faster,
    // so that the choice (which sets the grouping of the sweep's fused partial
    // sums, hence the last bits of the FP32 recursion) does not flap between runs
    const int dflt = L.gs_rows[slot];
    float best = 1e30f, t_dflt = 1e30f;
    int best_rows = dflt;
    for (int rows : opts) {
      float ms = 1e30f;  // best of 5 after a warm-up run (robust to noise)
      for (int rep = 0; rep < 6; ++rep) {
        MLMC_HIP(hipEventRecord(a, s_));
        poisson_rbgs_fused<T>(w.z, w.r, w.q, w.vb[l], omega_, L.side, L.d, L.c, nb_, nullptr,
                              true, nullptr, rows, sw, s_);
        MLMC_HIP(hipEventRecord(b, s_));
        MLMC_HIP(hipEventSynchronize(b));
        float t = 0.f;
        MLMC_HIP(hipEventElapsedTime(&t, a, b));
        if (rep > 0) ms = std::min(ms, t);
      }
      if (rows == dflt) t_dflt = ms;
      if (ms < best) {
        best = ms;
        best_rows = rows;
      }
    }
    L.gs_rows[slot] = best < 0.90f * t_dflt ? best_rows : dflt;
  };
  for (int l = 1; l < Ls_; ++l) {
    Level& L = lv_[l - 1];
    if (L.side < 64) continue;
    if (opt_.precision == MLMC_FP32_IR64) tune(float(), L, 0, l);
    if (opt_.precision == MLMC_FP64) tune(double(), L, 1, l);
  }
  ev_pool_.push_back(a);
  ev_pool_.push_back(b);
}

// 3D diffusion with face coefficients: every level keeps the 7-point form, the
// next level's faces being 1/8 of the sum of the four fine faces they cover
// (orthonormal 2x2x2 aggregation, Galerkin) and the shift carrying over.
void Context::build_varcoef(const double* k) {
  MLMC_REQUIRE(k != nullptr, MLMC_EINVAL, "VARCOEF3D needs face coefficients in field");
  MLMC_REQUIRE(op_.n_side >= 2 && op_.n_side <= 1024, MLMC_EINVAL, "n_side must be in [2, 1024]");
  MLMC_REQUIRE(std::isfinite(op_.shift) && op_.shift >= 0, MLMC_EINVAL, "shift must be >= 0");
  const int N = op_.n_side;
  const int64_t nf = 3LL * N * N * (N + 1);
  double kmin = INFINITY;
  for (int64_t t = 0; t < nf; ++t) {
    MLMC_REQUIRE(std::isfinite(k[t]) && k[t] >= 0, MLMC_EINVAL,
                 "face coefficients must be finite and >= 0");
    kmin = std::min(kmin, k[t]);
  }
  MLMC_REQUIRE(op_.shift > 0 || kmin > 0, MLMC_EINVAL,
               "VARCOEF3D needs shift > 0 or positive faces (positive definite)");
  lv_.resize(Ls_);
  int side = N;
  for (int l = 0; l < Ls_; ++l) {
    if (l > 0) {
      MLMC_REQUIRE(side % 2 == 0, MLMC_EINVAL,
                   "grid side not divisible by 2 at level " + std::to_string(l));
      side /= 2;
    }
    Level& L = lv_[l];
    L.index = l + 1;
    L.side = side;
    L.dof = 1;
    L.n = (int64_t)side * side * side;
    const int64_t f = 3LL * side * side * (side + 1);
    const int64_t fl = 3 * (L.n + (int64_t)side * side);
    L.kf64 = dalloc_n<double>(f);
    L.kl64 = dalloc_n<double>(fl);
    L.kl32 = dalloc_n<float>(fl);
    L.dg64 = dalloc_n<double>(L.n);
    L.dg32 = dalloc_n<float>(L.n);
  }
  MLMC_REQUIRE(lv_[Ls_ - 1].n <= 16384, MLMC_EINVAL, "coarsest solver level larger than 16384");
  MLMC_HIP(hipMemcpyAsync(lv_[0].kf64, k, sizeof(double) * (size_t)nf, hipMemcpyHostToDevice, s_));
  for (int l = 0; l < Ls_; ++l) {
    Level& L = lv_[l];
    if (l > 0) varcoef_coarsen(lv_[l - 1].kf64, L.kf64, lv_[l - 1].side, s_);
    varcoef_diag(L.kf64, op_.shift, L.side, L.dg64, L.dg32, L.kl64, L.kl32, s_);
  }
  finish_real_build();
  tune_varcoef();
}

// Autotuner of the 3D stencil kernels: per smoothed level, time one full
// red-black sweep over all nb columns with 1, 2, 4 and 8 right-hand sides per
// thread (the results are identical; only the load reuse of the couplings and
// the parallelism differ) and keep the fastest; on even sides up to 128 the
// sweeps run as the fused out-of-place pass instead, whose columns per wave
// (1 or 2) are tuned the same way.
// Runs once at setup on the library's own work vectors.
void Context::tune_varcoef() {
  const bool fp32 = opt_.precision == MLMC_FP32_IR64;
  hipEvent_t a = event(), b = event();
  for (int l = 1; l < Ls_; ++l) {
    Level& L = lv_[l - 1];
    float best = 1e30f;
    int best_cols = 4;
    for (int cols : {1, 2, 4, 8}) {
      float ms = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        MLMC_HIP(hipEventRecord(a, s_));
        if (fp32)
          varcoef_rbgs<float>(w32_.r, w32_.x, L.kl32, L.dg32, L.side, nb_, cols, nullptr,
                              rep == 0, false, nullptr, 0.0, s_);
        else
          varcoef_rbgs<double>(w64_.r, w64_.x, L.kl64, L.dg64, L.side, nb_, cols, nullptr,
                               rep == 0, false, nullptr, 0.0, s_);
        MLMC_HIP(hipEventRecord(b, s_));
        MLMC_HIP(hipEventSynchronize(b));
        float t = 0.f;
        MLMC_HIP(hipEventElapsedTime(&t, a, b));
        if (rep > 0) ms += t;  // the first run warms caches and code
      }
      if (ms < best) {
        best = ms;
        best_cols = cols;
      }
    }
    L.cols = best_cols;
    // the fused out-of-place sweep (even sides up to 128) replaces the in-place
    // pair of colour launches; tune its columns per wave
    L.mcols = 0;
    if (varcoef_march_ok(L.side)) {
      float mbest = 1e30f;
      for (int cols : {1, 2}) {
        float ms = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
          MLMC_HIP(hipEventRecord(a, s_));
          if (fp32)
            varcoef_rbgs_march<float>(rep == 0 ? nullptr : w32_.x, w32_.r, w32_.z, nullptr, 0.0,
                                      L.kl32, L.dg32, L.side, nb_, cols, nullptr, false, s_);
          else
            varcoef_rbgs_march<double>(rep == 0 ? nullptr : w64_.x, w64_.r, w64_.z, nullptr,
                                       0.0, L.kl64, L.dg64, L.side, nb_, cols, nullptr, false,
                                       s_);
          MLMC_HIP(hipEventRecord(b, s_));
          MLMC_HIP(hipEventSynchronize(b));
          float t = 0.f;
          MLMC_HIP(hipEventElapsedTime(&t, a, b));
          if (rep > 0) ms += t;
        }
        if (ms < mbest) {
          mbest = ms;
          L.mcols = cols;
        }
      }
    }
  }
  ev_pool_.push_back(a);
  ev_pool_.push_back(b);
}

// work buffers and coarsest inverses of a real symmetric positive definite
// operator (POISSON2D, VARCOEF3D)
void Context::finish_real_build() {
  const int64_t n1 = lv_[0].n;
  alloc_common();
  // the FP64 Krylov / V-cycle vectors serve the plain FP64 mode only; the
  // refined FP32 mode keeps its FP64 iterate in the sample-batch buffers
  if (opt_.precision == MLMC_FP64) alloc_work(w64_);
  MLMC_REQUIRE(opt_.narrow_fp64 >= 0, MLMC_EINVAL, "narrow_fp64 must be >= 0");
  if (opt_.precision == MLMC_FP32_IR64 && opt_.narrow_fp64 > 0)
    alloc_work(w64_, opt_.narrow_fp64);
  if (opt_.precision == MLMC_FP32_IR64) {
    alloc_work(w32_);
    r32_ = dalloc_n<float>(n1 * nb_);
    d32_ = dalloc_n<float>(n1 * nb_);
    if (kind_ == MLMC_POISSON2D) b32_ = dalloc_n<float>(n1 * nb_);
  }

  // coarsest inverses (FP64 on the device), the direct trace term (Remark 4.2)
  c64 tr_s;
  invert_coarse(Ls_, &ainv_solver_, &tr_s);
  // the transposed inverse, zero-padded to a multiple of 16 so that the MFMA
  // tile kernel applies it for any coarsest size, in that kernel's layout
  const int ns = (int)lv_[Ls_ - 1].n;
  const int ld = (ns + 15) / 16 * 16;
  double* plain = dalloc_n<double>((int64_t)ld * ld);
  w64_.ld = w32_.ld = ld;
  if (ld == ns) {
    dense_transpose<double>(ainv_solver_, plain, ns, s_);
  } else {
    double* t = dalloc_n<double>((int64_t)ns * ns);
    dense_transpose<double>(ainv_solver_, t, ns, s_);
    vec_zero<double>(plain, (int64_t)ld * ld, 1, nullptr, s_);
    MLMC_HIP(hipMemcpy2DAsync(plain, sizeof(double) * ld, t, sizeof(double) * ns,
                              sizeof(double) * ns, ns, hipMemcpyDeviceToDevice, s_));
    dfree(t);
  }
  static_assert(dense_mfma_layout<double>(16) && dense_mfma_layout<float>(16),
                "the padded inverse is applied by the MFMA tile kernel");
  w64_.ainvT = dalloc_n<double>((int64_t)ld * ld);
  dense_pack4<double>(plain, w64_.ainvT, ld, s_);
  dfree(plain);
  if (opt_.precision == MLMC_FP32_IR64) {
    w32_.ainvT = dalloc_n<float>((int64_t)ld * ld);
    vec_convert<float, double>(w64_.ainvT, w32_.ainvT, (int64_t)ld * ld, 1, nullptr, s_);
  }
  if (L_ == Ls_) {
    coarse_trace_ = tr_s;
  } else {
    invert_coarse(L_, &ainv_mlmc_, &coarse_trace_);
  }
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// operator dispatch
// ---------------------------------------------------------------------------
template <> const float* Context::vc_faces<float>(int l) const { return lv_[l - 1].kl32; }
template <> const double* Context::vc_faces<double>(int l) const { return lv_[l - 1].kl64; }
template <> const float* Context::vc_diag<float>(int l) const { return lv_[l - 1].dg32; }
template <> const double* Context::vc_diag<double>(int l) const { return lv_[l - 1].dg64; }

int Context::op_tiles(int l) const {
  const Level& L = lv_[l - 1];
  if (csr_) return csr_blocks((int)L.n);
  return varcoef_ ? varcoef_blocks(L.side) : poisson_march_tiles(L.side);
}

template <typename T>
void Context::op_apply(int l, const T* x, T* y, int nb, const int* act, c64* partials) {
  const Level& L = lv_[l - 1];
  if (csr_)
    csr_residual<T, T, T>(nullptr, x, y, csr_mat<T>(l), nb, csr_cols(L, nb), act, partials, s_);
  else if (varcoef_)
    varcoef_residual<T, T, T>(nullptr, x, y, vc_faces<T>(l), vc_diag<T>(l), L.side, nb, L.cols,
                              act, partials, s_);
  else
    poisson_apply<T>(x, y, L.side, L.d, L.c, nb, act, partials, s_);
}

template <typename Tb, typename Tx, typename Tr>
void Context::op_residual(int l, const Tb* b, const Tx* x, Tr* r, int nb, const int* act,
                          c64* partials) {
  const Level& L = lv_[l - 1];
  if (csr_)
    csr_residual<Tb, Tx, Tr>(b, x, r, csr_mat<Tx>(l), nb, csr_cols(L, nb), act, partials, s_);
  else if (varcoef_)
    varcoef_residual<Tb, Tx, Tr>(b, x, r, vc_faces<Tx>(l), vc_diag<Tx>(l), L.side, nb, L.cols,
                                 act, partials, s_);
  else
    poisson_residual<Tb, Tx, Tr>(b, x, r, L.side, L.d, L.c, nb, act, partials, s_);
}

template <typename T>
void Context::op_update_apply(int l, const T* p_old, const T* z, const c64* beta, T* p_new,
                              T* q, int nb, const int* act) {
  const Level& L = lv_[l - 1];
  if (csr_)
    csr_update_apply<T>(p_old, z, beta, p_new, q, csr_mat<T>(l), nb, csr_cols(L, nb), act,
                        partials_, s_);
  else if (varcoef_)
    varcoef_update_apply<T>(p_old, z, beta, p_new, q, vc_faces<T>(l), vc_diag<T>(l), L.side, nb,
                            L.cols, act, partials_, s_);
  else
    poisson_update_apply<T>(p_old, z, beta, p_new, q, L.side, L.d, L.c, nb, act, partials_, s_);
}

template <typename T>
void Context::op_res_restrict(int l, const T* b, const T* x, T* rc, int nb, const int* act) {
  const Level& L = lv_[l - 1];
  if (csr_ && general_) {
    T* r = work<T>().vt[l - 1];
    csr_residual<T, T, T>(b, x, r, csr_mat<T>(l), nb, csr_cols(L, nb), act, nullptr, s_);
    csr_spmm<T>(r, rc, csr_R<T>(l), 1.0, 0.0, nb, csr_cols(L, nb), act, s_);
  } else if (csr_) {
    csr_restrict<T>(b, x, rc, work<T>().vt[l - 1], csr_mat<T>(l), csr_agg<T>(l), nb,
                    csr_cols(L, nb), act, s_);
  }
  else if (varcoef_)
    varcoef_restrict<T>(b, x, rc, vc_faces<T>(l), vc_diag<T>(l), L.side, true, nb, L.cols, act,
                        s_);
  else
    poisson_residual_restrict<T>(b, x, rc, L.side, L.d, L.c, nb, act, s_);
}

template <typename T>
void Context::op_prolong(int l, const T* ec, T* x, int nb, const int* act, double beta) {
  const Level& L = lv_[l - 1];
  const double w = beta == 0.0 ? 1.0 : omega_;
  if (csr_ && general_)
    csr_spmm<T>(ec, x, csr_P<T>(l), w, beta, nb, csr_cols(L, nb), act, s_);
  else if (csr_)
    csr_prolong<T>(ec, x, csr_agg<T>(l), (int)L.n, w, beta, nb, act, s_);
  else if (varcoef_)
    varcoef_prolong<T>(ec, x, L.side, w, beta, nb, act, s_);
  else
    agg2d_prolong<T>(ec, x, L.side, w, beta, nb, act, s_);
}

template <typename T>
void Context::op_restrict(int l, const T* x, T* xc, int nb, const int* act) {
  const Level& L = lv_[l - 1];
  if (csr_ && general_)
    csr_spmm<T>(x, xc, csr_R<T>(l), 1.0, 0.0, nb, csr_cols(L, nb), act, s_);
  else if (csr_)
    csr_restrict<T>(nullptr, x, xc, nullptr, csr_mat<T>(l), csr_agg<T>(l), nb, csr_cols(L, nb),
                    act, s_);
  else if (varcoef_)
    varcoef_restrict<T>(nullptr, x, xc, nullptr, nullptr, L.side, false, nb, L.cols, act, s_);
  else
    agg2d_restrict<T>(x, xc, L.side, nb, act, s_);
}

// The second coarse-grid cycle, ec += V(bc - A ec) on level l + 1.  The 2D
// Poisson V-cycle runs it as one V-cycle on bc whose pre-smoothing starts from
// ec: Gauss-Seidel sweeps, the residual and the coarse correction are affine in
// the iterate, so that V-cycle equals ec + V(bc - A ec) in exact arithmetic,
// without the residual pass and the final addition (24 bytes per unknown and
// column) at the cost of reading ec in the first pre-smoothing pass (4).
template <typename T>
void Context::second_coarse_cycle(int l, const T* bc, T* ec, int nb, const int* act, bool top) {
  if (!top || top_cycles_ != 2 || l + 1 >= Ls_) return;
  if (!varcoef_ && !csr_) {
    vcycle<T>(l + 1, bc, ec, nb, act, nullptr, false, ec);
    return;
  }
  Work<T>& w = work<T>();
  T* r2 = w.vr2[l];
  T* e2 = w.ve2[l];
  op_residual<T, T, T>(l + 1, bc, ec, r2, nb, act, nullptr);
  vcycle<T>(l + 1, r2, e2, nb, act, nullptr);
  vec_add_to<T>(ec, e2, lv_[l].n, nb, act, s_);
}

// ---------------------------------------------------------------------------
// V-cycle of the 3D diffusion operator: in-place red-black sweeps (black first
// after the coarse correction, so the preconditioner is symmetric), fused
// residual + restriction, prolongation + omega-scaled correction.
// ---------------------------------------------------------------------------
template <typename T>
void Context::vcycle_vc(int l, const T* b, T* x, int nb, const int* act, c64* rz_partials,
                        bool top) {
  Work<T>& w = work<T>();
  if (l == 1) counters[2] += 1;
  const int64_t n = lv_[l - 1].n;
  const double en = (double)sizeof(T) * (double)n;
  if (l == Ls_) {
    dense_apply<T>(w.ainvT, b, x, (int)n, nb, act, s_, w.ld);
  } else if (lv_[l - 1].mcols > 0) {
    // fused out-of-place sweeps, ping-ponging between the level's scratch
    // buffer and x; the coarse correction is folded into the first post-sweep
    const Level& L = lv_[l - 1];
    const T* kf = vc_faces<T>(l);
    const T* dg = vc_diag<T>(l);
    const int pre = opt_.nu_pre, post = opt_.nu_post;
    T* tmp = w.vt[l - 1];
    const T* u = nullptr;  // current iterate (nullptr = 0)
    for (int i = 0; i < pre; ++i) {
      T* out = (i % 2 == 0) ? tmp : x;
      const T* in = u;
      timed<T>(l, kTimGs, en * ((in ? 3.0 : 2.0) + 4.0 / (double)nb), act, nb, [&] {
        varcoef_rbgs_march<T>(in, b, out, nullptr, 0.0, kf, dg, L.side, nb, L.mcols, act, false,
                              s_);
      });
      u = out;
    }
    T* bc = w.vb[l];
    T* ec = w.vx[l];
    if (u == nullptr)
      op_restrict<T>(l, b, bc, nb, act);
    else
      timed<T>(l, kTimResRestrict, en * (2.0 + 0.125 + 4.0 / (double)nb), act, nb,
               [&] { op_res_restrict<T>(l, b, u, bc, nb, act); });
    vcycle_vc<T>(l + 1, bc, ec, nb, act, nullptr);
    second_coarse_cycle<T>(l, bc, ec, nb, act, top);
    if (post == 0) {
      if (u != nullptr && u != x) vec_copy<T>(u, x, n, nb, act, s_);
      timed<T>(l, kTimProlong, en * (2.0 + 0.125), act, nb, [&] {
        varcoef_prolong<T>(ec, x, L.side, omega_, u == nullptr ? 0.0 : 1.0, nb, act, s_);
      });
    }
    for (int i = 0; i < post; ++i) {
      const int left = post - 1 - i;
      T* out = (left % 2 == 0) ? x : tmp;
      if (out == u) out = (out == x) ? tmp : x;  // never sweep in place
      const T* in = u;
      const T* corr = (i == 0) ? ec : nullptr;
      timed<T>(l, kTimGs,
               en * ((in ? 3.0 : 2.0) + (corr ? 0.125 : 0.0) + 4.0 / (double)nb), act, nb, [&] {
                 varcoef_rbgs_march<T>(in, b, out, corr, omega_, kf, dg, L.side, nb, L.mcols,
                                       act, true, s_);
               });
      u = out;
    }
    if (post > 0 && u != x) vec_copy<T>(u, x, n, nb, act, s_);
  } else {
    const Level& L = lv_[l - 1];
    const T* kf = vc_faces<T>(l);
    const T* dg = vc_diag<T>(l);
    const int pre = opt_.nu_pre, post = opt_.nu_post;
    for (int i = 0; i < pre; ++i)
      timed<T>(l, kTimGs, en * ((i == 0 ? 2.0 : 3.0) + 4.0 / (double)nb), act, nb, [&] {
        varcoef_rbgs<T>(b, x, kf, dg, L.side, nb, L.cols, act, i == 0, false, nullptr, 0.0, s_);
      });
    T* bc = w.vb[l];
    T* ec = w.vx[l];
    if (pre == 0)
      op_restrict<T>(l, b, bc, nb, act);
    else
      timed<T>(l, kTimResRestrict, en * (2.0 + 0.125 + 4.0 / (double)nb), act, nb,
               [&] { op_res_restrict<T>(l, b, x, bc, nb, act); });
    vcycle_vc<T>(l + 1, bc, ec, nb, act, nullptr);
    second_coarse_cycle<T>(l, bc, ec, nb, act, top);
    if (post == 0 || pre == 0) {
      timed<T>(l, kTimProlong, en * (2.0 + 0.125), act, nb, [&] {
        varcoef_prolong<T>(ec, x, L.side, omega_, pre == 0 ? 0.0 : 1.0, nb, act, s_);
      });
    }
    for (int i = 0; i < post; ++i) {
      // the first post-sweep reads the corrected iterate x + omega P ec on the fly
      const bool fold = (i == 0 && pre > 0);
      timed<T>(l, kTimGs, en * (3.0 + (fold ? 0.125 : 0.0) + 4.0 / (double)nb), act, nb, [&] {
        varcoef_rbgs<T>(b, x, kf, dg, L.side, nb, L.cols, act, false, true, fold ? ec : nullptr,
                        omega_, s_);
      });
    }
  }
  if (rz_partials) vec_dot_partials<T>(b, x, n, nb, act, rz_partials, s_);
}

// ---------------------------------------------------------------------------
// V-cycle on levels l..L_s: x = M b.  Pre-smoothing starts from zero; the
// coarse-grid correction (scaled by omega) is folded into the load of the first
// post-smoothing sweep.  Sweeps ping-pong between the level's scratch buffer
// and x.  rz_partials (top level of a Krylov solve only): per-block shares of
// conj(b)^T x, fused into the last sweep.
// ---------------------------------------------------------------------------
template <typename T>
void Context::vcycle(int l, const T* b, T* x, int nb, const int* act, c64* rz_partials,
                     bool top, const T* x0) {
  MLMC_REQUIRE(!x0 || (!varcoef_ && !csr_ && l < Ls_), MLMC_EINVAL,
               "a V-cycle from a given iterate is the 2D Poisson smoothed levels' only");
  if (varcoef_) {
    vcycle_vc<T>(l, b, x, nb, act, rz_partials, top);
    return;
  }
  if (csr_) {
    vcycle_csr<T>(l, b, x, nb, act, rz_partials, top);
    return;
  }
  Work<T>& w = work<T>();
  if (l == 1) counters[2] += 1;
  const int64_t n = lv_[l - 1].n;
  const double en = (double)sizeof(T) * (double)n;
  if (l == Ls_) {
    dense_apply<T>(w.ainvT, b, x, (int)n, nb, act, s_, w.ld);
    if (rz_partials) vec_dot_partials<T>(b, x, n, nb, act, rz_partials, s_);
    return;
  }
  const Level& L = lv_[l - 1];
  T* tmp = w.vt[l - 1];
  const int pre = opt_.nu_pre, post = opt_.nu_post;
  const int per = sweeps_per_pass(l);
  const int rows = gs_rows<T>(l);
  T* bc = w.vb[l];
  T* ec = w.vx[l];
  // pre-smoothing in passes of up to `per` sweeps: outputs alternate tmp, x, tmp,
  // ...; a last pass of two fused sweeps also writes the restricted residual
  const T* u = x0;  // current iterate (nullptr = 0); the first pass never writes it
  bool restricted = false;
  for (int i = 0, pass = 0; i < pre; ++pass) {
    // an odd remainder goes first, so the last pass is a full one
    const int sw = (pre - i) % per ? (pre - i) % per : per;
    T* out = (pass % 2 == 0) ? tmp : x;
    const T* in = u;
    if (sw == 2 && i + sw == pre) {
      timed<T>(l, kTimGs, en * (2.25 + (in ? 1.0 : 0.0)), act, nb, [&] {
        poisson_rbgs_restrict<T>(in, b, out, bc, L.side, L.d, L.c, nb, act, rows, s_);
      });
      restricted = true;
    } else {
      timed<T>(l, kTimGs, en * (2.0 + (in ? 1.0 : 0.0)), act, nb, [&] {
        poisson_rbgs_fused<T>(in, b, out, nullptr, 0.0, L.side, L.d, L.c, nb, act, false,
                              nullptr, rows, sw, s_);
      });
    }
    u = out;
    i += sw;
  }
  if (u == nullptr)
    op_restrict<T>(l, b, bc, nb, act);
  else if (!restricted)
    timed<T>(l, kTimResRestrict, 2.25 * en, act, nb,
             [&] { op_res_restrict<T>(l, b, u, bc, nb, act); });
  vcycle<T>(l + 1, bc, ec, nb, act, nullptr);
  second_coarse_cycle<T>(l, bc, ec, nb, act, top);
  if (post == 0) {
    if (u == nullptr) {
      agg2d_prolong<T>(ec, x, L.side, omega_, 0.0, nb, act, s_);
    } else {
      if (u != x) vec_copy<T>(u, x, n, nb, act, s_);
      agg2d_prolong<T>(ec, x, L.side, omega_, 1.0, nb, act, s_);
    }
    if (rz_partials) vec_dot_partials<T>(b, x, n, nb, act, rz_partials, s_);
    return;
  }
  // post-smoothing in passes of up to `per` sweeps; the last pass must land in x
  const int passes = (post + per - 1) / per;
  for (int i = 0, pass = 0; i < post; ++pass) {
    const int sw = std::min(per, post - i);
    const int left = passes - 1 - pass;
    T* out = (left % 2 == 0) ? x : tmp;
    if (out == u) out = (out == x) ? tmp : x;  // never sweep in place
    const T* in = u;
    const T* corr = (pass == 0) ? ec : nullptr;
    const bool last = (pass == passes - 1);
    timed<T>(l, kTimGs, en * (2.0 + (in ? 1.0 : 0.0) + (corr ? 0.25 : 0.0)), act, nb, [&] {
      poisson_rbgs_fused<T>(in, b, out, corr, omega_, L.side, L.d, L.c, nb, act, true,
                            last ? rz_partials : nullptr, rows, sw, s_);
    });
    u = out;
    i += sw;
  }
  if (u != x) {
    vec_copy<T>(u, x, n, nb, act, s_);
    if (rz_partials) vec_dot_partials<T>(b, x, n, nb, act, rz_partials, s_);
  }
}

// number of per-column partial sums that vcycle(l, ..., rz_partials) writes:
// the fused sweep's tile count when the last post-sweep lands in x, else the
// plain dot's block count (replays the buffer choice of vcycle symbolically)
template <typename T>
int Context::vcycle_partials(int l, bool* fused) const {
  const int64_t n = lv_[l - 1].n;
  *fused = false;
  if (varcoef_ || csr_ || l == Ls_ || opt_.nu_post == 0) return reduce_blocks(n);
  enum { kNull, kTmp, kX };
  const int per = sweeps_per_pass(l);
  int u = kNull;
  for (int pass = 0; pass < (opt_.nu_pre + per - 1) / per; ++pass) u = (pass % 2 == 0) ? kTmp : kX;
  const int passes = (opt_.nu_post + per - 1) / per;
  int last_sw = 1;
  for (int i = 0, pass = 0; i < opt_.nu_post; ++pass) {
    const int left = passes - 1 - pass;
    int out = (left % 2 == 0) ? kX : kTmp;
    if (out == u) out = (out == kX) ? kTmp : kX;
    u = out;
    last_sw = std::min(per, opt_.nu_post - i);
    i += last_sw;
  }
  if (u != kX) return reduce_blocks(n);
  *fused = true;
  const int tiles = poisson_gs_tiles<T>(lv_[l - 1].side, gs_rows<T>(l), last_sw);
  MLMC_REQUIRE((int64_t)tiles * nb_ <= partials_cap_, MLMC_EINVAL,
               "fused sweep partial sums exceed the partials buffer");
  return tiles;
}

// ---------------------------------------------------------------------------
// per-kernel timing with HIP events on the context stream (measurement mode):
// every launch of a timed kernel is bracketed by two events and preceded by a
// one-block count of its active columns, so the algorithmic bytes of the launch
// are known without a host synchronisation.
// ---------------------------------------------------------------------------

hipEvent_t Context::event() {
  if (!ev_pool_.empty()) {
    hipEvent_t e = ev_pool_.back();
    ev_pool_.pop_back();
    return e;
  }
  hipEvent_t e;
  MLMC_HIP(hipEventCreate(&e));
  return e;
}


void Context::set_timing(unsigned mask, int stride) {
  collect_timing();
  timing_ = mask != 0;
  timing_mask_ = mask;
  timing_stride_ = stride;
  for (int64_t& v : timing_seen_) v = 0;
  const bool on = timing_;
  if (on && !tlog_dev_) tlog_dev_ = dalloc_n<int>((int64_t)kTimingLog * nb_);
}

void Context::collect_timing() {
  if (pending_.empty()) return;
  MLMC_HIP(hipStreamSynchronize(s_));
  std::vector<int> flags((size_t)tlog_next_ * nb_);
  if (tlog_next_ > 0)
    MLMC_HIP(hipMemcpy(flags.data(), tlog_dev_, sizeof(int) * flags.size(),
                       hipMemcpyDeviceToHost));
  for (const Pending& p : pending_) {
    float ms = 0.f;
    MLMC_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    int count = 0;
    for (int k = 0; k < p.nb; ++k) count += flags[(size_t)p.idx * nb_ + k] ? 1 : 0;
    for (TimerStat* t : {&tstat_[p.slot], &tstat_lv_[p.slot][std::min(std::max(p.level, 1),
                                                                      MLMC_MAX_LEVELS) - 1]}) {
      t->launches += 1;
      t->ms += ms;
      t->bytes += p.bytes_per_col * count;
    }
    ev_pool_.push_back(p.a);
    ev_pool_.push_back(p.b);
  }
  pending_.clear();
  tlog_next_ = 0;
}

void Context::kernel_stats(int id, int fp64, double* out, int level) {
  collect_timing();
  MLMC_REQUIRE(id >= 0 && id < kNumTimers, MLMC_EINVAL, "unknown kernel id");
  MLMC_REQUIRE(level >= 0 && level <= Ls_, MLMC_EINVAL, "level out of range");
  const int slot = 2 * id + (fp64 ? 1 : 0);
  const TimerStat& t = level == 0 ? tstat_[slot] : tstat_lv_[slot][level - 1];
  out[0] = (double)t.launches;
  out[1] = t.ms;
  out[2] = t.bytes;
}

void Context::reset_kernel_stats() {
  collect_timing();
  for (TimerStat& t : tstat_) t = TimerStat();
  for (auto& row : tstat_lv_)
    for (TimerStat& t : row) t = TimerStat();
}

// the count of active columns, stored in count_map_[0] by the last
// convergence test on the stream
int Context::read_count() {
  MLMC_HIP(hipStreamSynchronize(s_));
  return count_host_[0];
}

// ---------------------------------------------------------------------------
// Preconditioned CG (A Hermitian positive definite), columns in lockstep with
// per-column scalars on the device.  Convergence: |r| <= tol |b| per column.
// Per iteration: [p_new = z + beta p_old ; q = A p_new ; p^T q] fused,
// [x += alpha p ; r -= alpha q ; |r|^2] fused, [z = M r ; r^T z] fused.
// lastcorr (nullable): per column alpha*rz of the last step, which equals
// b^H (alpha p) when x starts at 0 -- the last step's contribution to b^H x.
// Returns the iteration count.
// ---------------------------------------------------------------------------
template <typename T>
int Context::pcg(int l, const T* b, T* x, int nb, int* act, double tol, c64* lastcorr) {
  Work<T>& w = work<T>();
  const Level& L = lv_[l - 1];
  const int64_t n = L.n;
  const int nblk = reduce_blocks(n);
  const int ntiles = op_tiles(l);
  c64 *rr0 = scal_[kRr0], *rz = scal_[kRz], *tmp = scal_[kTmp], *alpha = scal_[kAlpha],
      *beta = scal_[kBeta];
  vec_zero<T>(x, n, nb, act, s_);
  if (l == Ls_) {  // direct solve on the coarsest level
    dense_apply<T>(w.ainvT, b, x, (int)n, nb, act, s_, w.ld);
    if (lastcorr) vec_zero<c64>(lastcorr, 1, nb, nullptr, s_);
    return 0;
  }
  const double en = (double)sizeof(T) * (double)n;
  vec_copy<T>(b, w.r, n, nb, act, s_);
  vec_dot_partials<T>(b, b, n, nb, act, partials_, s_);
  finish_sums(partials_, nblk, nb, rr0, s_);
  bool fused = false;
  const int nvp = vcycle_partials<T>(l, &fused);
  vcycle<T>(l, w.r, w.z, nb, act, partials_, true);
  finish_sums(partials_, nvp, nb, rz, s_);
  vec_zero<c64>(beta, 1, nb, nullptr, s_);
  T* p_old = w.z;  // first direction: p = z + 0 * z
  T* p_new = w.p;
  const int check = 2;
  int it = 0;
  for (it = 1; it <= opt_.max_iter; ++it) {
    timed<T>(l, kTimApply, 4.0 * en, act, nb,
             [&] { op_update_apply<T>(l, p_old, w.z, beta, p_new, w.q, nb, act); });
    finish_alpha(partials_, ntiles, nb, tmp, rz, act, alpha, s_);
    if (lastcorr) cg_lastcorr(alpha, rz, act, lastcorr, nb, s_);
    timed<T>(l, kTimCgXr, 6.0 * en, act, nb,
             [&] { cg_update_xr<T>(x, w.r, p_new, w.q, alpha, n, nb, act, partials_, s_); });
    finish_sums(partials_, nblk, nb, tmp, s_);
    mark_converged(tmp, rr0, tol * tol, act, nb, count_map_, s_);
    counters[0] += 1;
    if (it % check == 0 || it == opt_.max_iter) {
      if (read_count() == 0) break;
    }
    vcycle<T>(l, w.r, w.z, nb, act, partials_, true);
    finish_beta(partials_, nvp, nb, tmp, rz, act, beta, s_);
    // the new direction of this iteration is the old one of the next
    p_old = p_new;
    p_new = (p_new == w.p) ? w.p2 : w.p;
  }
  return it;
}

// ---------------------------------------------------------------------------
// FP32 preconditioned CG with FP64 iterative refinement by reliable updates:
// the CG recursion (x32, r32, p, q, z) runs in FP32; whenever a column's
// recursive residual has dropped by the factor inner_tol since the last
// refinement (or reaches solve_tol), every active column is refined in FP64:
// y64 += x32, x32 = 0, r = b - A y64 recomputed in FP64 (and rounded to FP32).
// The search direction is kept, so the Krylov space is not discarded as in a
// restarted refinement, unless the new FP64 residual exceeds the recursion's
// own by more than 100x in squared norm (the recursion ran below FP32
// accuracy); then the next direction restarts from z.  Only the FP64 residual
// marks a column converged.
// Stated error of a column (err): the last correction's share |b^H x32| of
// b^H y scaled by the residual reduction it achieved -- the linear-convergence
// estimate of what a further correction would add.  On return scal_[kRres]
// holds the final |b - A y|^2 per column.
// ---------------------------------------------------------------------------
void Context::pcg_refined(int l, const double* b, double* y, int nb, double tol, c64* err) {
  Work<float>& w = w32_;
  const Level& L = lv_[l - 1];
  const int64_t n = L.n;
  const int nblk = reduce_blocks(n);
  const int ntiles = op_tiles(l);
  int* act = act_outer_;
  c64 *bb = scal_[kBb], *bd = scal_[kBd], *rr_upd = scal_[kRres], *rr_new = scal_[kRres2];
  c64 *rz = scal_[kRz], *tmp = scal_[kTmp], *alpha = scal_[kAlpha], *beta = scal_[kBeta];
  float* x32 = d32_;
  float* r = w.r;
  const double en = 4.0 * (double)n;
  // y and x32 start at zero without a clearing pass: the first x/r update
  // writes x32 = 0 + alpha p without reading it, and the first fold writes
  // y = 0 + x32 without reading y (every column is active until then)
  bool y_written = false;
  // The refinements read b from an FP32 copy when every entry of b is an FP32
  // number (the 2D Poisson probes and their 2x2 restrictions, multiples of 1/2
  // of small integers): the same values for 4 instead of 8 bytes per unknown
  // in the fold and the residual.  Any other b keeps the FP64 reads (the check
  // runs on the device; its flag is read at the first refinement check).
  // With the FP32 copy, |b|^2 comes from the same pass (solve() leaves it to
  // this function then).
  const bool try32 = b32_ != nullptr;
  if (try32) {
    rhs_fp32(b, r, b32_, n, nb, count_dev_ + 4, partials_, s_);
    finish_sums(partials_, nblk, nb, bb, s_);
    MLMC_HIP(hipMemcpyAsync(count_host_ + 4, count_dev_ + 4, sizeof(int), hipMemcpyDeviceToHost,
                            s_));
  } else {
    vec_convert<float, double>(b, r, n, nb, nullptr, s_);
  }
  vec_copy<c64>(bb, rr_upd, 1, nb, nullptr, s_);
  bool fused = false;
  const int nvp = vcycle_partials<float>(l, &fused);
  vcycle<float>(l, r, w.z, nb, act, partials_, true);
  finish_sums(partials_, nvp, nb, rz, s_);
  vec_zero<c64>(beta, 1, nb, nullptr, s_);
  const double delta2 = opt_.inner_tol * opt_.inner_tol;
  const int max_it = opt_.max_iter * opt_.max_refine;
  float* P1 = w.p;
  float* P2 = w.p2;
  // one CG iteration: p_new = z + beta p_old, q = A p_new, alpha, x/r update
  // (|r|^2 lands in tmp only when a refinement check follows: otherwise the
  // next tail overwrites tmp unread)
  auto core = [&](float* p_old, float* p_new, bool checked, bool x_zero = false) {
    timed<float>(l, kTimApply, 4.0 * en, act, nb,
                 [&] { op_update_apply<float>(l, p_old, w.z, beta, p_new, w.q, nb, act); });
    finish_alpha(partials_, ntiles, nb, tmp, rz, act, alpha, s_);
    timed<float>(l, kTimCgXr, (x_zero ? 5.0 : 6.0) * en, act, nb, [&] {
      cg_update_xr<float>(x32, r, p_new, w.q, alpha, n, nb, act, partials_, s_, x_zero);
    });
    if (checked) finish_sums(partials_, nblk, nb, tmp, s_);
  };
  // preconditioner and the next direction's beta
  auto tail = [&] {
    vcycle<float>(l, r, w.z, nb, act, partials_, true);
    finish_beta(partials_, nvp, nb, tmp, rz, act, beta, s_);
  };
  // a refinement is due when some column's recursive residual has dropped by
  // inner_tol since its last refinement, or reached the tolerance
  auto due = [&] {
    refine_due(tmp, rr_upd, bb, delta2, tol * tol, act, nb, count_map_ + 1, s_);
  };
  // after due(): refine in FP64 if needed; true when every column converged
  auto refine = [&](bool force) {
    MLMC_HIP(hipStreamSynchronize(s_));
    if (count_host_[1] == 0 && !force) return false;
    const bool b_fp32 = try32 && count_host_[4] == 0;
    const double bbytes = b_fp32 ? 4.0 : 8.0;
    // y += x32, bd = b^T x32, x32 = 0 in one pass (FP64 y, b and FP32 x32 in;
    // y, x32 out: 32 bytes per unknown, 28 with b in FP32; 8 fewer on the
    // first fold, which does not read y)
    const bool y_zero = !y_written;
    timed<double>(l, kTimIrFold, ((y_zero ? 16.0 : 24.0) + bbytes) * (double)n, act, nb, [&] {
      if (b_fp32)
        ir_fold(y, x32, b32_, n, nb, act, partials_, s_, y_zero);
      else
        ir_fold(y, x32, b, n, nb, act, partials_, s_, y_zero);
    });
    y_written = true;
    finish_sums(partials_, nblk, nb, bd, s_);
    timed<double>(l, kTimIrResidual, (12.0 + bbytes) * (double)n, act, nb, [&] {
      if (b_fp32)
        poisson_residual<float, double, float>(b32_, y, r, L.side, L.d, L.c, nb, act, partials_,
                                               s_);
      else
        op_residual<double, double, float>(l, b, y, r, nb, act, partials_);
    });
    finish_sums(partials_, ntiles, nb, rr_new, s_);
    ir_stated_error(bd, rr_upd, rr_new, act, err, nb, s_);
    // the kept direction stays only while the recursion's residual (tmp, from
    // the last x/r update) still describes the true one; when the recursion has
    // run far below FP32 accuracy (a nearly exact preconditioner) restart it
    cg_restart_on_drift(rr_new, tmp, rz, act, 100.0, nb, s_);
    select_active(rr_upd, rr_new, act, nb, s_);
    mark_converged(rr_new, bb, tol * tol, act, nb, count_map_, s_);
    counters[1] += 1;
    return read_count() == 0;
  };
  // iterations 1 and 2 directly (the first direction is z itself), then pairs of
  // iterations between refinement checks: (p2 -> p), (p -> p2), which repeat
  // with fixed pointers and can be replayed from a graph
  int it = 1;
  core(w.z, P1, it == max_it, true);
  counters[0] += 1;
  if (it == max_it) {
    due();
    refine(true);
    return;
  }
  tail();
  core(P1, P2, true);
  counters[0] += 1;
  it = 2;
  due();
  if (refine(it == max_it)) return;
  const bool use_graph = opt_.graphs && !timing_;
  while (it < max_it) {
    if (it + 2 <= max_it) {
      auto pair = [&] {
        tail();
        core(P2, P1, false);
        tail();
        core(P1, P2, true);
        due();
      };
      if (use_graph)
        replay({0, l, nb, 0}, pair);
      else
        pair();
      counters[0] += 2;
      it += 2;
      if (refine(it == max_it)) return;
    } else {
      tail();
      core(P2, P1, true);
      counters[0] += 1;
      it += 1;
      due();
      refine(true);
      return;
    }
  }
}

void Context::replay(const std::array<int, 4>& key, const std::function<void()>& body) {
  auto found = graphs_.find(key);
  if (found == graphs_.end()) {
    // capture on a stream of our own (the caller's stream may be the legacy
    // default stream, which cannot be captured): the launches of `body` go to
    // s_, so s_ points at the capture stream while recording
    if (!cap_s_) MLMC_HIP(hipStreamCreateWithFlags(&cap_s_, hipStreamNonBlocking));
    int64_t c0[4], n0[2];
    std::memcpy(c0, counters, sizeof(c0));
    std::memcpy(n0, nn_stats, sizeof(n0));
    auto restore = [&] {  // capture only recorded the launches
      std::memcpy(counters, c0, sizeof(c0));
      std::memcpy(nn_stats, n0, sizeof(n0));
    };
    hipGraph_t g = nullptr;
    hipStream_t caller = s_;
    MLMC_HIP(hipStreamBeginCapture(cap_s_, hipStreamCaptureModeThreadLocal));
    s_ = cap_s_;
    try {
      body();
    } catch (...) {
      s_ = caller;
      (void)hipStreamEndCapture(cap_s_, &g);
      if (g) (void)hipGraphDestroy(g);
      restore();
      throw;
    }
    s_ = caller;
    MLMC_HIP(hipStreamEndCapture(cap_s_, &g));
    Graph gr;
    for (int i = 0; i < 4; ++i) gr.counters[i] = counters[i] - c0[i];
    for (int i = 0; i < 2; ++i) gr.nn_stats[i] = nn_stats[i] - n0[i];
    restore();
    const hipError_t e = hipGraphInstantiate(&gr.ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    MLMC_HIP(e);
    found = graphs_.emplace(key, gr).first;
  }
  const Graph& gr = found->second;
  MLMC_HIP(hipGraphLaunch(gr.ex, s_));
  for (int i = 0; i < 4; ++i) counters[i] += gr.counters[i];
  for (int i = 0; i < 2; ++i) nn_stats[i] += gr.nn_stats[i];
}

// ---------------------------------------------------------------------------
// FP64 solve of A_l y = b for nb columns.  err (device, nb): stated error
// contribution b^H d of the last correction d.  relres_host: final FP64
// relative residuals (nullable).  converged: all columns met solve_tol.
// ---------------------------------------------------------------------------
void Context::solve(int l, const double* b, double* y, int nb, c64* err, double* relres_host,
                    bool* converged) {
  const int64_t n = lv_[l - 1].n;
  const int nblk_pts = complex_ ? 0 : op_tiles(l);
  const int nblk = reduce_blocks(n);
  c64* bb = scal_[kBb];
  c64* bd = scal_[kBd];
  c64* rres = scal_[kRres];  // also the refinement loop's residual norms
  if (complex_) {
    solve_complex(l, reinterpret_cast<const c64*>(b), reinterpret_cast<c64*>(y), nb, err);
    // final FP64 relative residuals
    cop_residual<c64, c64, c64>(l, reinterpret_cast<const c64*>(b),
                                reinterpret_cast<const c64*>(y), reinterpret_cast<c64*>(r64_),
                                nb, nullptr, partials_);
    finish_sums(partials_, lv_[l - 1].wilson ? wilson_residual_blocks(lv_[l - 1].side)
                                             : bsr_residual_blocks(lv_[l - 1].side),
                nb, rres, s_);
    vec_dot_partials<c64>(reinterpret_cast<const c64*>(b), reinterpret_cast<const c64*>(b), n,
                          nb, nullptr, partials_, s_);
    finish_sums(partials_, nblk, nb, bb, s_);
  } else {
  const bool refined = l != Ls_ && opt_.precision != MLMC_FP64 && !fp64_batch(nb);
  if (!(refined && b32_)) {  // else pcg_refined forms |b|^2 with the FP32 copy of b
    vec_dot_partials<double>(b, b, n, nb, nullptr, partials_, s_);
    finish_sums(partials_, nblk, nb, bb, s_);
  }
  set_all_active(act_outer_, nb, s_);
  vec_zero<c64>(err, 1, nb, nullptr, s_);
  const double tol = opt_.solve_tol;
  if (l == Ls_) {
    dense_apply<double>(w64_.ainvT, b, y, (int)n, nb, nullptr, s_, w64_.ld);
  } else if (opt_.precision == MLMC_FP64 || fp64_batch(nb)) {
    MLMC_HIP(hipMemcpyAsync(act_inner_, act_outer_, sizeof(int) * nb,
                            hipMemcpyDeviceToDevice, s_));
    pcg<double>(l, b, y, nb, act_inner_, tol, err);
    counters[1] += 1;
  } else {
    pcg_refined(l, b, y, nb, tol, err);
  }
  // final FP64 relative residuals (the refined solver ends on a true FP64
  // residual already, kept in rres)
  if (l == Ls_ || opt_.precision == MLMC_FP64 || fp64_batch(nb)) {
    op_residual<double, double, double>(l, b, y, r64_, nb, nullptr, partials_);
    finish_sums(partials_, nblk_pts, nb, rres, s_);
  }
  }
  const double tol = opt_.solve_tol;
  MLMC_HIP(hipMemcpyAsync(host_c64_, rres, sizeof(c64) * nb, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipMemcpyAsync(host_c64_ + nb, bb, sizeof(c64) * nb, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  bool ok = true;
  col_ok_.assign((size_t)nb, 1);
  for (int k = 0; k < nb; ++k) {
    const double bn = host_c64_[nb + k].re;
    const double rel = bn > 0 ? std::sqrt(host_c64_[k].re / bn) : std::sqrt(host_c64_[k].re);
    if (relres_host) relres_host[k] = rel;
    if (!(rel <= tol)) {
      ok = false;
      col_ok_[(size_t)k] = 0;
    }
  }
  if (converged) *converged = ok;
}

// ---------------------------------------------------------------------------
// probes (Rademacher for real, Z4 for complex operators), their restriction
// and quadratic forms, on FP64 buffers (complex: interleaved)
// ---------------------------------------------------------------------------
void Context::write_probes(int level, uint64_t seed, uint64_t stream, uint64_t first, int nb,
                           double* out) {
  const int64_t n = lv_[level - 1].n;
  if (complex_)
    probes_write<c64>(reinterpret_cast<c64*>(out), n, nb, seed, 0, first, (uint64_t)level,
                      stream, s_);
  else
    probes_write<double>(out, n, nb, seed, 0, first, (uint64_t)level, stream, s_);
}

void Context::restrict64(int level, const double* x, double* xc, int nb) {
  if (complex_)
    cop_restrict<c64>(level, reinterpret_cast<const c64*>(x), reinterpret_cast<c64*>(xc), nb,
                      nullptr);
  else
    op_restrict<double>(level, x, xc, nb, nullptr);
}

void Context::probe_quad(int level, uint64_t seed, uint64_t stream, uint64_t first, int nb,
                         const double* y, c64* out) {
  const int64_t n = lv_[level - 1].n;
  const int64_t chunk = complex_ ? (int64_t)kThreads * 128 : (int64_t)kThreads * 256;
  const int nblk = (int)((n + chunk - 1) / chunk);
  if (complex_)
    probe_dot_partials<c64>(reinterpret_cast<const c64*>(y), n, nb, seed, 0, first,
                            (uint64_t)level, stream, partials_, s_);
  else
    probe_dot_partials<double>(y, n, nb, seed, 0, first, (uint64_t)level, stream, partials_, s_);
  finish_sums(partials_, nblk, nb, out, s_);
}

// ---------------------------------------------------------------------------
// level-difference samples: s = x^H A_l^-1 x - (R x)^H A_{l+1}^-1 (R x)
// ---------------------------------------------------------------------------
void Context::samples_batch(int level, uint64_t seed, uint64_t first, int nbatch, c64* out,
                            double* err_out) {
  MLMC_REQUIRE(level >= 1 && level < L_, MLMC_EINVAL, "sample level must be in [1, L-1]");
  MLMC_REQUIRE(nbatch >= 1 && nbatch <= nb_, MLMC_EINVAL, "batch size out of range");
  if (general_) {
    samples_batch_general(level, seed, first, nbatch, out, err_out);
    return;
  }
  const int64_t n1 = lv_[level - 1].n, n2 = lv_[level].n;
  write_probes(level, seed, kStreamProbe, first, nbatch, b1_);
  bool ok1 = true, ok2 = true;
  c64 *e1 = scal_[kErr1], *e2 = scal_[kErr2], *qa = scal_[kQa], *qb = scal_[kQb];
  solve(level, b1_, y1_, nbatch, e1, nullptr, &ok1);
  const std::vector<char> okc1 = col_ok_;
  restrict64(level, b1_, b2_, nbatch);
  solve(level + 1, b2_, y2_, nbatch, e2, nullptr, &ok2);
  const std::vector<char> okc2 = col_ok_;
  // x^H y with x regenerated, and (Rx)^H z
  probe_quad(level, seed, kStreamProbe, first, nbatch, y1_, qa);
  if (complex_) {
    vec_dot_partials<c64>(reinterpret_cast<const c64*>(b2_), reinterpret_cast<const c64*>(y2_),
                          n2, nbatch, nullptr, partials_, s_);
  } else {
    vec_dot_partials<double>(b2_, y2_, n2, nbatch, nullptr, partials_, s_);
  }
  finish_sums(partials_, reduce_blocks(n2), nbatch, qb, s_);
  finish_samples(level, nbatch, okc1.data(), okc2.data(), first, out, err_out);
}

// copy the batch's scalars (stated errors e1, e2 and quadratic forms qa, qb,
// consecutive blocks of nb_ entries) to the host, form s = qa - qb and the
// relative stated errors; throw if a solve missed solve_tol
void Context::finish_samples(int level, int nbatch, const char* ok1, const char* ok2,
                             uint64_t first, c64* out, double* err_out) {
  MLMC_HIP(hipMemcpyAsync(host_c64_, scal_[kErr1], sizeof(c64) * 4 * nb_,
                          hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
  const c64 *he1 = host_c64_, *he2 = host_c64_ + nb_, *ha = host_c64_ + 2 * nb_,
            *hb = host_c64_ + 3 * nb_;
  int failed = 0, first_bad = -1, bad_level = 0;
  for (int k = 0; k < nbatch; ++k) {
    const c64 a = ha[k], b = hb[k];
    const bool ok = ok1[k] && (!ok2 || ok2[k]);
    out[k] = ok ? c64{a.re - b.re, a.im - b.im} : c64{NAN, NAN};
    if (err_out) {
      const double den = std::hypot(a.re, a.im) + std::hypot(b.re, b.im);
      const double num = std::hypot(he1[k].re, he1[k].im) + std::hypot(he2[k].re, he2[k].im);
      err_out[k] = ok ? (den > 0 ? num / den : num) : NAN;
    }
    if (!ok) {
      if (failed++ == 0) {
        first_bad = k;
        bad_level = ok1[k] ? level + 1 : level;
      }
    }
  }
  counters[3] += 1;
  if (failed > 0)
    throw Error(MLMC_ENOCONV,
                "level " + std::to_string(level) + " samples: the solve on level " +
                    std::to_string(bad_level) + " missed solve_tol for sample " +
                    std::to_string(first + (uint64_t)first_bad) + " (column " +
                    std::to_string(first_bad) + " of a batch of " + std::to_string(nbatch) +
                    "; " + std::to_string(failed) + " of the batch failed, their samples NaN)");
}

void Context::hutch_batch(uint64_t seed, uint64_t stream, uint64_t first, int nbatch,
                          c64* out) {
  write_probes(1, seed, stream, first, nbatch, b1_);
  bool ok = true;
  solve(1, b1_, y1_, nbatch, scal_[kErr1], nullptr, &ok);
  probe_quad(1, seed, stream, first, nbatch, y1_, scal_[kQa]);
  MLMC_HIP(hipMemcpyAsync(host_c64_, scal_[kQa], sizeof(c64) * nbatch, hipMemcpyDeviceToHost,
                          s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  for (int k = 0; k < nbatch; ++k) out[k] = host_c64_[k];
  counters[3] += 1;
  if (!ok) throw Error(MLMC_ENOCONV, "solve on level 1 missed solve_tol");
}

void Context::sample_level(int level, uint64_t seed, int64_t first, int64_t count, double* out,
                           double* out_err) {
  MLMC_REQUIRE(level >= 1 && level < L_, MLMC_EINVAL, "sample level must be in [1, L-1]");
  MLMC_REQUIRE(first >= 0 && count >= 1, MLMC_EINVAL, "bad sample range");
  std::memset(counters, 0, sizeof(counters));
  std::vector<c64> buf(nb_);
  std::vector<double> eb(nb_);
  for (int64_t j = 0; j < count; j += nb_) {
    const int nbt = (int)std::min<int64_t>(nb_, count - j);
    auto copy_out = [&] {
      for (int k = 0; k < nbt; ++k) {
        out[2 * (j + k)] = buf[k].re;
        out[2 * (j + k) + 1] = buf[k].im;
        if (out_err) out_err[j + k] = eb[k];
      }
    };
    try {
      samples_batch(level, seed, (uint64_t)(first + j), nbt, buf.data(), eb.data());
    } catch (const Error& e) {
      // partial results: the batches before, and this batch's converged samples
      if (e.code == MLMC_ENOCONV) copy_out();
      throw;
    }
    copy_out();
  }
}

void Context::trace(double tol, uint64_t seed, mlmc_result* out) {
  std::memset(counters, 0, sizeof(counters));
  double level_s[MLMC_MAX_LEVELS] = {0};
  auto now = [] {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
  };
  SamplerIface smp;
  smp.sample = [&](int level, int64_t first, int64_t count, c64* o) {
    const double t0 = now();
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      samples_batch(level, seed, (uint64_t)(first + j), nbt, o + j, nullptr);
    }
    level_s[level - 1] += now() - t0;
  };
  smp.pilot = [&](int64_t count, c64* o) {
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      hutch_batch(seed, kStreamPilot, (uint64_t)j, nbt, o + j);
    }
  };
  std::vector<double> cost(L_ - 1);
  for (int l = 0; l < L_ - 1; ++l) cost[l] = (double)(lv_[l].n + lv_[l + 1].n);
  run_estimator(L_, smp, coarse_trace_, cost, opt_, tol, out);
  int64_t solves = 0;
  for (int l = 0; l < L_ - 1; ++l) {
    solves += 2 * out->n_samples[l];
    out->level_seconds[l] = level_s[l];
  }
  out->solves = solves + (opt_.tau > 0 ? 0 : 5);
  out->iterations = counters[0];
}

void Context::hutchinson(double tol, uint64_t seed, mlmc_result* out) {
  std::memset(counters, 0, sizeof(counters));
  auto sample = [&](int64_t first, int64_t count, c64* o) {
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      hutch_batch(seed, kStreamHutch, (uint64_t)(first + j), nbt, o + j);
    }
  };
  auto pilot = [&](int64_t count, c64* o) {
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      hutch_batch(seed, kStreamPilot, (uint64_t)j, nbt, o + j);
    }
  };
  run_hutchinson(sample, pilot, opt_, tol, out);
  out->solves = out->n_samples[0] + (opt_.tau > 0 ? 0 : 5);
  out->iterations = counters[0];
  out->coarse_trace[0] = coarse_trace_.re;
  out->coarse_trace[1] = coarse_trace_.im;
}

// ---------------------------------------------------------------------------
// FP64 building blocks exposed for tests
// ---------------------------------------------------------------------------
void Context::solve_fp64(int level, int nrhs, const double* b, double* y, double* relres,
                         bool throw_on_noconv) {
  MLMC_REQUIRE(level >= 1 && level <= Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nrhs >= 1 && nrhs <= nb_, MLMC_EINVAL, "nrhs must be in [1, nb]");
  std::memset(counters, 0, sizeof(counters));
  bool ok = true;
  solve(level, b, y, nrhs, scal_[kErr1], relres, &ok);
  if (!ok && throw_on_noconv) throw Error(MLMC_ENOCONV, "solve missed solve_tol");
}

void Context::apply_fp64(int level, int nrhs, const double* x, double* y) {
  MLMC_REQUIRE(level >= 1 && level <= Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nrhs >= 1, MLMC_EINVAL, "nrhs must be >= 1");
  if (complex_)
    cop_residual<c64, c64, c64>(level, nullptr, reinterpret_cast<const c64*>(x),
                                reinterpret_cast<c64*>(y), nrhs, nullptr, nullptr);
  else
    op_apply<double>(level, x, y, nrhs, nullptr, nullptr);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

// x <- `sweeps` red-black Gauss-Seidel sweeps of A_level x = b in the working
// precision, with the V-cycle's own kernels (passes of fused sweeps on the 2D
// Poisson levels); reverse: second colour first, as in post-smoothing.  rc
// (nullable): R (b - A x) of the final x, as the V-cycle's last pre-pass forms it
void Context::smooth_fp64(int level, int nrhs, int sweeps, bool reverse, bool zero_start,
                          const double* b, double* x, double* rc, void* ws, size_t ws_bytes,
                          int csr_tail) {
  MLMC_REQUIRE(level >= 1 && level < Ls_, MLMC_EINVAL, "level out of range (no smoother on L_s)");
  MLMC_REQUIRE(nrhs >= 1 && nrhs <= nb_, MLMC_EINVAL, "nrhs must be in [1, nb]");
  MLMC_REQUIRE(sweeps >= 0, MLMC_EINVAL, "sweeps must be >= 0");
  MLMC_REQUIRE(!(rc && reverse), MLMC_EINVAL, "the restricted residual follows a forward pass");
  MLMC_REQUIRE(!(zero_start && reverse), MLMC_EINVAL,
               "a zero start is the forward pre-smoothing's (no reverse sweeps from zero)");
  const int64_t n = lv_[level - 1].n;
  const int64_t elem = complex_ ? 2 : 1;
  const int64_t m = n * nrhs * elem, mc = lv_[level].n * nrhs * elem;
  auto to_t = [&](auto* dst, const double* src, int64_t cnt) {
    using T = typename std::remove_pointer<decltype(dst)>::type;
    if constexpr (std::is_same<T, double>::value)
      vec_copy<double>(src, dst, cnt, 1, nullptr, s_);
    else
      vec_convert<T, double>(src, dst, cnt, 1, nullptr, s_);
  };
  auto from_t = [&](const auto* src, double* dst, int64_t cnt) {
    using T = typename std::remove_const<typename std::remove_pointer<decltype(src)>::type>::type;
    if constexpr (std::is_same<T, double>::value)
      vec_copy<double>(src, dst, cnt, 1, nullptr, s_);
    else
      vec_convert<double, T>(src, dst, cnt, 1, nullptr, s_);
  };
  auto run = [&](auto tag) {
    using T = decltype(tag);
    // working-precision copies: allocated here, or carved from the caller's
    // workspace (256-byte aligned pieces)
    T *bt, *xa, *xb, *rct = nullptr;
    if (ws) {
      auto piece = [](int64_t cnt) { return (((size_t)cnt * sizeof(T)) + 255) & ~(size_t)255; };
      const size_t need = 3 * piece(m) + (rc ? piece(mc) : 0);
      MLMC_REQUIRE(need <= ws_bytes, MLMC_EINVAL,
                   "the smoother's working copies need " + std::to_string(need) +
                       " bytes of workspace, more than the " + std::to_string(ws_bytes) +
                       " available (fewer right-hand sides or a coarser level fit)");
      char* p = static_cast<char*>(ws);
      bt = reinterpret_cast<T*>(p);
      xa = reinterpret_cast<T*>(p + piece(m));
      xb = reinterpret_cast<T*>(p + 2 * piece(m));
      if (rc) rct = reinterpret_cast<T*>(p + 3 * piece(m));
    } else {
      bt = dalloc_n<T>(m);
      xa = dalloc_n<T>(m);
      xb = dalloc_n<T>(m);
      if (rc) rct = dalloc_n<T>(mc);
    }
    to_t(bt, b, m);
    if (!zero_start) to_t(xa, x, m);
    else if (sweeps == 0) vec_zero<T>(xa, m, 1, nullptr, s_);
    const Level& L = lv_[level - 1];
    bool restricted = false;
    if (complex_) {
      using C = typename std::conditional<sizeof(T) == 4, c32, c64>::type;
      // the V-cycle's sweep sequence (fused two-colour passes on the Wilson level;
      // from zero: the zero-start form of the first pass)
      cop_smooth_n<C>(level, reinterpret_cast<const C*>(bt), reinterpret_cast<C*>(xa), nrhs,
                      nullptr, sweeps, zero_start, reverse);
    } else if (csr_) {
      if (zero_start) vec_zero<T>(xa, n, nrhs, nullptr, s_);  // as the V-cycle starts
      for (int i = 0; i < sweeps; ++i)
        csr_gs_sweep<T>(bt, xa, csr_sweep<T>(level), (int)n, nrhs, csr_cols(L, nrhs),
                        csr_tail >= 0 ? csr_tail : this->csr_tail(L, nrhs), nullptr, reverse,
                        s_);
    } else if (varcoef_) {
      for (int i = 0; i < sweeps; ++i) {
        const bool z = zero_start && i == 0;
        if (L.mcols > 0) {
          varcoef_rbgs_march<T>(z ? nullptr : xa, bt, xb, nullptr, 0.0, vc_faces<T>(level),
                                vc_diag<T>(level), L.side, nrhs, L.mcols, nullptr, reverse, s_);
          std::swap(xa, xb);
        } else {
          varcoef_rbgs<T>(bt, xa, vc_faces<T>(level), vc_diag<T>(level), L.side, nrhs, L.cols,
                          nullptr, z, reverse, nullptr, 0.0, s_);
        }
      }
    } else {
      // passes of up to `per` fused sweeps in the V-cycle's grouping: forward
      // (pre-smoothing) takes an odd remainder first so that the last pass is a
      // full one that can write the restricted residual; reverse (post-smoothing)
      // takes full passes first
      const int per = sweeps_per_pass(level);
      for (int i = 0; i < sweeps;) {
        const int sw = reverse ? std::min(per, sweeps - i)
                               : ((sweeps - i) % per ? (sweeps - i) % per : per);
        const T* in = (zero_start && i == 0) ? nullptr : xa;
        if (rct && sw == 2 && i + sw == sweeps) {
          poisson_rbgs_restrict<T>(in, bt, xb, rct, L.side, L.d, L.c, nrhs, nullptr,
                                   gs_rows<T>(level), s_);
          restricted = true;
        } else {
          poisson_rbgs_fused<T>(in, bt, xb, nullptr, 0.0, L.side, L.d, L.c, nrhs, nullptr,
                                reverse, nullptr, gs_rows<T>(level), sw, s_);
        }
        std::swap(xa, xb);
        i += sw;
      }
    }
    if (rct && !restricted) {
      if (complex_) {
        using C = typename std::conditional<sizeof(T) == 4, c32, c64>::type;
        cop_residual<C, C, C>(level, reinterpret_cast<const C*>(bt),
                              reinterpret_cast<const C*>(xa), reinterpret_cast<C*>(xb), nrhs,
                              nullptr, nullptr);
        cop_restrict<C>(level, reinterpret_cast<const C*>(xb), reinterpret_cast<C*>(rct), nrhs,
                        nullptr);
      } else {
        op_res_restrict<T>(level, bt, xa, rct, nrhs, nullptr);
      }
    }
    from_t(xa, x, m);
    if (rct) from_t(rct, rc, mc);
    MLMC_HIP(hipGetLastError());
    if (ws) return;  // the caller's workspace: no stream synchronisation needed
    MLMC_HIP(hipStreamSynchronize(s_));
    dfree(bt);
    dfree(xa);
    dfree(xb);
    if (rct) dfree(rct);
  };
  if (opt_.precision == MLMC_FP64)
    run(double());
  else
    run(float());
}

void Context::restrict_fp64(int level, int nrhs, const double* x, double* xc) {
  MLMC_REQUIRE(level >= 1 && level < Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nrhs >= 1, MLMC_EINVAL, "nrhs must be >= 1");
  restrict64(level, x, xc, nrhs);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

void Context::prolong_fp64(int level, int nrhs, const double* xc, double* x) {
  MLMC_REQUIRE(level >= 1 && level < Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nrhs >= 1, MLMC_EINVAL, "nrhs must be >= 1");
  if (complex_)
    cop_prolong<c64>(level, reinterpret_cast<const c64*>(xc), reinterpret_cast<c64*>(x), nrhs,
                     nullptr, 1.0, 0.0);
  else
    op_prolong<double>(level, xc, x, nrhs, nullptr, 0.0);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

void Context::probes_fp64(int level, uint64_t seed, int stream, int64_t first, int nrhs,
                          double* out) {
  MLMC_REQUIRE(level >= 1 && level <= Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nrhs >= 1 && first >= 0 && stream >= 0, MLMC_EINVAL, "bad probe range");
  write_probes(level, seed, (uint64_t)stream, (uint64_t)first, nrhs, out);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

void Context::export_coarse(int which, double* out) {
  const int level = which == 1 ? L_ : Ls_;
  const Level& L = lv_[level - 1];
  const int n = (int)L.n;
  const int elem = complex_ ? 2 : 1;
  double* aug = dalloc_n<double>(2 * (int64_t)n * n * elem);
  if (complex_)
    dense_from_stencil(L.wilson ? nullptr : L.B64, L.U64, op_.mass + 2.0, L.side, L.dof,
                       reinterpret_cast<c64*>(aug), s_);
  else if (varcoef_)
    varcoef_dense(L.kf64, L.dg64, L.side, aug, s_);
  else if (csr_)
    csr_dense(L.A64, aug, s_);
  else
    poisson_dense_build<double>(aug, L.side, L.d, L.c, s_);
  for (int i = 0; i < n; ++i)
    MLMC_HIP(hipMemcpyAsync(out + (size_t)i * n * elem, aug + (size_t)i * 2 * n * elem,
                            sizeof(double) * n * elem, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
}

void Context::export_prolongation(int level, double* out) {
  MLMC_REQUIRE(complex_, MLMC_EUNSUPPORTED,
               "prolongation export is for test-vector aggregation only");
  MLMC_REQUIRE(level >= 1 && level < Ls_, MLMC_EINVAL, "level out of range");
  const Level& L = lv_[level - 1];
  MLMC_HIP(hipMemcpyAsync(out, L.q64, sizeof(c64) * (size_t)L.n * lv_[level].dof,
                          hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
}

template void Context::second_coarse_cycle<float>(int, const float*, float*, int, const int*,
                                                  bool);
template void Context::second_coarse_cycle<double>(int, const double*, double*, int, const int*,
                                                   bool);
template void Context::vcycle<float>(int, const float*, float*, int, const int*, c64*, bool,
                                      const float*);
template void Context::vcycle<double>(int, const double*, double*, int, const int*, c64*, bool,
                                       const double*);

}  // namespace mlmc
