// Complex lattice operators: the Wilson-like 2-spin operator and its
// test-vector aggregation hierarchy (Example 4.3), a V-cycle with red-black
// block Gauss-Seidel smoothing, and batched flexible GMRES inside FP64
// iterative refinement (each restart cycle is one refinement step).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "context.h"

namespace mlmc {

template <> const c32* Context::links<c32>(int l) const { return lv_[l - 1].U32; }
template <> const c64* Context::links<c64>(int l) const { return lv_[l - 1].U64; }
template <> const c32* Context::blocks<c32>(int l) const { return lv_[l - 1].B32; }
template <> const c64* Context::blocks<c64>(int l) const { return lv_[l - 1].B64; }
template <> const c32* Context::dinv<c32>(int l) const { return lv_[l - 1].Dinv32; }
template <> const c64* Context::dinv<c64>(int l) const { return lv_[l - 1].Dinv64; }
template <> const c32* Context::qmat<c32>(int l) const { return lv_[l - 1].q32; }
template <> const c64* Context::qmat<c64>(int l) const { return lv_[l - 1].q64; }
template <> Work<c32>& Context::work<c32>() { return wc32_; }
template <> Work<c64>& Context::work<c64>() { return wc64_; }
template <> Fgmres<c32>& Context::fg<c32>() { return fg32_; }
template <> Fgmres<c64>& Context::fg<c64>() {
  MLMC_REQUIRE(fg64_.V != nullptr, MLMC_ESTATE, "FP64 FGMRES buffers exist in MLMC_FP64 mode only");
  return fg64_;
}

// ---------------------------------------------------------------------------
// setup (Example 4.3 aggregation sketch): on each level, n_vec Z4 start
// vectors (Philox stream 2, sample j, this level) are smoothed by
// `setup_sweeps` red-black block Gauss-Seidel sweeps on A v = 0 (FP64), then
// orthonormalised per aggregate of block x block sites (modified Gram-Schmidt:
// R with a positive real diagonal); the Galerkin product P^H A P gives the next
// level's 5-point block stencil.  The coarsest level is inverted densely.
// ---------------------------------------------------------------------------
void Context::build_wilson(const double* theta) {
  const int N = op_.n_side, blk = h_.block, nv = h_.n_vec;
  // GAUGE2D: the finest level is a 1 x 1 block stencil of the gauge Laplacian
  const bool gauge = kind_ == MLMC_GAUGE2D;
  // coarse unknowns per site: the test vectors, doubled by the spin split
  const bool split = h_.spin_split != 0;
  const int nc = split ? 2 * nv : nv;
  MLMC_REQUIRE(theta != nullptr, MLMC_EINVAL, "WILSON2D and GAUGE2D need the link phases (field)");
  MLMC_REQUIRE(N >= 2 && blk >= 2, MLMC_EINVAL, "bad lattice or aggregate size");
  MLMC_REQUIRE(nv >= 1 && (nc == 2 || nc == 4 || nc == 8 || nc == 12 || nc == 16),
               MLMC_EUNSUPPORTED,
               "coarse unknowns per site (n_vec, doubled by spin_split) must be one of 2, 4, 8, "
               "12, 16");
  MLMC_REQUIRE(h_.setup_sweeps >= 0, MLMC_EINVAL, "setup_sweeps must be >= 0");
  MLMC_REQUIRE(opt_.krylov_restart >= 1 && opt_.krylov_restart <= 32, MLMC_EINVAL,
               "krylov_restart must be in [1, 32]");
  m_ = opt_.krylov_restart;
  const double diag = op_.mass + 2.0;
  lv_.resize(Ls_);
  int side = N;
  for (int l = 0; l < Ls_; ++l) {
    if (l > 0) {
      MLMC_REQUIRE(side % blk == 0, MLMC_EINVAL,
                   "lattice side not divisible by the aggregate side at level " +
                       std::to_string(l));
      side /= blk;
    }
    Level& L = lv_[l];
    L.index = l + 1;
    L.side = side;
    L.dof = l == 0 ? (gauge ? 1 : 2) : nc;
    L.n = (int64_t)side * side * L.dof;
    L.wilson = (l == 0) && !gauge;
    L.blk = blk;
    if (l < Ls_ - 1)
      MLMC_REQUIRE(side % 2 == 0, MLMC_EINVAL,
                   "smoothed levels need an even lattice side (red-black colouring)");
  }
  MLMC_REQUIRE(lv_[Ls_ - 1].n <= 16384, MLMC_EINVAL, "coarsest level too large (n > 16384)");
  alloc_common();
  const int64_t n1 = lv_[0].n;

  // links
  double* th = dalloc_n<double>(2 * (int64_t)N * N);
  MLMC_HIP(hipMemcpyAsync(th, theta, sizeof(double) * 2 * N * N, hipMemcpyHostToDevice, s_));
  theta_dev_ = th;
  lv_[0].U64 = dalloc_n<c64>(2 * (int64_t)N * N);
  lv_[0].U32 = dalloc_n<c32>(2 * (int64_t)N * N);
  wilson_links(th, lv_[0].U64, lv_[0].U32, N, s_);
  if (gauge) {
    Level& F = lv_[0];
    const int64_t ns = (int64_t)N * N;
    F.B64 = dalloc_n<c64>(ns * 5);
    F.B32 = dalloc_n<c32>(ns * 5);
    F.Dinv64 = dalloc_n<c64>(ns);
    F.Dinv32 = dalloc_n<c32>(ns);
    gauge_blocks(F.U64, N, 4.0 + op_.mass, F.B64, s_);
    vec_convert<c32, c64>(F.B64, F.B32, ns * 5, 1, nullptr, s_);
    block_diag_inverse(F.B64, F.Dinv64, F.Dinv32, (int)ns, 1, s_);
  }

  // hierarchy
  for (int l = 1; l < Ls_; ++l) {
    Level& F = lv_[l - 1];
    Level& C = lv_[l];
    c64* V = dalloc_n<c64>(F.n * nv);
    c64* zero = dalloc_n<c64>(F.n * nv);
    vec_zero<c64>(zero, F.n, nv, nullptr, s_);
    probes_write<c64>(V, F.n, nv, h_.setup_seed, 0, 0, (uint64_t)l, 2, s_);
    for (int sw = 0; sw < h_.setup_sweeps; ++sw) {
      if (F.wilson)
        wilson_rbgs<c64>(zero, V, F.U64, F.side, diag, nv, nullptr, false, false, s_);
      else
        bsr_rbgs<c64>(zero, V, F.B64, F.Dinv64, F.side, F.dof, nv, nullptr, false, false, 0, s_);
    }
    F.q64 = dalloc_n<c64>(F.n * nc);
    F.q32 = dalloc_n<c32>(F.n * nc);
    agg_orthonormalise(V, F.q64, F.side, F.dof, blk, nv, split, s_);
    vec_convert<c32, c64>(F.q64, F.q32, F.n * nc, 1, nullptr, s_);
    const int64_t nsc = (int64_t)C.side * C.side;
    C.B64 = dalloc_n<c64>(nsc * 5 * nc * nc);
    C.B32 = dalloc_n<c32>(nsc * 5 * nc * nc);
    galerkin_blocks(F.wilson ? nullptr : F.B64, F.U64, diag, F.q64, F.side, F.dof, blk, nc, C.B64,
                    s_);
    vec_convert<c32, c64>(C.B64, C.B32, nsc * 5 * nc * nc, 1, nullptr, s_);
    C.Dinv64 = dalloc_n<c64>(nsc * nc * nc);
    C.Dinv32 = dalloc_n<c32>(nsc * nc * nc);
    block_diag_inverse(C.B64, C.Dinv64, C.Dinv32, (int)nsc, nc, s_);
  }

  // work buffers
  auto alloc_cwork = [&](auto& w) {
    using T = std::remove_pointer_t<decltype(w.x)>;
    w.vb.assign(Ls_, nullptr);
    w.vx.assign(Ls_, nullptr);
    w.vt.assign(Ls_, nullptr);
    w.vr2.assign(Ls_, nullptr);
    w.ve2.assign(Ls_, nullptr);
    for (int m = 0; m < Ls_; ++m) {
      if (m > 0) {
        w.vb[m] = dalloc_n<T>(lv_[m].n * nb_);
        w.vx[m] = dalloc_n<T>(lv_[m].n * nb_);
      }
      w.vt[m] = dalloc_n<T>(lv_[m].n * nb_);
      if (top_cycles_ == 2 && m > 0 && m < Ls_ - 1) {  // second coarse-grid cycle
        w.vr2[m] = dalloc_n<T>(lv_[m].n * nb_);
        w.ve2[m] = dalloc_n<T>(lv_[m].n * nb_);
      }
    }
  };
  auto alloc_fg = [&](auto& f) {
    using T = std::remove_pointer_t<decltype(f.V)>;
    f.V = dalloc_n<T>(n1 * nb_ * (m_ + 1));
    f.Z = dalloc_n<T>(n1 * nb_ * m_);
    f.r = dalloc_n<T>(n1 * nb_);
    f.d = dalloc_n<T>(n1 * nb_);
  };
  alloc_cwork(wc64_);
  if (opt_.precision == MLMC_FP64) alloc_fg(fg64_);  // the FP32 mode iterates in fg32_
  if (opt_.precision == MLMC_FP32_IR64) {
    alloc_cwork(wc32_);
    alloc_fg(fg32_);
  }
  gH_ = dalloc_n<c64>((int64_t)nb_ * (m_ + 1) * m_);
  gcs_ = dalloc_n<c64>((int64_t)nb_ * m_);
  gsn_ = dalloc_n<c64>((int64_t)nb_ * m_);
  gg_ = dalloc_n<c64>((int64_t)nb_ * (m_ + 1));
  gy_ = dalloc_n<c64>((int64_t)nb_ * m_);
  ghcol_ = dalloc_n<c64>((int64_t)nb_ * (m_ + 1));
  gdims_ = dalloc_n<int>(nb_);
  gstart_ = dalloc_n<int>(nb_);

  // coarsest inverses (complex FP64), direct trace term (Remark 4.2)
  auto invert = [&](int level, c64** inv_out, c64* tr) {
    const Level& L = lv_[level - 1];
    const int n = (int)L.n;
    c64* aug = dalloc_n<c64>(2 * (int64_t)n * n);  // the builder's layout: n x 2n
    dense_from_stencil(L.wilson ? nullptr : L.B64, L.U64, diag, L.side, L.dof, aug, s_);
    c64* inv = dalloc_n<c64>((int64_t)n * n);
    dense_invert_checked<c64>(aug, n, inv);
    dense_trace<c64>(inv, n, scal_[kTmp], s_);
    MLMC_HIP(hipMemcpyAsync(host_c64_, scal_[kTmp], sizeof(c64), hipMemcpyDeviceToHost, s_));
    MLMC_HIP(hipStreamSynchronize(s_));
    *tr = host_c64_[0];
    *inv_out = inv;
    dfree(aug);
  };
  c64* inv_s = nullptr;
  c64 tr_s;
  invert(Ls_, &inv_s, &tr_s);
  const int ns = (int)lv_[Ls_ - 1].n;
  wc64_.ainvT = dalloc_n<c64>((int64_t)ns * ns);
  dense_transpose<c64>(inv_s, wc64_.ainvT, ns, s_);
  if (opt_.precision == MLMC_FP32_IR64) {
    wc32_.ainvT = dalloc_n<c32>((int64_t)ns * ns);
    vec_convert<c32, c64>(wc64_.ainvT, wc32_.ainvT, (int64_t)ns * ns, 1, nullptr, s_);
  }
  // the coarsest solve as a real MFMA product with the 2n x 2n real
  // representation (interleaved complex vectors are real vectors of length 2n)
  // (in the MFMA tile kernel's layout)
  if (dense_mfma_layout<double>(2 * ns)) {
    double* plain = dalloc_n<double>(4 * (int64_t)ns * ns);
    dense_complex_to_real<c64, double>(wc64_.ainvT, plain, ns, s_);
    wc64_.ainvR = dalloc_n<double>(4 * (int64_t)ns * ns);
    dense_pack4<double>(plain, wc64_.ainvR, 2 * ns, s_);
    dfree(plain);
    if (opt_.precision == MLMC_FP32_IR64) {
      float* plain32 = dalloc_n<float>(4 * (int64_t)ns * ns);
      dense_complex_to_real<c32, float>(wc32_.ainvT, plain32, ns, s_);
      wc32_.ainvR = dalloc_n<float>(4 * (int64_t)ns * ns);
      dense_pack4<float>(plain32, wc32_.ainvR, 2 * ns, s_);
      dfree(plain32);
    }
  }
  if (L_ == Ls_) {
    coarse_trace_ = tr_s;
  } else {
    c64* inv_m = nullptr;
    invert(L_, &inv_m, &coarse_trace_);
  }
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
  tune_bsr();
}

// Autotuner of the block-stencil kernels: per smoothed block level and per
// precision the V-cycle runs (complex64 in the refined mode, complex128 in the
// plain FP64 mode), time one red-black sweep over all nb columns in both
// kernel forms (best of 3 after a warm-up) and keep the faster.  The two forms
// agree up to rounding; runs once at setup on the level's work vectors.
void Context::tune_bsr() {
  hipEvent_t a = event(), b = event();
  auto time_form = [&](auto tag, Level& L, int l, int form) {
    using T = decltype(tag);
    Work<T>& w = work<T>();
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      MLMC_HIP(hipEventRecord(a, s_));
      bsr_rbgs<T>(w.vb[l - 1], w.vx[l - 1], blocks<T>(l), dinv<T>(l), L.side, L.dof, nb_,
                  nullptr, rep == 0, false, form, s_);
      MLMC_HIP(hipEventRecord(b, s_));
      MLMC_HIP(hipEventSynchronize(b));
      float t = 0.f;
      MLMC_HIP(hipEventElapsedTime(&t, a, b));
      if (rep > 0) best = std::min(best, t);
    }
    return best;
  };
  for (int l = 2; l < Ls_; ++l) {
    Level& L = lv_[l - 1];
    if (opt_.precision == MLMC_FP32_IR64)
      L.bsr_form[0] = time_form(c32(), L, l, 1) < time_form(c32(), L, l, 0) ? 1 : 0;
    else
      L.bsr_form[1] = time_form(c64(), L, l, 1) < time_form(c64(), L, l, 0) ? 1 : 0;
  }
  ev_pool_.push_back(a);
  ev_pool_.push_back(b);
}

// ---------------------------------------------------------------------------
// operator pieces
// ---------------------------------------------------------------------------
template <typename Tb, typename T, typename Tr>
void Context::cop_residual(int l, const Tb* b, const T* x, Tr* r, int nb, const int* act,
                           c64* partials) {
  const Level& L = lv_[l - 1];
  if (L.wilson)
    wilson_residual<Tb, T, Tr>(b, x, r, links<T>(l), L.side, op_.mass + 2.0, nb, act, partials,
                               s_);
  else
    bsr_residual<Tb, T, Tr>(b, x, r, blocks<T>(l), L.side, L.dof, nb, act, partials,
                            bsr_form<T>(L, nb), s_);
}

template <typename T>
void Context::cop_smooth(int l, const T* b, T* x, int nb, const int* act, bool zero_init,
                         bool reverse) {
  const Level& L = lv_[l - 1];
  if (L.wilson) {
    // algorithmic bytes per column: b and x read, x written (x read once more
    // by the second colour unless from zero), links once per launch
    const double es = 2.0 * sizeof(T) * (double)L.side * L.side;
    const double bytes = es * (zero_init ? 2.5 : 3.0) + es / (double)nb;
    timed<T>(l, kTimGs, bytes, act, nb, [&] {
      wilson_rbgs<T>(b, x, links<T>(l), L.side, op_.mass + 2.0, nb, act, zero_init, reverse, s_);
    });
  } else {
    // per column: b and x read, x written (dof complex values per site), the
    // site's 5 stencil blocks and inverted diagonal block once per launch
    const double es = (double)sizeof(T) * L.dof * (double)L.side * L.side;
    const double bytes = es * (zero_init ? 2.5 : 3.0) + 6.0 * L.dof * es / (double)nb;
    timed<T>(l, kTimGs, bytes, act, nb, [&] {
      bsr_rbgs<T>(b, x, blocks<T>(l), dinv<T>(l), L.side, L.dof, nb, act, zero_init, reverse,
                  bsr_form<T>(L, nb), s_);
    });
  }
}

// count sweeps at level l (from x = 0 when zero_init).  On the Wilson level
// they run as fused two-colour passes, out of place, alternating between x and
// the level's residual scratch (free while the level smooths) so that the last
// pass lands in x; an odd count from a given x starts with one in-place sweep.
template <typename T>
void Context::cop_smooth_n(int l, const T* b, T* x, int nb, const int* act, int count,
                           bool zero_init, bool reverse) {
  const Level& L = lv_[l - 1];
  if (!L.wilson || !wilson_rbgs_fused_ok(L.side)) {
    for (int i = 0; i < count; ++i) cop_smooth<T>(l, b, x, nb, act, zero_init && i == 0, reverse);
    return;
  }
  int i = 0;
  if (!zero_init && count % 2 == 1) {
    cop_smooth<T>(l, b, x, nb, act, false, reverse);
    i = 1;
  }
  T* tmp = work<T>().vt[l - 1];
  // algorithmic bytes per column: b read and x written (x read unless from
  // zero), links once per launch
  const double es = 2.0 * sizeof(T) * (double)L.side * L.side;
  for (; i < count; ++i) {
    const bool z = zero_init && i == 0;
    T* dst = ((count - 1 - i) % 2 == 0) ? x : tmp;
    const T* src = z ? dst : (dst == x ? tmp : x);
    const double bytes = es * (z ? 2.0 : 3.0) + es / (double)nb;
    timed<T>(l, kTimGs, bytes, act, nb, [&] {
      wilson_rbgs_fused<T>(b, src, dst, links<T>(l), L.side, op_.mass + 2.0, nb, act, z, reverse,
                           s_);
    });
  }
}

template <typename T>
void Context::cop_restrict(int l, const T* x, T* xc, int nb, const int* act) {
  const Level& L = lv_[l - 1];
  agg_restrict<T>(x, xc, qmat<T>(l), L.side, L.dof, L.blk, lv_[l].dof, nb, act, s_);
}

template <typename T>
void Context::cop_prolong(int l, const T* ec, T* x, int nb, const int* act, double omega,
                          double beta) {
  const Level& L = lv_[l - 1];
  agg_prolong<T>(ec, x, qmat<T>(l), L.side, L.dof, L.blk, lv_[l].dof, omega, beta, nb, act, s_);
}

// V-cycle on levels l..L_s: x = M b (pre-smoothing from zero, residual,
// restriction, recursion, prolongation with omega, post-smoothing in the
// reverse colour order)
// coarsest solve x = A_{L_s}^{-1} b of the complex hierarchy
template <typename T>
void Context::coarse_apply(const T* b, T* x, int nb, const int* act) {
  using R = typename Traits<T>::real;
  Work<T>& w = work<T>();
  const int n = (int)lv_[Ls_ - 1].n;
  if (w.ainvR)
    dense_apply<R>(w.ainvR, reinterpret_cast<const R*>(b), reinterpret_cast<R*>(x), 2 * n, nb,
                   act, s_);
  else
    dense_apply<T>(w.ainvT, b, x, n, nb, act, s_);
}

template <typename T>
void Context::csecond_coarse_cycle(int l, const T* bc, T* ec, int nb, const int* act, bool top) {
  if (!top || top_cycles_ != 2 || l + 1 >= Ls_) return;
  Work<T>& w = work<T>();
  T* r2 = w.vr2[l];
  T* e2 = w.ve2[l];
  cop_residual<T, T, T>(l + 1, bc, ec, r2, nb, act, nullptr);
  cvcycle<T>(l + 1, r2, e2, nb, act);
  vec_add_to<T>(ec, e2, lv_[l].n, nb, act, s_);
}

template <typename T>
void Context::cvcycle(int l, const T* b, T* x, int nb, const int* act, bool top) {
  Work<T>& w = work<T>();
  const int64_t n = lv_[l - 1].n;
  if (l == 1) counters[2] += 1;
  if (l == Ls_) {
    coarse_apply<T>(b, x, nb, act);
    return;
  }
  if constexpr (std::is_same<T, c32>::value) {
    if (l == 1 && nn_use_) {
      // learned finest level: sweep, network | coarse correction | network, sweep
      T* res = w.vt[0];
      cop_smooth<T>(l, b, x, nb, act, true, false);
      nn_step(b, x, nb, act);
      cop_residual<T, T, T>(l, b, x, res, nb, act, nullptr);
      cop_restrict<T>(l, res, w.vb[1], nb, act);
      cvcycle<T>(2, w.vb[1], w.vx[1], nb, act);
      csecond_coarse_cycle<T>(1, w.vb[1], w.vx[1], nb, act, top);
      cop_prolong<T>(l, w.vx[1], x, nb, act, omega_, 1.0);
      nn_step(b, x, nb, act);
      cop_smooth<T>(l, b, x, nb, act, false, true);
      return;
    }
  }
  const int pre = opt_.nu_pre, post = opt_.nu_post;
  if (pre == 0) vec_zero<T>(x, n, nb, act, s_);
  cop_smooth_n<T>(l, b, x, nb, act, pre, true, false);
  T* res = w.vt[l - 1];
  cop_residual<T, T, T>(l, b, x, res, nb, act, nullptr);
  cop_restrict<T>(l, res, w.vb[l], nb, act);
  cvcycle<T>(l + 1, w.vb[l], w.vx[l], nb, act);
  csecond_coarse_cycle<T>(l, w.vb[l], w.vx[l], nb, act, top);
  cop_prolong<T>(l, w.vx[l], x, nb, act, omega_, 1.0);
  cop_smooth_n<T>(l, b, x, nb, act, post, false, true);
}

// ---------------------------------------------------------------------------
// one cycle of right-preconditioned flexible GMRES(m) for A d = r, columns in
// lockstep (classical Gram-Schmidt; Givens rotations per column on the
// device).  act (in/out): columns to solve; a column stops at relative
// residual estimate tol.  d receives the correction for every column that was
// active on entry.
// ---------------------------------------------------------------------------
template <typename T>
void Context::fgmres_cycle(int l, const T* r, T* d, int nb, int* act, double tol) {
  Fgmres<T>& f = fg<T>();
  const int64_t n = lv_[l - 1].n;
  const int64_t vs = n * nb;  // stride between basis vectors
  const int nblk = reduce_blocks(n);
  c64 *beta2 = scal_[kRr0], *wn2 = scal_[kTmp];
  MLMC_HIP(hipMemcpyAsync(gstart_, act, sizeof(int) * nb, hipMemcpyDeviceToDevice, s_));
  vec_dot_partials<T>(r, r, n, nb, act, partials_, s_);
  finish_sums(partials_, nblk, nb, beta2, s_);
  vec_scale_inv_norm<T>(f.V, r, beta2, n, nb, act, s_);
  givens_init(gH_, gcs_, gsn_, gg_, gdims_, beta2, act, m_, nb, s_);
  // with opts.graphs (and no kernel timing) every iteration replays a HIP graph
  // captured once per (precision, level, batch width, iteration, smoother):
  // its launches, pointers and scalars (tol is the context's fixed inner
  // tolerance) are the same at every visit
  const bool use_graph = opt_.graphs && !timing_;
  for (hipEvent_t& e : fg_ev_)
    if (!e) MLMC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // Iteration j stores its count of active columns in count slot 5 + j % 2.
  // The host reads iteration j-1's count once iteration j is queued, so the
  // GPU does not drain between iterations; when that count is zero, iteration
  // j has run on no column (every kernel skips inactive columns) and the cycle
  // ends with the same state as if it had stopped after j-1.
  for (int j = 0; j < m_; ++j) {
    auto iteration = [&] {
      T* vj = f.V + j * vs;
      T* zj = f.Z + j * vs;
      T* w = f.V + (j + 1) * vs;
      cvcycle<T>(l, vj, zj, nb, act, true);
      cop_residual<T, T, T>(l, (const T*)nullptr, zj, w, nb, act, nullptr);
      int mb = 0;
      krylov_mdot<T>(f.V, vs, j + 1, w, n, nb, act, partials_, &mb, s_);
      finish_sums(partials_, mb, nb * (j + 1), ghcol_, s_);
      krylov_maxpy<T>(f.V, vs, j + 1, ghcol_, w, n, nb, act, s_);
      vec_dot_partials<T>(w, w, n, nb, act, partials_, s_);
      finish_sums(partials_, nblk, nb, wn2, s_);
      vec_scale_inv_norm<T>(w, w, wn2, n, nb, act, s_);
      givens_step(gH_, gcs_, gsn_, gg_, gdims_, ghcol_, wn2, beta2, tol, j, m_, act, nb,
                  count_map_ + 5 + (j & 1), s_);
    };
    if (use_graph)
      replay({sizeof(T) == sizeof(c32) ? 1 : 2, l, nb, j + (nn_use_ ? 64 : 0)}, iteration);
    else
      iteration();
    MLMC_HIP(hipEventRecord(fg_ev_[j & 1], s_));
    if (j > 0) {
      MLMC_HIP(hipEventSynchronize(fg_ev_[(j - 1) & 1]));
      if (count_host_[5 + ((j - 1) & 1)] == 0) break;
    }
    counters[0] += 1;
  }
  givens_solve(gH_, gcs_, gsn_, gg_, gdims_, gy_, gstart_, m_, nb, s_);
  krylov_combine<T>(f.Z, vs, gy_, m_, gdims_, d, n, nb, gstart_, s_);
}

// ---------------------------------------------------------------------------
// FP64 solve of a complex level: refinement loop y += d with d from one
// FGMRES cycle on the current FP64 residual (in complex64 for
// MLMC_FP32_IR64, complex128 for MLMC_FP64).  Converged when the FP64
// residual meets solve_tol.  err: stated error contribution per column (the
// last correction's |b^H d| scaled by the residual reduction it achieved).
// ---------------------------------------------------------------------------
void Context::solve_complex(int l, const c64* b, c64* y, int nb, c64* err) {
  const Level& L = lv_[l - 1];
  const int64_t n = L.n;
  const int nblk = reduce_blocks(n);
  const int rblk = L.wilson ? wilson_residual_blocks(L.side) : bsr_residual_blocks(L.side);
  c64 *bb = scal_[kBb], *bd = scal_[kBd], *rr_old = scal_[kRres], *rr_new = scal_[kRres2];
  const double tol = opt_.solve_tol;
  vec_dot_partials<c64>(b, b, n, nb, nullptr, partials_, s_);
  finish_sums(partials_, nblk, nb, bb, s_);
  set_all_active(act_outer_, nb, s_);
  vec_zero<c64>(err, 1, nb, nullptr, s_);
  if (l == Ls_) {
    coarse_apply<c64>(b, y, nb, nullptr);
    return;
  }
  vec_zero<c64>(y, n, nb, nullptr, s_);
  vec_copy<c64>(bb, rr_old, 1, nb, nullptr, s_);
  c64* res64 = reinterpret_cast<c64*>(r64_);
  const bool fp32 = opt_.precision == MLMC_FP32_IR64;
  // the learned smoother runs on the finest level of FP32 solves; the FP64
  // residual below stays the judge, and a cycle that reduces some column's
  // residual norm by less than 2x switches the rest of this solve to the plain
  // smoother
  nn_use_ = nn_ready_ && opt_.learned && fp32 && l == 1;
  struct Reset {
    bool& f;
    ~Reset() { f = false; }
  } reset{nn_use_};
  const double inner = fp32 ? std::max(opt_.inner_tol, 1e-6) : std::max(opt_.inner_tol, 1e-12);
  bool have_corr = false;
  for (int it = 0; it <= opt_.max_refine * 4; ++it) {
    // FP64 residual of the current iterate
    if (fp32)
      cop_residual<c64, c64, c32>(l, b, y, fg32_.r, nb, act_outer_, partials_);
    else
      cop_residual<c64, c64, c64>(l, b, y, fg64_.r, nb, act_outer_, partials_);
    finish_sums(partials_, rblk, nb, rr_new, s_);
    if (have_corr) ir_stated_error(bd, rr_old, rr_new, act_outer_, err, nb, s_);
    const bool guard = nn_use_ && have_corr;
    if (guard) {
      // columns that met a 2x norm reduction (or the tolerance) vs. all active
      refine_due(rr_new, rr_old, bb, 0.25, tol * tol, act_outer_, nb, count_map_ + 2, s_);
      count_active(act_outer_, nb, count_map_ + 3, s_);
    }
    select_active(rr_old, rr_new, act_outer_, nb, s_);
    mark_converged(rr_new, bb, tol * tol, act_outer_, nb, count_map_, s_);
    counters[1] += 1;
    if (guard) {
      MLMC_HIP(hipStreamSynchronize(s_));
      if (count_host_[2] < count_host_[3]) {
        nn_use_ = false;
        nn_stats[1] += 1;
      }
      if (count_host_[0] == 0) break;
    } else if (read_count() == 0) {
      break;
    }
    MLMC_HIP(hipMemcpyAsync(act_inner_, act_outer_, sizeof(int) * nb, hipMemcpyDeviceToDevice,
                            s_));
    if (fp32) {
      fgmres_cycle<c32>(l, fg32_.r, fg32_.d, nb, act_inner_, inner);
      ir_accumulate<c64, c32>(y, fg32_.d, n, nb, act_outer_, s_);
      vec_convert<c64, c32>(fg32_.d, res64, n, nb, act_outer_, s_);
    } else {
      fgmres_cycle<c64>(l, fg64_.r, fg64_.d, nb, act_inner_, inner);
      ir_accumulate<c64, c64>(y, fg64_.d, n, nb, act_outer_, s_);
      vec_copy<c64>(fg64_.d, res64, n, nb, act_outer_, s_);
    }
    vec_dot_partials<c64>(b, res64, n, nb, act_outer_, partials_, s_);
    finish_sums(partials_, nblk, nb, bd, s_);
    have_corr = true;
  }
}

template void Context::cop_residual<c64, c64, c64>(int, const c64*, const c64*, c64*, int,
                                                   const int*, c64*);
template void Context::cop_restrict<c64>(int, const c64*, c64*, int, const int*);
template void Context::cop_restrict<c32>(int, const c32*, c32*, int, const int*);
template void Context::cop_prolong<c64>(int, const c64*, c64*, int, const int*, double, double);
template void Context::cop_residual<c32, c32, c32>(int, const c32*, const c32*, c32*, int,
                                                   const int*, c64*);
template void Context::cop_smooth<c64>(int, const c64*, c64*, int, const int*, bool, bool);
template void Context::cop_smooth<c32>(int, const c32*, c32*, int, const int*, bool, bool);
template void Context::cop_smooth_n<c64>(int, const c64*, c64*, int, const int*, int, bool,
                                         bool);
template void Context::cop_smooth_n<c32>(int, const c32*, c32*, int, const int*, int, bool,
                                         bool);
template void Context::cvcycle<c64>(int, const c64*, c64*, int, const int*, bool);

}  // namespace mlmc
