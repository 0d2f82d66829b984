// Deflated Hutchinson, the comparison method of Sec. 5 (Sec. 4.2 eqs. orth_proj
// and defl): tr(A^{-1}) = tr(A^{-1}(I - Pi)) + tr(A^{-1} Pi) with Pi = U U^H
// for the n_defl eigenvectors of the smallest eigenvalues of a Hermitian A.
// The first trace is estimated with Hutchinson samples x^H A^{-1} (x - U U^H x)
// (the 2 n n_defl projection work per sample that Sec. 5 counts), the second is
// computed directly as tr(U^H A^{-1} U) (= sum 1/lambda_i for exact
// eigenvectors; exact split for approximate ones).
//
// The eigenvectors come from block subspace iteration with the library's own
// multigrid-preconditioned solves: W = A^{-1} V, orthonormalisation by two
// passes of Cholesky QR, Rayleigh-Ritz on span(W) (dense symmetric eigenproblem
// of the m x m projected matrix by cyclic Jacobi rotations on the host), until
// the first n_defl Ritz pairs have relative residuals |A v - theta v| / theta
// below eig_tol.  Real symmetric operators (POISSON2D, VARCOEF3D, CSR).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "context.h"

namespace mlmc {

namespace {

constexpr uint64_t kStreamDeflStart = 6;  // RNG stream of the start block

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// eigenvalues (ascending) and orthonormal eigenvectors (columns of V, row-major
// m x m) of a symmetric matrix S (row-major, destroyed), by cyclic Jacobi
// rotations: each rotation J = [[c, s], [-s, c]] in the (p, q) plane is chosen
// so that (J^T S J)_pq = 0 (Golub and Van Loan, symmetric Schur decomposition)
void jacobi_eigh(std::vector<double>& S, int m, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  auto at = [&](int i, int j) -> double& { return S[(size_t)i * m + j]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < m; ++i) {
      dia += at(i, i) * at(i, i);
      for (int j = i + 1; j < m; ++j) off += at(i, j) * at(i, j);
    }
    if (off <= 1e-30 * dia || off == 0.0) break;
    for (int p = 0; p < m; ++p) {
      for (int q = p + 1; q < m; ++q) {
        const double apq = at(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        const double tau = (at(q, q) - at(p, p)) / (2.0 * apq);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < m; ++k) {  // S <- S J
          const double skp = at(k, p), skq = at(k, q);
          at(k, p) = c * skp - s * skq;
          at(k, q) = s * skp + c * skq;
        }
        for (int k = 0; k < m; ++k) {  // S <- J^T S
          const double spk = at(p, k), sqk = at(q, k);
          at(p, k) = c * spk - s * sqk;
          at(q, k) = s * spk + c * sqk;
        }
        for (int k = 0; k < m; ++k) {  // V <- V J
          double* vr = &V[(size_t)k * m];
          const double vkp = vr[p], vkq = vr[q];
          vr[p] = c * vkp - s * vkq;
          vr[q] = s * vkp + c * vkq;
        }
      }
    }
  }
  std::vector<int> ord(m);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return at(a, a) < at(b, b); });
  w.resize(m);
  std::vector<double> Vs((size_t)m * m);
  for (int j = 0; j < m; ++j) {
    w[j] = at(ord[j], ord[j]);
    for (int i = 0; i < m; ++i) Vs[(size_t)i * m + j] = V[(size_t)i * m + ord[j]];
  }
  V.swap(Vs);
}

// R^{-1} for the Cholesky factor R (upper, G = R^T R) of a symmetric positive
// definite G (row-major m x m); false if G is not numerically positive definite
bool chol_inverse_factor(const std::vector<double>& G, int m, std::vector<double>& Rinv) {
  std::vector<double> R((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double d = G[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= R[(size_t)k * m + j] * R[(size_t)k * m + j];
    if (!(d > 0.0)) return false;
    const double rjj = std::sqrt(d);
    R[(size_t)j * m + j] = rjj;
    for (int i = j + 1; i < m; ++i) {
      double v = G[(size_t)j * m + i];
      for (int k = 0; k < j; ++k) v -= R[(size_t)k * m + j] * R[(size_t)k * m + i];
      R[(size_t)j * m + i] = v / rjj;
    }
  }
  // back substitution column by column: R Rinv = I, Rinv upper triangular
  Rinv.assign((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    for (int i = j; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) v -= R[(size_t)i * m + k] * Rinv[(size_t)k * m + j];
      Rinv[(size_t)i * m + j] = v / R[(size_t)i * m + i];
    }
  }
  return true;
}

}  // namespace

void Context::defl_require() const {
  MLMC_REQUIRE(!complex_, MLMC_EUNSUPPORTED,
               "deflated Hutchinson is implemented for the real symmetric operator kinds");
}

// C (ma x mb, row-major, device) = A^T B for RHS-major blocks A [ma][n], B [mb][n]
void Context::defl_gram(const double* A, int ma, const double* B, int mb, double* C) {
  const int64_t n = lv_[0].n;
  const int nch = gram_chunks(n, ma, mb);
  const int64_t need = (int64_t)nch * ma * mb;
  if (need > defl_part_cap_) {
    if (defl_part_) dfree(defl_part_);
    defl_part_ = dalloc_n<double>(need);
    defl_part_cap_ = need;
  }
  gram_partials(A, ma, B, mb, n, nch, defl_part_, s_);
  gram_finish(defl_part_, nch, ma, mb, C, s_);
}

std::vector<double> Context::defl_gram_host(const double* A, int ma, const double* B, int mb) {
  defl_gram(A, ma, B, mb, defl_small_);
  std::vector<double> h((size_t)ma * mb);
  MLMC_HIP(hipMemcpyAsync(h.data(), defl_small_, sizeof(double) * h.size(),
                          hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  return h;
}

// Y = A^{-1} X column batch by column batch (the samples' solver); false if a
// column missed the solve tolerance
bool Context::defl_solve_block(const double* X, double* Y, int m) {
  const int64_t n = lv_[0].n;
  bool all = true;
  for (int j = 0; j < m; j += nb_) {
    const int nbt = std::min(nb_, m - j);
    bool ok = true;
    solve(1, X + (int64_t)j * n, Y + (int64_t)j * n, nbt, scal_[kErr1], nullptr, &ok);
    all = all && ok;
  }
  return all;
}

// Y = A X on level 1 in FP64 (the operator product of mlmc_apply; the residual
// kernels of the real kinds always read a right-hand side)
void Context::defl_apply_block(const double* X, double* Y, int m) {
  const int64_t n = lv_[0].n;
  for (int j = 0; j < m; j += nb_) {
    const int nbt = std::min(nb_, m - j);
    op_apply<double>(1, X + (int64_t)j * n, Y + (int64_t)j * n, nbt, nullptr, nullptr);
  }
}

void Context::deflation_setup(const mlmc_deflation_options& o, mlmc_deflation_report* rep) {
  defl_require();
  const int64_t n = lv_[0].n;
  const int k = o.n_defl;
  const int p = o.oversample > 0 ? o.oversample : std::max(8, k / 2);
  MLMC_REQUIRE(k >= 1 && k <= 1024, MLMC_EINVAL, "n_defl must be in [1, 1024]");
  MLMC_REQUIRE((int64_t)(k + p) <= n, MLMC_EINVAL, "n_defl + oversample exceeds the unknowns");
  MLMC_REQUIRE(o.eig_tol > 0 && o.max_iter >= 1, MLMC_EINVAL,
               "eig_tol must be > 0 and max_iter >= 1");
  const int m = k + p;
  const double t0 = now_s();
  // work blocks (kept: V holds the Ritz vectors afterwards)
  for (double* q : {defl_V_, defl_W_, defl_Z_, defl_small_}) dfree(q);
  defl_V_ = dalloc_n<double>((int64_t)m * n);
  defl_W_ = dalloc_n<double>((int64_t)m * n);
  defl_Z_ = dalloc_n<double>((int64_t)m * n);
  defl_small_ = dalloc_n<double>((int64_t)m * std::max(m, nb_));
  defl_k_ = 0;
  // start block: Rademacher vectors of their own RNG stream, orthonormalised
  for (int j = 0; j < m; j += nb_) {
    const int nbt = std::min(nb_, m - j);
    probes_write<double>(defl_W_ + (int64_t)j * n, n, nbt, o.seed, 0, (uint64_t)j, 1,
                         kStreamDeflStart, s_);
  }
  // orthonormalise src into dst by two passes of Cholesky QR (dst <- src R^{-1})
  auto cholqr = [&](double* src, double* dst, double* tmp) {
    std::vector<double> Rinv;
    for (int pass = 0; pass < 2; ++pass) {
      double* from = pass == 0 ? src : tmp;
      double* to = pass == 0 ? tmp : dst;
      std::vector<double> G = defl_gram_host(from, m, from, m);
      if (!chol_inverse_factor(G, m, Rinv)) {
        // nearly dependent columns: a small diagonal shift keeps the first pass
        // defined; the second pass restores orthonormality
        double tr = 0.0;
        for (int i = 0; i < m; ++i) tr += G[(size_t)i * m + i];
        for (int i = 0; i < m; ++i) G[(size_t)i * m + i] += 1e-12 * tr / m;
        MLMC_REQUIRE(chol_inverse_factor(G, m, Rinv), MLMC_ENOCONV,
                     "deflation: the iterated block lost rank");
      }
      MLMC_HIP(hipMemcpyAsync(defl_small_, Rinv.data(), sizeof(double) * Rinv.size(),
                              hipMemcpyHostToDevice, s_));
      block_combine(from, m, defl_small_, m, nullptr, to, m, n, 1.0, 0.0, s_);
    }
  };
  cholqr(defl_W_, defl_V_, defl_Z_);
  const double saved_tol = opt_.solve_tol;
  const double it_tol = o.solve_tol > 0 ? o.solve_tol : 1e-8;
  std::vector<double> theta, Q;
  double maxres = INFINITY;
  int it = 0;
  int64_t solves = 0;
  for (it = 1; it <= o.max_iter; ++it) {
    opt_.solve_tol = it_tol;
    bool ok = true;
    try {
      ok = defl_solve_block(defl_V_, defl_W_, m);  // W = A^{-1} V
    } catch (...) {
      opt_.solve_tol = saved_tol;
      throw;
    }
    opt_.solve_tol = saved_tol;
    solves += m;
    MLMC_REQUIRE(ok, MLMC_ENOCONV, "deflation: a subspace-iteration solve missed its tolerance");
    cholqr(defl_W_, defl_W_, defl_Z_);       // W orthonormal (Z scratch)
    defl_apply_block(defl_W_, defl_Z_, m);   // Z = A W
    std::vector<double> H = defl_gram_host(defl_W_, m, defl_Z_, m);
    for (int i = 0; i < m; ++i)  // symmetrise the projected operator
      for (int j = i + 1; j < m; ++j) {
        const double v = 0.5 * (H[(size_t)i * m + j] + H[(size_t)j * m + i]);
        H[(size_t)i * m + j] = v;
        H[(size_t)j * m + i] = v;
      }
    std::vector<double> G2 = defl_gram_host(defl_Z_, m, defl_Z_, m);  // (AW)^T (AW)
    jacobi_eigh(H, m, theta, Q);
    // Ritz vectors V = W Q; residuals |A v_i - theta_i v_i|^2 = |A W q_i|^2 - theta_i^2
    MLMC_HIP(hipMemcpyAsync(defl_small_, Q.data(), sizeof(double) * Q.size(),
                            hipMemcpyHostToDevice, s_));
    block_combine(defl_W_, m, defl_small_, m, nullptr, defl_V_, m, n, 1.0, 0.0, s_);
    maxres = 0.0;
    for (int i = 0; i < k; ++i) {
      double a2 = 0.0;
      for (int r = 0; r < m; ++r) {
        double row = 0.0;
        for (int c = 0; c < m; ++c) row += G2[(size_t)r * m + c] * Q[(size_t)c * m + i];
        a2 += Q[(size_t)r * m + i] * row;
      }
      const double res = std::sqrt(std::max(a2 - theta[i] * theta[i], 0.0)) / std::fabs(theta[i]);
      maxres = std::max(maxres, res);
    }
    if (maxres <= o.eig_tol) break;
  }
  if (it > o.max_iter) it = o.max_iter;
  MLMC_REQUIRE(theta[0] > 0.0, MLMC_EINVAL, "deflation: the operator is not positive definite");
  // the direct term tr(U^H A^{-1} U) with U = the first k Ritz vectors, solved
  // to the context's tolerance: W = A^{-1} U, sum_i u_i^T w_i
  MLMC_REQUIRE(defl_solve_block(defl_V_, defl_W_, k), MLMC_ENOCONV,
               "deflation: a direct-term solve missed solve_tol");
  solves += k;
  defl_lambda_.assign(theta.begin(), theta.begin() + k);
  defl_k_ = k;
  double direct = 0.0, sinv = 0.0;
  {
    // per-vector dots u_i^T w_i in fixed order (batches of nb columns)
    std::vector<c64> d(nb_);
    for (int j = 0; j < k; j += nb_) {
      const int nbt = std::min(nb_, k - j);
      vec_dot_partials<double>(defl_V_ + (int64_t)j * n, defl_W_ + (int64_t)j * n, n, nbt, nullptr,
                               partials_, s_);
      finish_sums(partials_, reduce_blocks(n), nbt, scal_[kTmp], s_);
      MLMC_HIP(hipMemcpyAsync(d.data(), scal_[kTmp], sizeof(c64) * nbt, hipMemcpyDeviceToHost,
                              s_));
      MLMC_HIP(hipStreamSynchronize(s_));
      for (int i = 0; i < nbt; ++i) direct += d[i].re;
    }
  }
  for (int i = 0; i < k; ++i) sinv += 1.0 / defl_lambda_[i];
  defl_direct_ = direct;
  MLMC_HIP(hipGetLastError());
  if (rep) {
    rep->iterations = it;
    rep->seconds = now_s() - t0;
    rep->max_residual = maxres;
    rep->direct_trace = direct;
    rep->sum_inv_eig = sinv;
    rep->solves = solves;
  }
}

void Context::deflated_batch(uint64_t seed, uint64_t first, int nbatch, c64* out,
                             double* err_out) {
  MLMC_REQUIRE(defl_k_ > 0, MLMC_ESTATE, "no deflation set up (mlmc_deflation_setup)");
  MLMC_REQUIRE(nbatch >= 1 && nbatch <= nb_, MLMC_EINVAL, "batch size out of range");
  const int64_t n = lv_[0].n;
  // x (plain Hutchinson probes), C = U^T x, x_perp = x - U C in place
  write_probes(1, seed, kStreamHutch, first, nbatch, b1_);
  defl_gram(defl_V_, defl_k_, b1_, nbatch, defl_small_);
  block_combine(defl_V_, defl_k_, defl_small_, nbatch, b1_, b1_, nbatch, n, -1.0, 1.0, s_);
  bool ok = true;
  solve(1, b1_, y1_, nbatch, scal_[kErr1], nullptr, &ok);
  const std::vector<char> okc = col_ok_;
  // x^H A^{-1} x_perp with x regenerated
  probe_quad(1, seed, kStreamHutch, first, nbatch, y1_, scal_[kQa]);
  vec_zero<c64>(scal_[kErr2], 1, nbatch, nullptr, s_);
  vec_zero<c64>(scal_[kQb], 1, nbatch, nullptr, s_);
  finish_samples(1, nbatch, okc.data(), nullptr, first, out, err_out);
}

void Context::deflated_sample(uint64_t seed, int64_t first, int64_t count, double* out,
                              double* out_err) {
  MLMC_REQUIRE(first >= 0 && count >= 1, MLMC_EINVAL, "bad sample range");
  std::memset(counters, 0, sizeof(counters));
  std::vector<c64> buf(nb_);
  std::vector<double> eb(nb_);
  for (int64_t j = 0; j < count; j += nb_) {
    const int nbt = (int)std::min<int64_t>(nb_, count - j);
    auto copy_out = [&] {
      for (int i = 0; i < nbt; ++i) {
        out[2 * (j + i)] = buf[i].re;
        out[2 * (j + i) + 1] = buf[i].im;
        if (out_err) out_err[j + i] = eb[i];
      }
    };
    try {
      deflated_batch(seed, (uint64_t)(first + j), nbt, buf.data(), eb.data());
    } catch (const Error& e) {
      if (e.code == MLMC_ENOCONV) copy_out();  // partial results
      throw;
    }
    copy_out();
  }
}

void Context::deflated_hutchinson(double tol, uint64_t seed, mlmc_result* out) {
  MLMC_REQUIRE(defl_k_ > 0, MLMC_ESTATE, "no deflation set up (mlmc_deflation_setup)");
  std::memset(counters, 0, sizeof(counters));
  auto sample = [&](int64_t first, int64_t count, c64* o) {
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      deflated_batch(seed, (uint64_t)(first + j), nbt, o + j, nullptr);
    }
  };
  // tau from the plain pilot of Sec. 5 (the same five estimates as MLMC and
  // plain Hutchinson use)
  auto pilot = [&](int64_t count, c64* o) {
    for (int64_t j = 0; j < count; j += nb_) {
      const int nbt = (int)std::min<int64_t>(nb_, count - j);
      hutch_batch(seed, kStreamPilot, (uint64_t)j, nbt, o + j);
    }
  };
  run_hutchinson(sample, pilot, opt_, tol, out);
  out->trace[0] += defl_direct_;
  out->coarse_trace[0] = defl_direct_;  // the direct term tr(A^{-1} Pi)
  out->coarse_trace[1] = 0.0;
  out->solves = out->n_samples[0] + (opt_.tau > 0 ? 0 : 5);
  out->iterations = counters[0];
}

void Context::deflation_export(double* eigenvalues, double* vectors_dev, double* direct) {
  MLMC_REQUIRE(defl_k_ > 0, MLMC_ESTATE, "no deflation set up (mlmc_deflation_setup)");
  if (eigenvalues)
    std::memcpy(eigenvalues, defl_lambda_.data(), sizeof(double) * defl_lambda_.size());
  if (vectors_dev) {
    MLMC_HIP(hipMemcpyAsync(vectors_dev, defl_V_, sizeof(double) * (size_t)defl_k_ * lv_[0].n,
                            hipMemcpyDeviceToDevice, s_));
    MLMC_HIP(hipStreamSynchronize(s_));
  }
  if (direct) *direct = defl_direct_;
}

}  // namespace mlmc
