// MLMC estimator and accuracy control on the host (Sec. 2 estimator, Sec. 5 control).
//
// tau: mean of five pilot plain-Hutchinson estimates minus their RMSD (Sec. 5);
// per-level RMSD targets rho_l with sum_l rho_l^2 = (eps tau)^2: equal split,
// given weights (Example 4.3) or the optimal allocation of Sec. 2
// (N_l ~ sqrt(V_l/C_l), multiplier eps^-2 sum_k sqrt(V_k C_k)); at least
// min_samples estimates per level difference (Example 4.1).  The RMSD of a
// level mean is the standard error sqrt(s^2/N) with the Bessel-corrected
// sample variance.  Batch rule: every round, each level above its target draws
// min(nb, ceil(V_l/rho_l^2) - N_l) more samples (at least one).
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "context.h"

namespace mlmc {

namespace {

struct Stats {
  double mre = 0, mim = 0, var = 0;
};

// two-pass mean and Bessel-corrected variance E|s - mean|^2, index order
Stats mean_var(const std::vector<c64>& s) {
  Stats st;
  const size_t N = s.size();
  if (N == 0) return st;
  double sr = 0, si = 0;
  for (const c64& v : s) {
    sr += v.re;
    si += v.im;
  }
  st.mre = sr / (double)N;
  st.mim = si / (double)N;
  if (N < 2) return st;
  double acc = 0;
  for (const c64& v : s) {
    double dr = v.re - st.mre, di = v.im - st.mim;
    acc += dr * dr + di * di;
  }
  st.var = acc / (double)(N - 1);
  return st;
}

std::vector<double> weights(const mlmc_options& opt, int L, const std::vector<double>& var,
                            const std::vector<double>& cost) {
  const int nl = L - 1;
  std::vector<double> w(nl, 1.0 / nl);
  if (opt.alloc == MLMC_ALLOC_WEIGHTS) {
    double t = 0;
    for (int l = 0; l < nl; ++l) t += opt.rho_weights[l];
    for (int l = 0; l < nl; ++l) w[l] = opt.rho_weights[l] / t;
  } else if (opt.alloc == MLMC_ALLOC_GILES) {
    std::vector<double> g(nl);
    double t = 0;
    for (int l = 0; l < nl; ++l) {
      g[l] = std::sqrt(std::max(var[l], 0.0) * cost[l]);
      t += g[l];
    }
    if (t > 0)
      for (int l = 0; l < nl; ++l) w[l] = g[l] / t;
  }
  return w;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

void run_estimator(int L, const SamplerIface& smp, c64 coarse, const std::vector<double>& cost,
                   const mlmc_options& opt, double tol, mlmc_result* out) {
  const double t0 = now_s();
  MLMC_REQUIRE(L >= 2 && L <= MLMC_MAX_LEVELS, MLMC_EINVAL, "levels out of range");
  MLMC_REQUIRE(tol > 0, MLMC_EINVAL, "tol must be positive");
  MLMC_REQUIRE(opt.alloc != MLMC_ALLOC_WEIGHTS || opt.rho_weights, MLMC_EINVAL,
               "MLMC_ALLOC_WEIGHTS needs rho_weights");
  const int nl = L - 1;
  const int64_t minN = opt.min_samples > 1 ? opt.min_samples : 2;
  const int64_t nb = opt.nb;
  std::memset(out, 0, sizeof(*out));

  double tau = opt.tau;
  if (!(tau > 0)) {
    MLMC_REQUIRE((bool)smp.pilot, MLMC_EINVAL, "no pilot sampler and no tau given");
    std::vector<c64> p(5);
    smp.pilot(5, p.data());
    Stats st = mean_var(p);
    tau = std::hypot(st.mre, st.mim) - std::sqrt(st.var / 5.0);
    if (tau <= 0) tau = std::hypot(st.mre, st.mim);
  }
  const double target2 = (tol * tau) * (tol * tau);

  std::vector<std::vector<c64>> samples(nl);
  for (int l = 0; l < nl; ++l) {
    samples[l].resize(minN);
    smp.sample(l + 1, 0, minN, samples[l].data());
  }
  std::vector<Stats> st(nl);
  for (;;) {
    std::vector<double> var(nl);
    for (int l = 0; l < nl; ++l) {
      st[l] = mean_var(samples[l]);
      var[l] = st[l].var;
    }
    std::vector<double> w = weights(opt, L, var, cost);
    std::vector<std::pair<int, int64_t>> todo;
    for (int l = 0; l < nl; ++l) {
      const int64_t N = (int64_t)samples[l].size();
      const double rho2 = w[l] * target2;
      if (var[l] / (double)N > rho2) {
        int64_t need = nb;
        if (rho2 > 0) {
          double r = std::ceil(var[l] / rho2) - (double)N;
          need = r > (double)nb ? nb : (int64_t)r;
        }
        int64_t add = need < nb ? need : nb;
        if (add > opt.max_samples - N) add = opt.max_samples - N;
        if (add < 1) add = 1;
        MLMC_REQUIRE(N < opt.max_samples, MLMC_ENOCONV,
                     "level " + std::to_string(l + 1) + " reached max_samples");
        todo.push_back({l, add});
      }
    }
    if (todo.empty()) break;
    for (auto& t : todo) {
      const int l = t.first;
      const int64_t N = (int64_t)samples[l].size();
      samples[l].resize(N + t.second);
      smp.sample(l + 1, N, t.second, samples[l].data() + N);
    }
  }
  double tre = coarse.re, tim = coarse.im, v = 0;
  out->levels = L;
  for (int l = 0; l < nl; ++l) {
    st[l] = mean_var(samples[l]);
    tre += st[l].mre;
    tim += st[l].mim;
    v += st[l].var / (double)samples[l].size();
    out->n_samples[l] = (int64_t)samples[l].size();
    out->level_mean[l][0] = st[l].mre;
    out->level_mean[l][1] = st[l].mim;
    out->level_var[l] = st[l].var;
    out->level_cost[l] = cost[l];
  }
  out->trace[0] = tre;
  out->trace[1] = tim;
  out->rmsd = std::sqrt(v);
  out->tau = tau;
  out->coarse_trace[0] = coarse.re;
  out->coarse_trace[1] = coarse.im;
  out->seconds = now_s() - t0;
}

void run_hutchinson(const std::function<void(int64_t, int64_t, c64*)>& sample,
                    const std::function<void(int64_t, c64*)>& pilot, const mlmc_options& opt,
                    double tol, mlmc_result* out) {
  const double t0 = now_s();
  MLMC_REQUIRE(tol > 0, MLMC_EINVAL, "tol must be positive");
  std::memset(out, 0, sizeof(*out));
  double tau = opt.tau;
  if (!(tau > 0)) {
    std::vector<c64> p(5);
    pilot(5, p.data());
    Stats st = mean_var(p);
    tau = std::hypot(st.mre, st.mim) - std::sqrt(st.var / 5.0);
    if (tau <= 0) tau = std::hypot(st.mre, st.mim);
  }
  const double target2 = (tol * tau) * (tol * tau);
  const int64_t nb = opt.nb;
  const int64_t minN = opt.min_samples > 1 ? opt.min_samples : 2;
  std::vector<c64> s(minN);
  sample(0, minN, s.data());
  Stats st;
  for (;;) {
    st = mean_var(s);
    const int64_t N = (int64_t)s.size();
    if (st.var / (double)N <= target2) break;
    int64_t need = nb;
    if (target2 > 0) {
      double r = std::ceil(st.var / target2) - (double)N;
      need = r > (double)nb ? nb : (int64_t)r;
    }
    int64_t add = need < nb ? need : nb;
    if (add > opt.max_samples - N) add = opt.max_samples - N;
    if (add < 1) add = 1;
    MLMC_REQUIRE(N < opt.max_samples, MLMC_ENOCONV, "reached max_samples");
    s.resize(N + add);
    sample(N, add, s.data() + N);
  }
  out->levels = 1;
  out->trace[0] = st.mre;
  out->trace[1] = st.mim;
  out->rmsd = std::sqrt(st.var / (double)s.size());
  out->tau = tau;
  out->n_samples[0] = (int64_t)s.size();
  out->level_mean[0][0] = st.mre;
  out->level_mean[0][1] = st.mim;
  out->level_var[0] = st.var;
  out->seconds = now_s() - t0;
}

}  // namespace mlmc
