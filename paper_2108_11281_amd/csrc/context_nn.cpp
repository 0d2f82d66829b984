// Learned smoother of the 2-spin lattice operator: weights, the network step
// inside the finest-level V-cycle, generation of training pairs from the
// method's own plain multigrid solves, and Adam training on the device.
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "context.h"

namespace mlmc {

namespace {
constexpr uint64_t kStreamTrain = 5;

uint64_t splitmix(uint64_t& st) {
  uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}
}  // namespace

void Context::nn_require() const {
  MLMC_REQUIRE(complex_ && !lv_.empty() && lv_[0].wilson, MLMC_EUNSUPPORTED,
               "the learned smoother is defined for WILSON2D only");
  MLMC_REQUIRE(lv_[0].side % 16 == 0, MLMC_EUNSUPPORTED,
               "the learned smoother needs a lattice side that is a multiple of 16");
}

void Context::nn_alloc() {
  nn_require();
  if (nn_w_) return;
  const int nw = nn_num_weights();
  nn_w_ = dalloc_n<float>(nw);
  nn_m_ = dalloc_n<float>(nw);
  nn_v_ = dalloc_n<float>(nw);
  nn_g_ = dalloc_n<float>(nw);
  nn_frag_ = dalloc((size_t)nn_frag_count() * 16);
  const int N = lv_[0].side;
  nn_links_ = dalloc((size_t)N * N * 4 * 2);
  nn_links(theta_dev_, nn_links_, N, s_);
}

void Context::nn_set_weights(const float* w) {
  nn_alloc();
  MLMC_HIP(hipMemcpyAsync(nn_w_, w, sizeof(float) * nn_num_weights(), hipMemcpyHostToDevice, s_));
  nn_pack(nn_w_, nn_frag_, s_);
  MLMC_HIP(hipStreamSynchronize(s_));
  nn_ready_ = true;
}

void Context::nn_get_weights(float* w) {
  MLMC_REQUIRE(nn_w_ != nullptr, MLMC_ESTATE, "no network weights set or trained");
  MLMC_HIP(hipMemcpyAsync(w, nn_w_, sizeof(float) * nn_num_weights(), hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
}

void Context::nn_step(const c32* b, c32* x, int nb, const int* act) {
  const Level& L = lv_[0];
  c32* res = wc32_.vt[0];
  cop_residual<c32, c32, c32>(1, b, x, res, nb, act, partials_);
  finish_sums(partials_, wilson_residual_blocks(L.side), nb, scal_[kNn], s_);
  // 2 x 4032 flops per site and column (three 3x3 convolutions, no bias)
  const double flops = 2.0 * nn_num_weights() * (double)L.side * L.side;
  timed<c32>(1, kTimNn, flops, act, nb, [&] {
    nn_apply(res, x, scal_[kNn], 1.0 / (double)L.n, nn_links_, nn_frag_, L.side, nb, act, s_);
  });
  nn_stats[0] += 1;
}

void Context::nn_apply_fp64(int nrhs, const double* r, double* e) {
  MLMC_REQUIRE(nn_ready_, MLMC_ESTATE, "no network weights set or trained");
  MLMC_REQUIRE(nrhs >= 1 && nrhs <= nb_, MLMC_EINVAL, "nrhs must be in [1, nb]");
  MLMC_REQUIRE(opt_.precision == MLMC_FP32_IR64, MLMC_EUNSUPPORTED,
               "the network runs in the FP32 (complex64) precision mode");
  const Level& L = lv_[0];
  const c64* r64 = reinterpret_cast<const c64*>(r);
  c32* r32 = wc32_.vt[0];
  c32* x32 = fg32_.d;
  vec_dot_partials<c64>(r64, r64, L.n, nrhs, nullptr, partials_, s_);
  finish_sums(partials_, reduce_blocks(L.n), nrhs, scal_[kNn], s_);
  vec_convert<c32, c64>(r64, r32, L.n, nrhs, nullptr, s_);
  vec_zero<c32>(x32, L.n, nrhs, nullptr, s_);
  nn_apply(r32, x32, scal_[kNn], 1.0 / (double)L.n, nn_links_, nn_frag_, L.side, nrhs, nullptr,
           s_);
  vec_convert<c64, c32>(x32, reinterpret_cast<c64*>(e), L.n, nrhs, nullptr, s_);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

void Context::nn_loss_grad(int ncrops, const float* in, const float* tgt, double* loss,
                           float* grad) {
  MLMC_REQUIRE(nn_ready_, MLMC_ESTATE, "no network weights set or trained");
  MLMC_REQUIRE(ncrops >= 1 && ncrops <= 65536, MLMC_EINVAL, "ncrops must be in [1, 65536]");
  const int nw = nn_num_weights();
  const int64_t nin = (int64_t)ncrops * nn_crop_in_elems();
  void* inb = dalloc((size_t)nin * 2);
  float* gpart = dalloc_n<float>((int64_t)ncrops * nw);
  double* lpart = dalloc_n<double>(ncrops);
  double* l = dalloc_n<double>(1);
  nn_round_inputs(in, inb, nin, s_);
  nn_train_step(inb, tgt, nullptr, ncrops, nn_frag_, nn_w_, gpart, lpart, nn_g_, l, s_);
  MLMC_HIP(hipMemcpyAsync(grad, nn_g_, sizeof(float) * nw, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipMemcpyAsync(loss, l, sizeof(double), hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
  dfree(l);
  dfree(lpart);
  dfree(gpart);
  dfree(inb);
}

void Context::nn_crops_fp64(int nrhs, const double* r, const double* e, int ncrops,
                            const int* origin, float* in_host, float* tgt_host) {
  nn_require();
  MLMC_REQUIRE(nrhs >= 1 && nrhs <= nb_, MLMC_EINVAL, "nrhs must be in [1, nb]");
  MLMC_REQUIRE(ncrops >= 1 && ncrops <= 65536, MLMC_EINVAL, "ncrops must be in [1, 65536]");
  const Level& L = lv_[0];
  const int N = L.side;
  for (int c = 0; c < ncrops; ++c) {
    MLMC_REQUIRE(origin[3 * c] >= 0 && origin[3 * c] < nrhs, MLMC_EINVAL,
                 "crop column out of range");
    MLMC_REQUIRE(origin[3 * c + 1] >= 0 && origin[3 * c + 1] < N && origin[3 * c + 2] >= 0 &&
                     origin[3 * c + 2] < N,
                 MLMC_EINVAL, "crop corner outside the lattice");
  }
  if (!nn_links_) {  // the link features exist once the network state does
    nn_alloc();
  }
  const c64* r64 = reinterpret_cast<const c64*>(r);
  const int64_t nin = (int64_t)ncrops * nn_crop_in_elems();
  const int64_t nout = (int64_t)ncrops * nn_crop_out_elems();
  void* inb = dalloc((size_t)nin * 2);
  float* tg = dalloc_n<float>(nout);
  int* org = dalloc_n<int>(3 * (int64_t)ncrops);
  // the RMS of each residual column, as the training-pair generator forms it
  vec_dot_partials<c64>(r64, r64, L.n, nrhs, nullptr, partials_, s_);
  finish_sums(partials_, reduce_blocks(L.n), nrhs, scal_[kNn], s_);
  MLMC_HIP(hipMemcpyAsync(org, origin, sizeof(int) * 3 * (size_t)ncrops, hipMemcpyHostToDevice,
                          s_));
  nn_crops(r64, reinterpret_cast<const c64*>(e), scal_[kNn], 1.0 / (double)L.n, nn_links_, org,
           ncrops, N, inb, tg, s_);
  std::vector<uint16_t> hb((size_t)nin);
  MLMC_HIP(hipMemcpyAsync(hb.data(), inb, (size_t)nin * 2, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipMemcpyAsync(tgt_host, tg, sizeof(float) * (size_t)nout, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
  for (int64_t i = 0; i < nin; ++i) {  // BF16 is the upper half of an FP32
    const uint32_t u = (uint32_t)hb[(size_t)i] << 16;
    std::memcpy(in_host + i, &u, 4);
  }
  dfree(org);
  dfree(tg);
  dfree(inb);
}

void Context::nn_adam_step(const float* grad, double lr, int t) {
  MLMC_REQUIRE(nn_w_ != nullptr, MLMC_ESTATE, "no network weights set or trained");
  MLMC_REQUIRE(t >= 1, MLMC_EINVAL, "the Adam step count starts at 1");
  MLMC_REQUIRE(lr > 0 && std::isfinite(lr), MLMC_EINVAL, "learning rate must be > 0");
  const int nw = nn_num_weights();
  if (t == 1) {  // first step: zero moments
    vec_zero<float>(nn_m_, nw, 1, nullptr, s_);
    vec_zero<float>(nn_v_, nw, 1, nullptr, s_);
  }
  MLMC_HIP(hipMemcpyAsync(nn_g_, grad, sizeof(float) * nw, hipMemcpyHostToDevice, s_));
  nn_adam(nn_w_, nn_m_, nn_v_, nn_g_, lr, 0.9, 0.999, 1e-8, t, s_);
  nn_pack(nn_w_, nn_frag_, s_);
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
void Context::nn_train(const float* w_init, const mlmc_train_options& o,
                       mlmc_train_report* rep) {
  nn_require();
  MLMC_REQUIRE(o.n_batches >= 1 && o.crops_per_column >= 1 && o.steps >= 1 && o.batch >= 1,
               MLMC_EINVAL, "training options must be >= 1");
  MLMC_REQUIRE(o.lr > 0 && std::isfinite(o.lr), MLMC_EINVAL, "learning rate must be > 0");
  const int64_t ncrops = (int64_t)o.n_batches * nb_ * 2 * o.crops_per_column;
  MLMC_REQUIRE(ncrops <= (1 << 22), MLMC_EINVAL, "too many training crops (> 2^22)");
  MLMC_REQUIRE(o.batch <= ncrops && o.batch <= 65536, MLMC_EINVAL,
               "batch exceeds the number of crops (or 65536)");
  nn_alloc();
  const int nw = nn_num_weights();
  const Level& L = lv_[0];
  const int N = L.side;
  const int64_t n = L.n;
  const double t0 = now_s();
  MLMC_HIP(hipMemcpyAsync(nn_w_, w_init, sizeof(float) * nw, hipMemcpyHostToDevice, s_));
  vec_zero<float>(nn_m_, nw, 1, nullptr, s_);
  vec_zero<float>(nn_v_, nw, 1, nullptr, s_);

  // pair generation with the plain solver
  nn_ready_ = false;
  void* in = dalloc((size_t)ncrops * nn_crop_in_elems() * 2);
  float* tgt = dalloc_n<float>(ncrops * nn_crop_out_elems());
  c64* b = reinterpret_cast<c64*>(b1_);
  c64* y = reinterpret_cast<c64*>(y1_);
  c64* xs = dalloc_n<c64>(n * nb_);
  c64* rs = dalloc_n<c64>(n * nb_);
  c64* es = dalloc_n<c64>(n * nb_);
  const int per_state = nb_ * o.crops_per_column;
  int* origin = dalloc_n<int>(3 * (int64_t)per_state);
  std::vector<int> org(3 * (size_t)per_state);
  uint64_t rng = o.seed ^ 0x243F6A8885A308D3ULL;
  int64_t done = 0;
  const int rblk = wilson_residual_blocks(N);
  for (int j = 0; j < o.n_batches; ++j) {
    write_probes(1, o.seed, kStreamTrain, (uint64_t)j * nb_, nb_, b1_);
    bool ok = true;
    {
      // the targets need only the accuracy of BF16 training data
      const double saved = opt_.solve_tol;
      opt_.solve_tol = o.pair_tol > 0 ? o.pair_tol : 1e-6;
      try {
        solve(1, b1_, y1_, nb_, scal_[kErr1], nullptr, &ok);
      } catch (...) {
        opt_.solve_tol = saved;
        throw;
      }
      opt_.solve_tol = saved;
    }
    MLMC_REQUIRE(ok, MLMC_ENOCONV, "a training solve missed solve_tol");
    // state 1: one red-black sweep from zero
    cop_smooth<c64>(1, b, xs, nb_, nullptr, true, false);
    for (int state = 0; state < 2; ++state) {
      if (state == 1) {
        // state 2: plus the coarse-grid correction of the V-cycle
        cop_restrict<c64>(1, rs, wc64_.vb[1], nb_, nullptr);
        cvcycle<c64>(2, wc64_.vb[1], wc64_.vx[1], nb_, nullptr);
        cop_prolong<c64>(1, wc64_.vx[1], xs, nb_, nullptr, omega_, 1.0);
      }
      cop_residual<c64, c64, c64>(1, b, xs, rs, nb_, nullptr, partials_);
      finish_sums(partials_, rblk, nb_, scal_[kNn], s_);
      vec_sub<c64>(y, xs, es, n, nb_, s_);
      for (int c = 0; c < per_state; ++c) {
        org[3 * c] = c % nb_;
        org[3 * c + 1] = (int)(splitmix(rng) % (uint64_t)N);
        org[3 * c + 2] = (int)(splitmix(rng) % (uint64_t)N);
      }
      MLMC_HIP(hipMemcpyAsync(origin, org.data(), sizeof(int) * org.size(),
                              hipMemcpyHostToDevice, s_));
      nn_crops(rs, es, scal_[kNn], 1.0 / (double)n, nn_links_, origin, per_state, N,
               static_cast<char*>(in) + (size_t)done * nn_crop_in_elems() * 2,
               tgt + done * nn_crop_out_elems(), s_);
      // the host array is rewritten for the next state only after the copy
      MLMC_HIP(hipStreamSynchronize(s_));
      done += per_state;
    }
  }
  const double t1 = now_s();

  // Adam on the FP32 master weights; crops in a shuffled order, one pass of the
  // order after another
  std::vector<int> order((size_t)ncrops);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t i = ncrops - 1; i > 0; --i) {
    const int64_t k = (int64_t)(splitmix(rng) % (uint64_t)(i + 1));
    std::swap(order[(size_t)i], order[(size_t)k]);
  }
  int* order_dev = dalloc_n<int>(ncrops + o.batch);
  // the tail repeats the head so that a step's window never wraps
  std::vector<int> ext(order);
  ext.insert(ext.end(), order.begin(), order.begin() + o.batch);
  MLMC_HIP(hipMemcpyAsync(order_dev, ext.data(), sizeof(int) * ext.size(), hipMemcpyHostToDevice,
                          s_));
  float* gpart = dalloc_n<float>((int64_t)o.batch * nw);
  double* lpart = dalloc_n<double>(o.batch);
  double* losses = dalloc_n<double>(o.steps);
  int64_t pos = 0;
  for (int t = 1; t <= o.steps; ++t) {
    nn_pack(nn_w_, nn_frag_, s_);
    nn_train_step(in, tgt, order_dev + pos, o.batch, nn_frag_, nn_w_, gpart, lpart, nn_g_,
                  losses + (t - 1), s_);
    nn_adam(nn_w_, nn_m_, nn_v_, nn_g_, o.lr, 0.9, 0.999, 1e-8, t, s_);
    pos += o.batch;
    if (pos >= ncrops) pos -= ncrops;
  }
  nn_pack(nn_w_, nn_frag_, s_);
  std::vector<double> hl((size_t)o.steps);
  MLMC_HIP(hipMemcpyAsync(hl.data(), losses, sizeof(double) * o.steps, hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  MLMC_HIP(hipGetLastError());
  const double t2 = now_s();
  nn_ready_ = true;
  for (void* p : {(void*)losses, (void*)lpart, (void*)gpart, (void*)order_dev, (void*)origin,
                  (void*)es, (void*)rs, (void*)xs, (void*)tgt, in})
    dfree(p);
  if (rep) {
    rep->loss_first = hl[0];
    const int k = std::min(10, o.steps);
    double s = 0.0;
    for (int i = o.steps - k; i < o.steps; ++i) s += hl[(size_t)i];
    rep->loss_last = s / k;
    rep->solves = (int64_t)o.n_batches * nb_;
    rep->crops = ncrops;
    rep->gen_seconds = t1 - t0;
    rep->train_seconds = t2 - t1;
  }
}

}  // namespace mlmc
