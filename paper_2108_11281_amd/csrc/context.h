// Library context: the hierarchy, work buffers and the solvers.
#pragma once

#include <array>
#include <functional>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"

namespace mlmc {

// counter-RNG streams of the probes: level samples, pilot, plain Hutchinson
constexpr uint64_t kStreamProbe = 0, kStreamPilot = 1, kStreamHutch = 3;

// Device memory hooks (set through mlmc_set_allocator).
struct AllocHooks {
  mlmc_alloc_fn alloc = nullptr;
  mlmc_free_fn free_fn = nullptr;
  void* user = nullptr;
};
AllocHooks& alloc_hooks();

// One level of the hierarchy (1-based index `index`).
struct Level {
  int index = 1;
  int side = 0;       // grid / lattice side
  int dof = 1;        // unknowns per site (1 for scalar grids)
  int64_t n = 0;      // unknowns
  double d = 0, c = 0;  // POISSON2D stencil: A = d I - c (neighbours)
  // complex lattice levels: level 1 is the Wilson operator (links U), the
  // others 5-point block stencils B with inverted diagonal blocks Dinv
  bool wilson = false;
  c64* U64 = nullptr;
  c32* U32 = nullptr;
  c64 *B64 = nullptr, *Dinv64 = nullptr;
  c32 *B32 = nullptr, *Dinv32 = nullptr;
  // aggregation to the next level: row i (fine unknown) holds the coarse
  // coefficients q[i][0..dof_next-1]; aggregates are blk x blk sites
  c64* q64 = nullptr;
  c32* q32 = nullptr;
  int blk = 0;
  // VARCOEF3D levels: face coefficients k[3][side][side][side+1] and the
  // diagonal (shift + six faces), FP64 and FP32 copies
  double *kf64 = nullptr, *dg64 = nullptr, *kl64 = nullptr;
  float *dg32 = nullptr, *kl32 = nullptr;
  int cols = 4;  // right-hand sides per thread of the stencil kernels (autotuned)
  int cols_narrow = 4;  // CSR kernels: the same for launches of at most 16 columns
  // CSR sweep: largest class (in slices) of the trailing classes that share
  // launches, full and narrow batches (autotuned; 0: a launch per class)
  int tail_slices = 0, tail_slices_narrow = 0;
  int bsr_form[2] = {0, 0};  // block-stencil kernel form, complex64 / complex128 (autotuned)
  int mcols = 0;  // right-hand sides per wave of the fused 3D sweep (0: in-place sweeps)
  // POISSON2D: rows per segment of the fused sweep, FP32 and FP64 (autotuned)
  int gs_rows[2] = {16, 8};
  // CSR levels: the matrix by rows, the colour-sorted off-diagonal part for the
  // sweep and the aggregation to the next level, with FP32 and FP64 values
  // (device); host copies of the matrix, aggregate map and colours for export
  CsrMat<float> A32;
  CsrMat<double> A64;
  CsrSweep<float> S32;
  CsrSweep<double> S64;
  CsrAgg<float> G32;
  CsrAgg<double> G64;
  std::vector<int64_t> h_rp;
  std::vector<int> h_ci, h_agg, h_colour;
  std::vector<double> h_v;
  // CSR levels with given prolongations: P (n x pcols) and R = P^T, device
  // copies in both precisions, and P's host copy
  CsrMat<float> P32, R32;
  CsrMat<double> P64, R64;
  int pcols = 0;
  std::vector<int64_t> hp_rp;
  std::vector<int> hp_ci;
  std::vector<double> hp_v;
};

// Batched flexible GMRES workspace (precision T)
template <typename T>
struct Fgmres {
  T* V = nullptr;   // (m+1) basis vectors of n1*nb
  T* Z = nullptr;   // m preconditioned vectors
  T* r = nullptr;   // right-hand side of the cycle
  T* d = nullptr;   // correction
  T* tmp = nullptr;
};

// Per-precision work buffers (T = float or double for real operators).
template <typename T>
struct Work {
  T *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;
  // V-cycle right-hand side / solution / sweep scratch per level (0-based)
  std::vector<T*> vb, vx, vt;
  // residual and correction of the second coarse-grid cycle below a solve's
  // top level (levels 2 .. L_s - 1, 0-based index; top_cycles = 2 of the 3D
  // and CSR kinds only: the 2D Poisson V-cycle starts that cycle from ec)
  std::vector<T*> vr2, ve2;
  // transposed inverse of the solver's coarsest operator: real operators in
  // the MFMA tile kernel's layout (dense_pack4), complex ones plain row-major
  T* ainvT = nullptr;
  int ld = 0;               // its leading dimension (n rounded up to 16, zero padded)
  // complex operators: its real representation (2n x 2n, transposed) for the
  // real MFMA product on interleaved vectors, in the tile kernel's layout
  typename Traits<T>::real* ainvR = nullptr;
};

struct Estimate;

class GroupSolver;

class Context {
  friend class GroupSolver;  // lockstep solves over several contexts

 public:
  Context(const mlmc_operator& A, const mlmc_hierarchy& h, const mlmc_options& o,
          hipStream_t s);
  ~Context();

  // --- entry points used by the C ABI ---
  void trace(double tol, uint64_t seed, mlmc_result* out);
  void hutchinson(double tol, uint64_t seed, mlmc_result* out);
  void sample_level(int level, uint64_t seed, int64_t first, int64_t count, double* out,
                    double* out_err);
  void solve_fp64(int level, int nrhs, const double* b, double* y, double* relres,
                  bool throw_on_noconv);
  void apply_fp64(int level, int nrhs, const double* x, double* y);
  // ws: nullptr (working copies allocated for the call) or a device workspace
  // of ws_bytes that holds them
  // csr_tail (CSR levels): -1 the level's tuned sweep schedule, 0 a launch per
  // colour class, > 0 the trailing classes of at most that many slices share
  // launches
  void smooth_fp64(int level, int nrhs, int sweeps, bool reverse, bool zero_start,
                   const double* b, double* x, double* rc, void* ws = nullptr,
                   size_t ws_bytes = 0, int csr_tail = -1);
  void restrict_fp64(int level, int nrhs, const double* x, double* xc);
  void prolong_fp64(int level, int nrhs, const double* xc, double* x);
  void probes_fp64(int level, uint64_t seed, int stream, int64_t first, int nrhs,
                   double* out);
  void export_coarse(int which, double* out);
  void export_prolongation(int level, double* out);
  void export_csr(int level, int64_t* nnz, int64_t* row_ptr, int32_t* col_idx, double* vals,
                  int32_t* agg, int32_t* colour);
  void export_level(int level, int which, int64_t* rows, int64_t* cols, int64_t* nnz,
                    int64_t* row_ptr, int32_t* col_idx, double* vals);
  // learned smoother (WILSON2D)
  void nn_train(const float* w_init, const mlmc_train_options& o, mlmc_train_report* rep);
  void nn_set_weights(const float* w);
  void nn_get_weights(float* w);
  void nn_apply_fp64(int nrhs, const double* r, double* e);
  void nn_loss_grad(int ncrops, const float* in, const float* tgt, double* loss, float* grad);
  void nn_crops_fp64(int nrhs, const double* r, const double* e, int ncrops, const int* origin,
                     float* in_host, float* tgt_host);
  void nn_adam_step(const float* grad, double lr, int t);
  int64_t nn_stats[2] = {0, 0};  // network applications, fallbacks
  // deflated Hutchinson (real symmetric kinds)
  void deflation_setup(const mlmc_deflation_options& o, mlmc_deflation_report* rep);
  void deflated_sample(uint64_t seed, int64_t first, int64_t count, double* out,
                       double* out_err);
  void deflated_hutchinson(double tol, uint64_t seed, mlmc_result* out);
  void deflation_export(double* eigenvalues, double* vectors_dev, double* direct);

  int levels_mlmc() const { return L_; }
  int levels_solver() const { return Ls_; }
  int64_t level_size(int level) const { return lv_.at(level - 1).n; }
  double coarse_trace_re() const { return coarse_trace_.re; }
  double coarse_trace_im() const { return coarse_trace_.im; }
  int64_t counters[4] = {0, 0, 0, 0};
  std::string last_error;
  const mlmc_options& options() const { return opt_; }
  int device() const { return device_; }

  // kernel timing (measurement mode)
  // kTimNn counts flops (not bytes) per column: the network is MFMA-bound
  enum { kTimGs, kTimResRestrict, kTimProlong, kTimApply, kTimCgXr, kTimNn, kTimIrFold,
         kTimIrResidual, kNumTimers };
  void set_timing(unsigned mask, int stride);
  // level 0: all levels; 1..L_s: launches on that level only
  void kernel_stats(int id, int fp64, double* out, int level = 0);
  void reset_kernel_stats();

  // level-difference samples and pilot/Hutchinson samples in batches <= nb
  void samples_batch(int level, uint64_t seed, uint64_t first, int nbatch, c64* out,
                     double* err);
  void hutch_batch(uint64_t seed, uint64_t stream, uint64_t first, int nbatch, c64* out);

 private:
  void* dalloc(size_t bytes);
  void dfree(void* p);  // synchronises the stream, then releases p
  template <typename T> T* dalloc_n(int64_t count) {
    return static_cast<T*>(dalloc(sizeof(T) * (size_t)count));
  }
  void build_poisson();
  void build_varcoef(const double* k);
  void build_csr(const mlmc_operator& A, const int32_t* const* aggs, const mlmc_csr* P);
  void csr_general_coarse_trace();
  void samples_batch_general(int level, uint64_t seed, uint64_t first, int nbatch, c64* out,
                             double* err);
  // per-column convergence of the two solves of a sample batch (ok2 may be null:
  // no second solve); writes every sample (NaN where a solve missed solve_tol) and
  // then throws MLMC_ENOCONV naming the level and the first failed sample
  void finish_samples(int level, int nbatch, const char* ok1, const char* ok2, uint64_t first,
                      c64* out, double* err);
  std::vector<char> col_ok_;  // per column of the last solve(): met solve_tol
  void csr_upload(Level& L, bool last);
  void tune_csr();
  template <typename T> const CsrMat<T>& csr_mat(int l) const;
  template <typename T> const CsrSweep<T>& csr_sweep(int l) const;
  template <typename T> const CsrAgg<T>& csr_agg(int l) const;
  template <typename T> const CsrMat<T>& csr_P(int l) const;  // given prolongation
  template <typename T> const CsrMat<T>& csr_R(int l) const;  // its transpose
  template <typename T> void vcycle_csr(int l, const T* b, T* x, int nb, const int* act,
                                        c64* rz_partials, bool top = false);
  void tune_varcoef();
  void tune_bsr();
  void tune_poisson();
  // block-stencil kernel form for a call over nb columns: the tuned form, but
  // the thread-per-site form for narrow batches (a wave-uniform wave serves 64
  // columns, so fewer than 32 would leave most of its lanes idle)
  template <typename T> int bsr_form(const Level& L, int nb) const {
    return nb >= 32 ? L.bsr_form[sizeof(T) == sizeof(c64) ? 1 : 0] : 0;
  }
  // right-hand sides per thread of the CSR kernels on level L for nb columns
  // (narrow batches, such as the pilot and the first samples of a level, have
  // their own tuned value)
  int csr_cols(const Level& L, int nb) const { return nb <= 16 ? L.cols_narrow : L.cols; }
  int csr_tail(const Level& L, int nb) const {
    return nb <= 16 ? L.tail_slices_narrow : L.tail_slices;
  }
  // red-black sweeps fused into one pass of the Poisson smoother on level l
  int sweeps_per_pass(int l) const { return lv_[l - 1].side >= 64 ? 2 : 1; }
  template <typename T> int gs_rows(int l) const {
    return lv_[l - 1].gs_rows[sizeof(typename Traits<T>::real) == 8 ? 1 : 0];
  }
  void finish_real_build();
  void build_wilson(const double* theta);
  void nn_alloc();
  void defl_require() const;
  void defl_gram(const double* A, int ma, const double* B, int mb, double* C);
  std::vector<double> defl_gram_host(const double* A, int ma, const double* B, int mb);
  bool defl_solve_block(const double* X, double* Y, int m);
  void defl_apply_block(const double* X, double* Y, int m);
  void deflated_batch(uint64_t seed, uint64_t first, int nbatch, c64* out, double* err_out);
  void nn_require() const;
  // r = b - A_1 x ; x += s * net(r / s)  (finest level, FP32 / complex64)
  void nn_step(const c32* b, c32* x, int nb, const int* act);
  void alloc_common();
  // complex operators: op on level l in precision T (c32 / c64)
  template <typename T> const T* links(int l) const;
  template <typename T> const T* blocks(int l) const;
  template <typename T> const T* dinv(int l) const;
  template <typename T> const T* qmat(int l) const;
  template <typename Tb, typename T, typename Tr>
  void cop_residual(int l, const Tb* b, const T* x, Tr* r, int nb, const int* act, c64* partials);
  template <typename T> void cop_smooth(int l, const T* b, T* x, int nb, const int* act,
                                        bool zero_init, bool reverse);
  template <typename T> void cop_smooth_n(int l, const T* b, T* x, int nb, const int* act,
                                          int count, bool zero_init, bool reverse);
  template <typename T> void cop_restrict(int l, const T* x, T* xc, int nb, const int* act);
  template <typename T> void cop_prolong(int l, const T* ec, T* x, int nb, const int* act,
                                         double omega, double beta);
  template <typename T> void cvcycle(int l, const T* b, T* x, int nb, const int* act,
                                     bool top = false);
  // the complex counterpart of second_coarse_cycle
  template <typename T> void csecond_coarse_cycle(int l, const T* bc, T* ec, int nb,
                                                  const int* act, bool top);
  template <typename T> void coarse_apply(const T* b, T* x, int nb, const int* act);
  template <typename T> void fgmres_cycle(int l, const T* r, T* d, int nb, int* act,
                                          double tol);
  void solve_complex(int l, const c64* b, c64* y, int nb, c64* err);
  template <typename T> Fgmres<T>& fg();
  void invert_coarse(int level, double** inv_out, c64* trace_out);
  template <typename T> void dense_invert_checked(T* aug, int n, T* out);
  template <typename T> void alloc_work(Work<T>& w, int width = 0);
  // batches solved in plain FP64 although the mode is MLMC_FP32_IR64
  bool fp64_batch(int nb) const {
    return opt_.precision == MLMC_FP32_IR64 && !complex_ && nb <= opt_.narrow_fp64;
  }

  // operator pieces on level l (1-based) in precision T
  template <typename T> void op_apply(int l, const T* x, T* y, int nb, const int* act,
                                      c64* partials);
  template <typename T> void op_res_restrict(int l, const T* b, const T* x, T* rc, int nb,
                                             const int* act);
  template <typename T> void op_prolong(int l, const T* ec, T* x, int nb, const int* act,
                                        double beta);
  template <typename T> void op_restrict(int l, const T* x, T* xc, int nb, const int* act);
  template <typename Tb, typename Tx, typename Tr>
  void op_residual(int l, const Tb* b, const Tx* x, Tr* r, int nb, const int* act,
                   c64* partials);

  template <typename T> const T* vc_faces(int l) const;
  template <typename T> const T* vc_diag(int l) const;
  // partial sums per column written by op_residual / op_update_apply
  int op_tiles(int l) const;
  template <typename T> void op_update_apply(int l, const T* p_old, const T* z, const c64* beta,
                                             T* p_new, T* q, int nb, const int* act);
  template <typename T> void vcycle_vc(int l, const T* b, T* x, int nb, const int* act,
                                       c64* rz_partials, bool top = false);
  template <typename T> Work<T>& work();
  // top: l is the solve's top level (top_cycles_ coarse-grid cycles there).
  // x0 (POISSON2D, not the coarsest level; nullable): the pre-smoothing starts
  // from x0 instead of 0 (x0 may be x), which gives x0 + V(b - A x0)
  template <typename T> void vcycle(int l, const T* b, T* x, int nb, const int* act,
                                    c64* rz_partials, bool top = false,
                                    const T* x0 = nullptr);
  // with top and top_cycles_ == 2 (and level l + 1 not the coarsest): a second
  // coarse-grid cycle on level l + 1 on the residual of the first, ec += V(bc - A ec)
  template <typename T> void second_coarse_cycle(int l, const T* bc, T* ec, int nb,
                                                 const int* act, bool top);
  int top_cycles_ = 1;
  template <typename T> int vcycle_partials(int l, bool* fused) const;
  // CG on level l in precision T: x = A^-1 b to relative residual tol;
  // act: per-column flags (in: columns to solve; out: still unconverged)
  template <typename T> int pcg(int l, const T* b, T* x, int nb, int* act, double tol,
                                c64* lastcorr);
  void pcg_refined(int l, const double* b, double* y, int nb, double tol, c64* err);
  // Launches the HIP graph of `body`, captured on the context stream at the
  // key's first use; the host-side counters the body advances (recorded while
  // capturing) advance by the same amounts at every launch.  Keys: {0, level,
  // batch width, 0} the refined CG's iteration pairs; {1 (complex64) or 2
  // (complex128), level, batch width, iteration + 64 (learned smoother on)}
  // the FGMRES iterations.
  void replay(const std::array<int, 4>& key, const std::function<void()>& body);
  struct Graph {
    hipGraphExec_t ex = nullptr;
    int64_t counters[4] = {0, 0, 0, 0};
    int64_t nn_stats[2] = {0, 0};
  };
  std::map<std::array<int, 4>, Graph> graphs_;
  hipStream_t cap_s_ = nullptr;  // library-owned stream that graphs are captured on
  // ends of the last two FGMRES iterations: the host reads an iteration's
  // convergence count while the next one runs
  hipEvent_t fg_ev_[2] = {nullptr, nullptr};
  // FP64 solve of level l for nb columns; b, y FP64; err: per-column stated error
  // contributions (device c64 nb), relres host (nullable)
  void solve(int l, const double* b, double* y, int nb, c64* err, double* relres_host,
             bool* converged);
  int read_count();
  void write_probes(int level, uint64_t seed, uint64_t stream, uint64_t first, int nb,
                    double* out);
  void restrict64(int level, const double* x, double* xc, int nb);
  void probe_quad(int level, uint64_t seed, uint64_t stream, uint64_t first, int nb,
                  const double* y, c64* out);
  hipEvent_t event();
  void collect_timing();
  // launch() on level `level` (1-based), timed as kernel `id` in measurement mode
  template <typename T, typename F>
  void timed(int level, int id, double bytes_per_col, const int* act, int nb, F&& launch);
  struct TimerStat {
    int64_t launches = 0;
    double ms = 0, bytes = 0;
  };
  struct Pending {
    int slot, idx, nb, level;
    double bytes_per_col;
    hipEvent_t a, b;
  };

  static constexpr int kTimingLog = 1 << 16;
  bool timing_ = false;
  unsigned timing_mask_ = 0;
  int timing_stride_ = 1;
  int64_t timing_seen_[kNumTimers] = {};
  int* tlog_dev_ = nullptr;
  int tlog_next_ = 0;
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> ev_pool_;
  TimerStat tstat_[2 * kNumTimers];
  TimerStat tstat_lv_[2 * kNumTimers][MLMC_MAX_LEVELS];

  int kind_;
  int device_ = 0;
  mlmc_operator op_;
  mlmc_hierarchy h_;
  mlmc_options opt_;
  hipStream_t s_;
  int Ls_ = 0, L_ = 0, nb_ = 0;
  std::vector<Level> lv_;
  std::vector<void*> allocs_;
  AllocHooks hooks_;

  Work<float> w32_;
  Work<double> w64_;
  Work<c32> wc32_;
  Work<c64> wc64_;
  Fgmres<c32> fg32_;
  Fgmres<c64> fg64_;
  bool complex_ = false;
  bool varcoef_ = false;
  bool csr_ = false;
  // CSR with given prolongations: the general decomposition of Sec. 4.1
  // (finest-level probes restricted level by level through gA_/gB_)
  bool general_ = false;
  double *gA_ = nullptr, *gB_ = nullptr;
  // learned smoother state: FP32 master weights, Adam moments, gradient, BF16
  // fragments, BF16 link features; nn_use_ is true while a solve runs with it
  bool nn_ready_ = false, nn_use_ = false;
  float *nn_w_ = nullptr, *nn_m_ = nullptr, *nn_v_ = nullptr, *nn_g_ = nullptr;
  void *nn_frag_ = nullptr, *nn_links_ = nullptr;
  double* theta_dev_ = nullptr;
  double* nn_loss_ = nullptr;
  int m_ = 16;                    // FGMRES restart length
  double omega_ = 1.0;            // coarse-correction scaling in use
  // FGMRES scalars: Hessenberg, rotations, rhs, solution, dims, cycle flags
  c64 *gH_ = nullptr, *gcs_ = nullptr, *gsn_ = nullptr, *gg_ = nullptr, *gy_ = nullptr;
  c64* ghcol_ = nullptr;
  int *gdims_ = nullptr, *gstart_ = nullptr;
  double* ainv_mlmc_ = nullptr;   // inverse of A_L (row-major), if L < L_s
  double* ainv_solver_ = nullptr; // inverse of A_{L_s} (row-major)
  c64 coarse_trace_ = {0, 0};

  // FP64 buffers of a sample batch
  double *b1_ = nullptr, *y1_ = nullptr, *b2_ = nullptr, *y2_ = nullptr, *r64_ = nullptr;
  float* r32_ = nullptr;
  float* d32_ = nullptr;
  // POISSON2D with MLMC_FP32_IR64: the refined solve's right-hand side in FP32
  // when every entry is an FP32 number (probes and their 2x2 restrictions)
  float* b32_ = nullptr;
  c64* partials_ = nullptr;
  int64_t partials_cap_ = 0;
  // per-column scalar arrays (nb_ entries each); kErr1..kQb are consecutive
  enum { kRr0, kRz, kTmp, kAlpha, kBeta, kBb, kBd, kRres, kRres2, kErr1, kErr2, kQa, kQb,
         kNn, kNumScalars };
  c64* scal_[kNumScalars] = {};
  int *act_outer_ = nullptr, *act_inner_ = nullptr, *count_dev_ = nullptr;  // count_dev_: 8 ints
  // pinned host counts (8 ints) and their device address: the single-thread
  // count kernels whose results the host tests store there directly, so a
  // check needs no copy, only the stream synchronisation
  int* count_host_ = nullptr;
  int* count_map_ = nullptr;
  c64* host_c64_ = nullptr;  // pinned, 8*nb
  // deflation: Ritz block V (the first defl_k_ vectors are U), work blocks W
  // and Z, small device matrices, Gram partial sums; eigenvalues and the direct
  // term tr(U^T A^{-1} U)
  double *defl_V_ = nullptr, *defl_W_ = nullptr, *defl_Z_ = nullptr, *defl_small_ = nullptr;
  double* defl_part_ = nullptr;
  int64_t defl_part_cap_ = 0;
  int defl_k_ = 0;
  std::vector<double> defl_lambda_;
  double defl_direct_ = 0.0;
};

// level-difference samples of several VARCOEF3D problems solved in lockstep
// (mode 1: persistent V-cycle stage kernel, 2: one launch per stage depth);
// status: per problem MLMC_OK or its first failure
void group_batch_sample(const std::vector<Context*>& cs, int level, const uint64_t* seeds,
                        int64_t first, int64_t count, int mode, double* out, int* status);

// mlmc_smooth flags: known bits, at most one CSR sweep schedule; the schedule
// as Context::smooth_fp64's csr_tail
inline bool smooth_flags_valid(int flags) {
  const int sched = MLMC_SMOOTH_CLASS_LAUNCHES | MLMC_SMOOTH_SHARED_TAIL;
  return (flags & ~(MLMC_SMOOTH_REVERSE | MLMC_SMOOTH_ZERO_START | sched)) == 0 &&
         (flags & sched) != sched;
}
inline int smooth_csr_tail(int flags) {
  if (flags & MLMC_SMOOTH_CLASS_LAUNCHES) return 0;
  return (flags & MLMC_SMOOTH_SHARED_TAIL) ? kTailWaves : -1;
}

// splitmix64 finaliser (sampling of timed launches)
inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

template <typename T, typename F>
inline void Context::timed(int level, int id, double bytes_per_col, const int* act, int nb,
                           F&& launch) {
  (void)act;
  // with stride k, a launch is timed with probability 1/k, chosen by a hash of
  // its index so that the sample does not alias with the period of the V-cycle
  if (!timing_ || !(timing_mask_ & (1u << id)) ||
      (timing_stride_ > 1 && mix64((uint64_t)timing_seen_[id]++ * kNumTimers + id) %
                                     (uint64_t)timing_stride_ != 0)) {
    launch();
    return;
  }
  if (tlog_next_ >= kTimingLog) collect_timing();
  const int slot = 2 * id + (sizeof(typename Traits<T>::real) == 8 ? 1 : 0);
  const int idx = tlog_next_++;
  hipEvent_t a = event(), b = event();
  LaunchEvents ev;
  ev.start = a;
  ev.stop = b;
  timing_log() = tlog_dev_ + (int64_t)idx * nb_;
  timing_events() = &ev;
  launch();
  timing_events() = nullptr;
  timing_log() = nullptr;
  MLMC_HIP(hipGetLastError());
  if (!ev.used) {  // nothing was launched through MLMC_LAUNCH: no sample
    ev_pool_.push_back(a);
    ev_pool_.push_back(b);
    return;
  }
  pending_.push_back({slot, idx, nb, level, bytes_per_col, a, b});
}

// ---------------------------------------------------------------------------
// Estimator driver (host only).  The sampler fills `count` samples of a level.
// ---------------------------------------------------------------------------
struct SamplerIface {
  std::function<void(int level, int64_t first, int64_t count, c64* out)> sample;
  std::function<void(int64_t count, c64* out)> pilot;
};

// Fixed device workspace of the allocation-free entry points: looked up for
// device `dev` (current) once, at the first mlmc_setup on it.
void noalloc_init(int dev);

void run_estimator(int L, const SamplerIface& smp, c64 coarse, const std::vector<double>& cost,
                   const mlmc_options& opt, double tol, mlmc_result* out);
void run_hutchinson(const std::function<void(int64_t, int64_t, c64*)>& sample,
                    const std::function<void(int64_t, c64*)>& pilot, const mlmc_options& opt,
                    double tol, mlmc_result* out);

}  // namespace mlmc
