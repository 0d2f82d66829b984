// Launchers of the HIP kernels.  All vectors are RHS-major blocks: column k of
// length n starts at k*n.  `active` (nullable) is a per-column flag array on
// the device: kernels skip columns whose flag is 0 (converged solves).
#pragma once

#include <hip/hip_ext.h>

#include <type_traits>
#include <vector>

#include "common.h"

namespace mlmc {

constexpr int kThreads = 256;
constexpr int kMaxPartials = 1024;  // per-column partial sums of a reduction

// Measurement mode: when non-null, the next timed launch records, for each
// column k, its active flag at tlog[k] (written by the kernel itself).
int*& timing_log();

// Measurement mode: when non-null, launches made through MLMC_LAUNCH carry
// these events in the dispatch itself (hipExtLaunchKernel), so the events
// time the kernel's execution and not the gaps between launches.  The first
// such launch records `start`; every one records `stop` (the last one wins).
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;
};
LaunchEvents*& timing_events();

#define MLMC_LAUNCH(kern, grid, block, shmem, stream, ...)                                   \
  do {                                                                                       \
    ::mlmc::LaunchEvents* ev_ = ::mlmc::timing_events();                                     \
    if (ev_) {                                                                               \
      hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, ev_->used ? nullptr : ev_->start, \
                            ev_->stop, 0, __VA_ARGS__);                                      \
      ev_->used = true;                                                                      \
    } else {                                                                                 \
      hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                     \
    }                                                                                        \
  } while (0)

// ----- blocks of vectors (deflation): FP64, RHS-major [m][n] -----------------
// row chunks of the Gram reduction over n for an ma x mb product
int gram_chunks(int64_t n, int ma, int mb);
// part[c][i][j] = sum over chunk c of A[i][r] B[j][r] (nchunks chunks of n)
void gram_partials(const double* A, int ma, const double* B, int mb, int64_t n, int nchunks,
                   double* part, hipStream_t s);
// C[i][j] = sum_c part[c][i][j] in chunk order (row-major ma x mb)
void gram_finish(const double* part, int nchunks, int ma, int mb, double* C, hipStream_t s);
// Out[j][r] = beta X[j][r] + alpha sum_{m < kk} U[m][r] C[m * ldc + j], j < nc;
// Out may equal X; X is not read when beta == 0
void block_combine(const double* U, int kk, const double* C, int ldc, const double* X,
                   double* Out, int nc, int64_t n, double alpha, double beta, hipStream_t s);

// streaming device copy of bytes (a multiple of 16, 16-byte aligned pointers)
void stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

// ----- vectors ---------------------------------------------------------------
template <typename T>
void vec_zero(T* x, int64_t n, int nb, const int* active, hipStream_t s);
template <typename T>
void vec_copy(const T* x, T* y, int64_t n, int nb, const int* active, hipStream_t s);
template <typename To, typename From>
void vec_convert(const From* x, To* y, int64_t n, int nb, const int* active, hipStream_t s);

// number of partial sums per column for a reduction over n elements
int reduce_blocks(int64_t n);
// partials[k*nblk + b] (re, im) = sum over block b of conj(x) y, column k
template <typename T>
void vec_dot_partials(const T* x, const T* y, int64_t n, int nb, const int* active,
                      c64* partials, hipStream_t s);
// out[k] = fixed-order sum of column k's nblk partials
void finish_sums(const c64* partials, int nblk, int nb, c64* out, hipStream_t s);
// refined CG: rz = 0 (so the next beta is 0) for active columns whose FP64
// residual after a refinement exceeds factor x the recursion's own residual
void cg_restart_on_drift(const c64* rr_new, const c64* rr_rec, c64* rz, const int* active,
                         double factor, int nb, hipStream_t s);

// ----- Krylov scalars (one thread per column) --------------------------------
// finish_sums into pq, then cg_alpha from it, in one launch (same values)
void finish_alpha(const c64* partials, int nblk, int nb, c64* pq, const c64* rz,
                  const int* active, c64* alpha, hipStream_t s);
// finish_sums into rz_new, then cg_beta from it, in one launch (same values)
void finish_beta(const c64* partials, int nblk, int nb, c64* rz_new, c64* rz, const int* active,
                 c64* beta, hipStream_t s);
// alpha = active ? rz/pq : 0   (Hermitian CG, real rz and pq)
void cg_alpha(const c64* rz, const c64* pq, const int* active, c64* alpha, int nb,
              hipStream_t s);
// beta = rz_new/rz ; rz = rz_new
void cg_beta(const c64* rz_new, c64* rz, const int* active, c64* beta, int nb,
             hipStream_t s);
// active[k] &= (rr[k] > tol2 * ref[k]); count = number still active
void mark_converged(const c64* rr, const c64* ref, double tol2, int* active, int nb,
                    int* count, hipStream_t s);
void count_active(const int* active, int nb, int* count, hipStream_t s);
void set_all_active(int* active, int nb, hipStream_t s);
void set_count(int* count, int value, hipStream_t s);
// count = number of active columns with rr <= delta2 * rr_upd or rr <= tol2 * bb
void refine_due(const c64* rr, const c64* rr_upd, const c64* bb, double delta2, double tol2,
                const int* active, int nb, int* count, hipStream_t s);
// err[k] = |bd[k]| * sqrt(rr_new[k]/rr_old[k]) for active columns
void ir_stated_error(const c64* bd, const c64* rr_old, const c64* rr_new, const int* active,
                     c64* err, int nb, hipStream_t s);
// dst[k] = active[k] ? src[k] : dst[k]
void select_active(c64* dst, const c64* src, const int* active, int nb, hipStream_t s);
// lastcorr[k] = alpha[k]*rz[k] for active columns (CG step's share of b^H x)
void cg_lastcorr(const c64* alpha, const c64* rz, const int* active, c64* lastcorr, int nb,
                 hipStream_t s);

// x += alpha p ; r -= alpha q ; partials of |r|^2.  x_zero: x is taken as zero
// and not read (the first update of a solve), x = alpha p
template <typename T>
void cg_update_xr(T* x, T* r, const T* p, const T* q, const c64* alpha, int64_t n,
                  int nb, const int* active, c64* partials, hipStream_t s,
                  bool x_zero = false);
// p = z + beta p
template <typename T>
void cg_update_p(T* p, const T* z, const c64* beta, int64_t n, int nb,
                 const int* active, hipStream_t s);
// refinement fold in one pass: y += d, partials of b^T d (reduce_blocks(n)
// blocks per column, as vec_dot_partials(b, d)), d = 0.  y_zero: y is taken as
// zero and not read (the first fold of a solve), y = 0 + d
void ir_fold(double* y, float* d, const double* b, int64_t n, int nb, const int* active,
             c64* partials, hipStream_t s, bool y_zero = false);
// the same with b given in FP32 (exactly: the values of the FP64 b)
void ir_fold(double* y, float* d, const float* b, int64_t n, int nb, const int* active,
             c64* partials, hipStream_t s, bool y_zero = false);
// r = b32 = b rounded to FP32 (nb columns of n); *inexact = 0 when every entry of
// b is an FP32 number (b32 then holds b exactly), else 1; partials of b^T b as
// vec_dot_partials(b, b) writes them (reduce_blocks(n) per column, same sums)
void rhs_fp32(const double* b, float* r, float* b32, int64_t n, int nb, int* inexact,
              c64* partials, hipStream_t s);
// y64 += convert(d)
template <typename T64, typename T32>
void ir_accumulate(T64* y, const T32* d, int64_t n, int nb, const int* active,
                   hipStream_t s);
// out = a - b
template <typename T>
void vec_sub(const T* a, const T* b, T* out, int64_t n, int nb, hipStream_t s);
// y += x (active columns)
template <typename T>
void vec_add_to(T* y, const T* x, int64_t n, int nb, const int* active, hipStream_t s);
// y += a[k] * x  (column scalars)
template <typename T>
void vec_axpy_cols(T* y, const T* x, const c64* a, int64_t n, int nb,
                   const int* active, hipStream_t s);

// ----- probes and quadratic forms -------------------------------------------
template <typename T>
void probes_write(T* out, int64_t n, int nb, uint64_t seed, uint64_t problem,
                  uint64_t first_sample, uint64_t level, uint64_t stream,
                  hipStream_t s);
// partials of x_k^H y_k with x_k regenerated from the RNG
template <typename T>
void probe_dot_partials(const T* y, int64_t n, int nb, uint64_t seed, uint64_t problem,
                        uint64_t first_sample, uint64_t level, uint64_t stream,
                        c64* partials, hipStream_t s);

// ----- dense coarsest level -------------------------------------------------
// inverse of the n x n matrix A held row-major with leading dimension lda in M
// (overwritten) by blocked Gauss-Jordan with partial pivoting; out receives
// A^{-1} row-major with leading dimension n.  Work: rowbuf kGjPanel + 1
// elements, colbuf n, tbuf kGjPanel * n, ipiv 2n + 1 ints; ipiv[2n] is set to
// 1 when a pivot is zero or not a number (A singular)
constexpr int kGjPanel = 64;
template <typename T>
void dense_inverse(T* M, int n, int64_t lda, T* out, T* rowbuf, T* colbuf, T* tbuf, int* ipiv,
                   hipStream_t s);
// trace partial: out = sum_i A[i][i] (single block)
template <typename T>
void dense_trace(const T* A, int n, c64* out, hipStream_t s);
// Z[k][i] = sum_j At[j][i] B[k][j], k < nb: the coarsest solve z_k = A^{-1} b_k
// with At the transposed inverse.  ld (0: n): leading dimension of At.  Real T
// with ld a multiple of 16 (dense_mfma_layout): the MFMA tile kernel, for any
// n, with At zero-padded to ld x ld and given in the layout of dense_pack4;
// otherwise (ld == n) a plain row-major At.
template <typename T>
void dense_apply(const T* At, const T* B, T* Z, int n, int nb, const int* active,
                 hipStream_t s, int ld = 0);
template <typename T>
constexpr bool dense_mfma_layout(int ld) {
  return (std::is_same<T, float>::value || std::is_same<T, double>::value) && ld % 16 == 0;
}
// the MFMA tile kernel's layout of an ld x ld row-major matrix At (ld a
// multiple of 4): out[((j / 4) ld + i) 4 + j % 4] = At[j][i], so the four
// consecutive rows j a lane reads for one column i are contiguous
template <typename T>
void dense_pack4(const T* At, T* out, int ld, hipStream_t s);
// Mt (2n x 2n, real) = transposed real representation of the complex matrix
// whose transpose is At, for dense_apply<R> on interleaved (re, im) vectors
template <typename T, typename R>
void dense_complex_to_real(const T* At, R* Mt, int n, hipStream_t s);
// out[j][i] = in[i][j] (n x n)
template <typename T>
void dense_transpose(const T* in, T* out, int n, hipStream_t s);

// ----- 2D Poisson stencil: A = d I - c (grid neighbours), N x N Dirichlet -----
// partial-sum counts per column of the tiled kernels
int poisson_march_tiles(int N);   // apply / residual
// fused Gauss-Seidel pass of `sweeps` (1 or 2) sweeps, `rows` per segment
template <typename T>
int poisson_gs_tiles(int N, int rows, int sweeps);
// the three segment lengths the sweep is compiled for (ascending)
template <typename T>
void gs_rows_options(int out[3]);
template <typename T>
void poisson_dense_build(T* aug, int N, double d, double c, hipStream_t s);
// y = A x ; optional partials of conj(x)^T y (pass partials = nullptr to skip)
template <typename T>
void poisson_apply(const T* x, T* y, int N, double d, double c, int nb,
                   const int* active, c64* partials, hipStream_t s);
// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q
template <typename T>
void poisson_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q, int N,
                          double d, double c, int nb, const int* active, c64* partials,
                          hipStream_t s);
// r = b - A x (Tr may be lower precision) ; optional partials of |r|^2
template <typename Tb, typename Tx, typename Tr>
void poisson_residual(const Tb* b, const Tx* x, Tr* r, int N, double d, double c,
                      int nb, const int* active, c64* partials, hipStream_t s);
// one pass of `sweeps` (1 or 2; 2 needs N >= 64) red-black Gauss-Seidel sweeps,
// fused: xout = S^sweeps(xin + omega/2 P ec ; b), red first (reverse: black
// first) in every sweep; xin == nullptr means 0, ec == nullptr no correction;
// partials (nullable): shares of conj(b)^T xout, gs_tiles per column; rows:
// segment length (one of gs_rows_options; a tuning choice that does not change
// the swept values).  Two sweeps in one pass equal two one-sweep passes bit for
// bit.
template <typename T>
void poisson_rbgs_fused(const T* xin, const T* b, T* xout, const T* ec, double omega, int N,
                        double d, double c, int nb, const int* active, bool reverse,
                        c64* partials, int rows, int sweeps, hipStream_t s);
// last pre-smoothing pass: xout = S^2(xin ; b) (two fused sweeps, red first;
// xin == nullptr means 0) and rc = R (b - A xout) in the same pass; N even, >= 64
template <typename T>
void poisson_rbgs_restrict(const T* xin, const T* b, T* xout, T* rc, int N, double d, double c,
                           int nb, const int* active, int rows, hipStream_t s);
// rc = R (b - A x), R = P^T, P the orthonormal 2x2 aggregation (entries 1/2)
template <typename T>
void poisson_residual_restrict(const T* b, const T* x, T* rc, int N, double d,
                               double c, int nb, const int* active, hipStream_t s);
// xc = R x
template <typename T>
void agg2d_restrict(const T* x, T* xc, int N, int nb, const int* active, hipStream_t s);
// x = beta*x + omega * P ec
template <typename T>
void agg2d_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                   const int* active, hipStream_t s);

// ----- 3D 7-point variable-coefficient operator, N^3 cells, Dirichlet faces -----
// Face coefficients of one level: k[3][N][N][N+1] (x-faces [z][y][f], y-faces
// [z][x][f], z-faces [y][x][f]); the stencil kernels read the cell-major
// couplings kl[3][N^3 + N^2] (face below cell i in x, y, z; zero on the
// boundary; padded) and diag dg[i] = shift + the six faces of cell i.  `cols`
// (1, 2, 4 or 8): right-hand sides per thread, a tuning choice that does not
// change results.
int varcoef_blocks(int N);  // partial sums per column of residual / update_apply
// r = b - A x ; b == nullptr: r = A x (partials then of conj(x)^T r)
template <typename Tb, typename T, typename Tr>
void varcoef_residual(const Tb* b, const T* x, Tr* r, const typename Traits<T>::real* kl,
                      const typename Traits<T>::real* dg, int N, int nb, int cols,
                      const int* active, c64* partials, hipStream_t s);
// one in-place red-black Gauss-Seidel sweep (reverse: black first); zero_init:
// x = 0 on entry (not read); ec (nullable): x + omega P ec is swept instead of
// x (the coarse-grid correction folded into the sweep; the result is written
// to x)
template <typename T>
void varcoef_rbgs(const T* b, T* x, const typename Traits<T>::real* kl,
                  const typename Traits<T>::real* dg, int N, int nb, int cols, const int* active,
                  bool zero_init, bool reverse, const T* ec, double omega, hipStream_t s);
// one red-black sweep fused into one out-of-place pass (both colours; reverse:
// black first): xout = S(xin + omega/sqrt(8) P ec ; b); xin == nullptr means 0,
// ec nullable; `cols` in {1, 2, 4}: right-hand sides per lane.  For even sides
// up to 128 (varcoef_march_ok).
bool varcoef_march_ok(int N);
template <typename T>
void varcoef_rbgs_march(const T* xin, const T* b, T* xout, const T* ec, double omega,
                        const typename Traits<T>::real* kl, const typename Traits<T>::real* dg,
                        int N, int nb, int cols, const int* active, bool reverse,
                        hipStream_t s);
// xc = R (b - A x) when residual, else xc = R x; R the orthonormal 2x2x2
// aggregation (entries 1/sqrt(8))
template <typename T>
void varcoef_restrict(const T* b, const T* x, T* xc, const typename Traits<T>::real* kl,
                      const typename Traits<T>::real* dg, int N, bool residual, int nb, int cols,
                      const int* active, hipStream_t s);
// x = beta x + omega P ec
template <typename T>
void varcoef_prolong(const T* ec, T* x, int N, double omega, double beta, int nb,
                     const int* active, hipStream_t s);
// p_new = z + beta p_old ; q = A p_new ; partials of conj(p_new)^T q
template <typename T>
void varcoef_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                          const typename Traits<T>::real* kl,
                          const typename Traits<T>::real* dg, int N, int nb, int cols,
                          const int* active, c64* partials, hipStream_t s);
// Galerkin faces of the next level: kc = 1/8 (sum of the 4 fine faces covered)
void varcoef_coarsen(const double* kf, double* kc, int N, hipStream_t s);
// diagonal and cell-major couplings (FP64 and FP32) of one level
void varcoef_diag(const double* k, double shift, int N, double* d64, float* d32, double* kl64,
                  float* kl32, hipStream_t s);
// left half of aug (n x 2n row-major, n = N^3) = the dense operator
void varcoef_dense(const double* k, const double* diag, int N, double* aug, hipStream_t s);

// ----- learned smoother (2-spin lattice; N a multiple of 16) --------------------
// weights: 4032 FP32 values, W1 [16][8][3][3], W2 [16][16][3][3], W3 [4][16][3][3]
int nn_num_weights();
int nn_frag_count();          // packed BF16 B fragments (16 bytes each)
int nn_crop_in_elems();       // BF16 per training-crop input (22 * 22 * 8)
int nn_crop_out_elems();      // FP32 per training-crop target (16 * 16 * 4)
int nn_crop_side();           // 22
// link features (cos, sin of theta_mu) in BF16 [site][4]; theta [2][N][N] FP64
void nn_links(const double* theta, void* links, int N, hipStream_t s);
// BF16 B fragments of the three layers from the FP32 master weights
void nn_pack(const float* w, void* frag, hipStream_t s);
// x += s * net(r / s), s^2 = rr[k].re * inv_n per column (skipped when 0)
void nn_apply(const c32* r, c32* x, const c64* rr, double inv_n, const void* links,
              const void* frag, int N, int nb, const int* active, hipStream_t s);
// forward + backward of ncrops crops (crop order[i], or i when order is null):
// per-crop gradients, then grad = their fixed-order sum and *loss = the mean
// squared error
void nn_train_step(const void* in, const float* tgt, const int* order, int ncrops,
                   const void* frag, const float* w, float* gpart, double* lpart, float* grad,
                   double* loss, hipStream_t s);
// Adam step t (from 1) on the FP32 master weights
void nn_adam(float* w, float* m, float* v, const float* g, double lr, double b1, double b2,
             double eps, int t, hipStream_t s);
// training crops from FP64 residual / error fields (origin: column, y0, x0 per crop)
void nn_crops(const c64* r, const c64* e, const c64* rr, double inv_n, const void* links,
              const int* origin, int ncrops, int N, void* in, float* tgt, hipStream_t s);
void nn_round_inputs(const float* src, void* dst, int64_t count, hipStream_t s);

// ----- complex lattice operators (Wilson 2-spin, block stencils, transfers) ---
int wilson_residual_blocks(int N);
int bsr_residual_blocks(int Nc);
// r = b - D x ; b == nullptr: r = D x (partials then of conj(x)^T r)
template <typename Tb, typename T, typename Tr>
void wilson_residual(const Tb* b, const T* x, Tr* r, const T* U, int N, double diag, int nb,
                     const int* active, c64* partials, hipStream_t s);
template <typename T>
void wilson_rbgs(const T* b, T* x, const T* U, int N, double diag, int nb, const int* active,
                 bool zero_init, bool reverse, hipStream_t s);
// one red-black sweep with both colours in one launch, out of place: xout =
// S(xin) (xin unread when zero_init, else it must differ from xout); needs
// wilson_rbgs_fused_ok(N) (side divisible by 16)
bool wilson_rbgs_fused_ok(int N);
template <typename T>
void wilson_rbgs_fused(const T* b, const T* xin, T* xout, const T* U, int N, double diag, int nb,
                       const int* active, bool zero_init, bool reverse, hipStream_t s);
// block stencils: form 0 = a thread per (site, column), 1 = a wave per site
// and 64 columns with the site's blocks read wave-uniformly (a tuning choice;
// results agree up to rounding); partial sums always come from form 0
template <typename Tb, typename T, typename Tr>
void bsr_residual(const Tb* b, const T* x, Tr* r, const T* B, int Nc, int dof, int nb,
                  const int* active, c64* partials, int form, hipStream_t s);
template <typename T>
void bsr_rbgs(const T* b, T* x, const T* B, const T* Dinv, int Nc, int dof, int nb,
              const int* active, bool zero_init, bool reverse, int form, hipStream_t s);
template <typename T>
void agg_restrict(const T* x, T* xc, const T* q, int Nf, int dofF, int blk, int dofC, int nb,
                  const int* active, hipStream_t s);
template <typename T>
void agg_prolong(const T* xc, T* x, const T* q, int Nf, int dofF, int blk, int dofC,
                 double omega, double beta, int nb, const int* active, hipStream_t s);
void wilson_links(const double* theta, c64* U64, c32* U32, int N, hipStream_t s);
// gauge Laplacian (4 + m) I - linked neighbours as 1 x 1 blocks B[site][5]
void gauge_blocks(const c64* U, int N, double diag, c64* B, hipStream_t s);
void agg_orthonormalise(const c64* V, c64* q, int Nf, int dofF, int blk, int nv, bool split,
                        hipStream_t s);
void galerkin_blocks(const c64* Bf, const c64* U, double wdiag, const c64* q, int Nf, int dofF,
                     int blk, int nv, c64* Bc, hipStream_t s);
void dense_from_stencil(const c64* Bf, const c64* U, double wdiag, int Nf, int dof, c64* aug,
                        hipStream_t s);
void block_diag_inverse(const c64* B, c64* Dinv64, c32* Dinv32, int ns, int dof, hipStream_t s);
// the 5 dof-blocks of every row of a block stencil (or the Wilson operator) as
// column indices and values, 5 * dof entries per row, direction-major
void stencil_entries(const c64* Bf, const c64* U, double wdiag, int Nf, int dof, int* cols,
                     c64* vals, hipStream_t s);

// ----- batched flexible GMRES helpers ------------------------------------------
template <typename T>
void krylov_mdot(const T* V, int64_t vstride, int nv, const T* w, int64_t n, int nb,
                 const int* active, c64* partials, int* nblk_out, hipStream_t s);
template <typename T>
void krylov_maxpy(const T* V, int64_t vstride, int nv, const c64* h, T* w, int64_t n, int nb,
                  const int* active, hipStream_t s);
template <typename T>
void krylov_combine(const T* Z, int64_t vstride, const c64* y, int ldy, const int* dims, T* d,
                    int64_t n, int nb, const int* start, hipStream_t s);
template <typename T>
void vec_scale_inv_norm(T* dst, const T* src, const c64* nrm2, int64_t n, int nb,
                        const int* active, hipStream_t s);
void givens_init(c64* H, c64* cs, c64* sn, c64* g, int* dims, const c64* beta2,
                 const int* active, int m, int nb, hipStream_t s);
void givens_step(c64* H, c64* cs, c64* sn, c64* g, int* dims, const c64* h, const c64* wn2,
                 const c64* beta2, double tol, int j, int m, int* active, int nb, int* count,
                 hipStream_t s);
void givens_solve(c64* H, c64* cs, c64* sn, c64* g, int* dims, c64* y, const int* start, int m,
                  int nb, hipStream_t s);

// ----- general sparse (CSR) operators -----------------------------------------
// The kernels read sliced ELLPACK copies (SELL-64): slice s holds 64
// consecutive rows (or colour-class positions) and w_s = (sptr[s+1] -
// sptr[s]) / 64 entries per row, entry e of lane l at sptr[s] + 64 e + l, so
// the column indices and values of a wave's rows load coalesced and every lane
// runs the same trip count.  Entries keep the row's column order; rows shorter
// than w_s are padded with value 0 and their own row as column.
//
// A by rows, diagonal included (device arrays; values in precision T); rp/ci/v
// are the plain CSR arrays (dense build of the coarsest level)
template <typename T>
struct CsrMat {
  int n = 0;                  // rows
  int ncol = 0;               // columns (the length of the vectors it multiplies)
  const int* rp = nullptr;    // n + 1 row offsets
  const int* ci = nullptr;    // column of each entry
  const T* v = nullptr;       // value of each entry
  const int* sptr = nullptr;  // SELL-64 slice offsets (ceil(n/64) + 1)
  const int* sci = nullptr;
  const T* sv = nullptr;
};
// the off-diagonal part with rows grouped by colour class, in SELL-64 slices
// that never straddle two classes: class c owns slices soff[c]..soff[c+1]-1
// (host offsets); position k = 64 s + l holds row srow[k] (-1: padding) with
// sdi[k] = 1 / a_ii
template <typename T>
struct CsrSweep {
  const int *srow = nullptr, *sptr = nullptr, *sci = nullptr;
  const T *sv = nullptr, *sdi = nullptr;
  std::vector<int> soff;
};
// aggregation to the next level: agg[i] = aggregate of unknown i; the members
// of J are arows[aptr[J]..aptr[J+1]-1] (ascending); fs[i] = cs[agg[i]] = 1/sqrt|J|
template <typename T>
struct CsrAgg {
  int nc = 0;
  const int *agg = nullptr, *aptr = nullptr, *arows = nullptr;
  const T *fs = nullptr, *cs = nullptr;
};
int csr_blocks(int n);  // partial sums per column of csr_residual / csr_update_apply
// r = b - A x (r = A x when b is null); partials as the stencil residuals
template <typename Tb, typename T, typename Tr>
void csr_residual(const Tb* b, const T* x, Tr* r, const CsrMat<T>& A, int nb, int cols,
                  const int* active, c64* partials, hipStream_t s);
// p_new = z + beta p_old, q = A p_new, partials of p_new^T q
template <typename T>
void csr_update_apply(const T* p_old, const T* z, const c64* beta, T* p_new, T* q,
                      const CsrMat<T>& A, int nb, int cols, const int* active, c64* partials,
                      hipStream_t s);
// One Gauss-Seidel sweep in place over the colour classes (reverse: last class
// first).  Each class is one launch, except the trailing run of classes of at
// most tail_slices slices each (csr_tail_start; tail_slices 0: none), which
// shares launches of up to kMaxTailClasses classes: one workgroup of
// kTailWaves waves per column group, a barrier between classes.  The rows of a
// class are independent, so both schedules give the same result.
constexpr int kTailWaves = 16;
constexpr int kMaxTailClasses = 64;
struct CsrTail {
  int count, reverse;
  int soff[kMaxTailClasses + 1];
};
inline int csr_tail_start(const std::vector<int>& soff, int tail_slices) {
  int c = (int)soff.size() - 1;
  if (tail_slices <= 0) return c;
  while (c > 0 && soff[c] - soff[c - 1] <= tail_slices) --c;
  return c;
}
template <typename T>
void csr_gs_sweep(const T* b, T* x, const CsrSweep<T>& S, int n, int nb, int cols,
                  int tail_slices, const int* active, bool reverse, hipStream_t s);
// xc = R (b - A x) (b non-null; the residual goes through rtmp, n x nb) or
// xc = R x (b null), R = P^T
template <typename T>
void csr_restrict(const T* b, const T* x, T* xc, T* rtmp, const CsrMat<T>& A,
                  const CsrAgg<T>& G, int nb, int cols, const int* active, hipStream_t s);
// x = beta x + omega P ec
template <typename T>
void csr_prolong(const T* ec, T* x, const CsrAgg<T>& G, int n, double omega, double beta, int nb,
                 const int* active, hipStream_t s);
// left half of the n x 2n augmented matrix [A | .] (rows of width 2n)
void csr_dense(const CsrMat<double>& A, double* aug, hipStream_t s);
// y = beta y + w M x for a rectangular M (M.n x M.ncol; y has M.n, x M.ncol
// entries per column; beta = 0: y is not read): the general prolongation
// (M = P) and restriction (M = R = P^T) between CSR levels
template <typename T>
void csr_spmm(const T* x, T* y, const CsrMat<T>& M, double w, double beta, int nb, int cols,
              const int* active, hipStream_t s);

}  // namespace mlmc
