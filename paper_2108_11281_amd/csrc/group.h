// Grouped solves over several problems (a batch of uneven 3D diffusion
// problems): the refined CG of every problem runs in lockstep on one stream,
// each of its steps one launch over all problems, and each V-cycle of all
// problems as one launch per stage position (the stages at that position of
// every problem's V-cycle: (problem, level, stage, tile) items of one launch).
#pragma once

#include "kernels.h"

namespace mlmc {

// ---- V-cycle stages ---------------------------------------------------------
enum GStageKind : int {
  kGsMarch = 0,        // fused red-black sweep marching along z (both colours)
  kGsResRestrict = 1,  // rc = R (b - A x), 2x2x2 aggregates
  kGsDense = 2,        // coarsest level: Z = B A^-1 on MFMA
  kGsDot = 3,          // partials of conj(b)^T x (the preconditioned r^T z)
  kGsCopy = 4,         // y = x (active columns)
};

// workgroup of the stage kernel (eight waves: the march needs them)
constexpr int kGroupThreads = 512;
// right-hand sides per wave of the grouped march and per thread of the grouped
// residual restriction (the results do not depend on them)
constexpr int kGroupMarchCols = 2;
constexpr int kGroupRrCols = 2;

struct GStage {
  int kind;
  int hx, he, f;     // march: x_in given, folded correction, first colour
  int rpw;           // march: rows per wave (1, 2, 4)
  int N;             // grid side (march, residual restriction)
  int nb;            // columns
  int gx, gy, gz;    // virtual grid of the stage
  int tiles;         // workgroup items
  int sz;            // march: planes per z segment
  int ld, nblk;      // dense: leading dimension of the inverse; dot: blocks per column
  int64_t n;         // unknowns of the level
  float ws;          // march: omega / sqrt(8)
  const float* in;   // x_in (march), x (residual restriction, dot, copy), B (dense)
  const float* b;    // right-hand side (march, residual restriction, dot)
  const float* ec;   // coarse correction (march)
  const float* kl;   // couplings
  const float* dg;   // diagonal
  const float* At;   // transposed, padded coarsest inverse (dense)
  float* out;        // x_out / rc / Z / y
  const int* act;    // per-column flags
  c64* partials;     // dot
};

// kernel instance of a stage: its kind, or for sweeps one of 12 forms (rows
// per wave 1, 2, 4 x from zero / from x / with correction / without)
int group_stage_key(const GStage& g);
// Runs a set of independent stages of one key in one launch (grid = total
// items, item i of the concatenated stages per workgroup).  tstart: prefix
// sums of the stages' items (nst + 1 entries).
void group_stages(const GStage* st, int nst, const int* tstart, int total, int key,
                  hipStream_t s);

// Persistent V-cycle: one workgroup per unit (a problem's column pair) runs
// every stage of that problem's V-cycle for its two columns.  units: nunits x
// (first stage, end stage, column pair) into st; stage items and the bodies
// are those of group_stages, restricted to the pair.
void group_vcycle_units(const GStage* st, const int* units, int nunits, hipStream_t s);

// ---- refined CG steps over several problems -----------------------------------
struct GTask {
  int N, nb, ntiles, nblk;  // side, columns, stencil blocks, reduction blocks
  int64_t n;
  const float *kl32, *dg32;
  const double *kl64, *dg64;
  float *x32, *r, *z, *P1, *P2, *q;
  const double* b;
  double* y;
  c64 *rz, *tmp, *alpha, *beta, *bb, *bd, *rr_upd, *rr_new, *err;
  int* act;
  c64* partials;
  int* count;  // the task's refinement-due and still-active counts
  double delta2, tol2;
};

// Launch tables of a set of tasks (device ints): [0] = count t, [1 .. t] =
// indices into the GTask array, then four prefix arrays of t + 1 entries:
// blocks of the stencil shape (ntiles x ceil(nb / kGroupStencilCols)), of the
// reduction shape (nblk x nb), of the per-column shape (nb) and one per task.
constexpr int kGroupStencilCols = 8;
enum { kShStencil = 0, kShReduce = 1, kShColumn = 2, kShTask = 3 };
inline int group_table_ints(int t) { return 1 + t + 4 * (t + 1); }

// p_new = z + beta p_old ; q = A p_new ; partials (stencil shape).  sel: which
// of z, P1, P2 is p_old (0, 1, 2) and which of P1, P2 is p_new (1, 2)
void group_update_apply(const GTask* tasks, const int* tab, int blocks, int old_sel,
                        int new_sel, hipStream_t s);
// pq = finish(partials over ntiles) into tmp ; alpha from it
void group_finish_alpha(const GTask* tasks, const int* tab, int blocks, hipStream_t s);
// x32 += alpha p_new ; r -= alpha q ; partials of |r|^2 (reduction shape)
void group_cg_xr(const GTask* tasks, const int* tab, int blocks, int new_sel, hipStream_t s);
// which: 0 tmp (nblk), 1 rz (nblk), 2 bd (nblk), 3 rr_new (ntiles)
void group_finish(const GTask* tasks, const int* tab, int blocks, int which, hipStream_t s);
// rz_new (into tmp) = finish(partials over nblk) ; beta ; rz = rz_new
void group_finish_beta(const GTask* tasks, const int* tab, int blocks, hipStream_t s);
// count[0] = columns due for a refinement (one block per task)
void group_refine_due(const GTask* tasks, const int* tab, int blocks, hipStream_t s);
// y += x32 ; partials of b^T x32 ; x32 = 0 (reduction shape)
void group_ir_fold(const GTask* tasks, const int* tab, int blocks, hipStream_t s);
// r = b - A y in FP64, rounded to FP32, partials of |r|^2 (stencil shape)
void group_ir_residual(const GTask* tasks, const int* tab, int blocks, hipStream_t s);
// per column, in this order: stated error, direction restart on drift,
// rr_upd = rr_new, convergence mark; count[1] = columns still active
void group_refine_rules(const GTask* tasks, const int* tab, int blocks, double factor,
                        hipStream_t s);

}  // namespace mlmc
