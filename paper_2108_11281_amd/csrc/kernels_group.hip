// Kernels of the grouped solves over several problems: the steps of the
// refined CG as one launch over all problems (each block finds its problem in
// a table of prefix sums and runs the one-problem kernel's body on its own
// block index), and the V-cycle stage kernel, which runs one stage of every
// problem's V-cycle (the stages at the same position of each) per launch.  The
// bodies are those of the one-problem kernels, so every problem's results are
// identical to its own solve.
#include "group.h"
#include "vc_body.h"
#include "vec_body.h"

namespace mlmc {
namespace {

// task of block b: the last t with start[t] <= b
__device__ __forceinline__ int find_slot(const int* start, int nt, int b) {
  int lo = 0, hi = nt;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

struct Slot {
  const GTask* t;
  int local;  // block index within the task's grid
};

__device__ __forceinline__ Slot slot_of(const GTask* tasks, const int* tab, int shape) {
  const int nt = tab[0];
  const int* start = tab + 1 + nt + shape * (nt + 1);
  const int i = find_slot(start, nt, (int)blockIdx.x);
  return Slot{tasks + tab[1 + i], (int)blockIdx.x - start[i]};
}

__device__ __forceinline__ float* pick(const GTask& t, int sel) {
  return sel == 0 ? t.z : (sel == 1 ? t.P1 : t.P2);
}

__global__ __launch_bounds__(kThreads) void kg_update_apply(const GTask* tasks, const int* tab,
                                                            int old_sel, int new_sel) {
  __shared__ double red[16];
  const Slot s = slot_of(tasks, tab, kShStencil);
  const GTask& t = *s.t;
  const int gx = t.ntiles;
  vcb::vc_update_apply<float, kGroupStencilCols>(pick(t, old_sel), t.z, t.beta, pick(t, new_sel),
                                                 t.q, t.kl32, t.dg32, t.N, t.nb, t.act,
                                                 t.partials, nullptr, s.local % gx,
                                                 s.local / gx, gx, red);
}

__global__ __launch_bounds__(kThreads) void kg_finish_alpha(const GTask* tasks, const int* tab) {
  __shared__ double lds[16];
  const Slot s = slot_of(tasks, tab, kShColumn);
  const GTask& t = *s.t;
  const int k = s.local;
  const c64 v = body::finish(t.partials, t.ntiles, k, lds);
  if (threadIdx.x == 0) {
    t.tmp[k] = v;
    body::alpha_rule(v, t.rz, t.act, k, t.alpha);
  }
}

__global__ __launch_bounds__(kThreads) void kg_cg_xr(const GTask* tasks, const int* tab,
                                                     int new_sel) {
  __shared__ double lds[16];
  const Slot s = slot_of(tasks, tab, kShReduce);
  const GTask& t = *s.t;
  const int k = s.local / t.nblk, bx = s.local % t.nblk;
  if (!t.act[k]) return;
  body::cg_xr(t.x32, t.r, pick(t, new_sel), t.q, t.alpha[k], t.n, t.nblk, bx, k, t.partials,
              lds);
}

__global__ __launch_bounds__(kThreads) void kg_finish(const GTask* tasks, const int* tab,
                                                      int which) {
  __shared__ double lds[16];
  const Slot s = slot_of(tasks, tab, kShColumn);
  const GTask& t = *s.t;
  const int k = s.local;
  const int nblk = which == 3 ? t.ntiles : t.nblk;
  const c64 v = body::finish(t.partials, nblk, k, lds);
  if (threadIdx.x == 0) {
    c64* out = which == 0 ? t.tmp : (which == 1 ? t.rz : (which == 2 ? t.bd : t.rr_new));
    out[k] = v;
  }
}

__global__ __launch_bounds__(kThreads) void kg_finish_beta(const GTask* tasks, const int* tab) {
  __shared__ double lds[16];
  const Slot s = slot_of(tasks, tab, kShColumn);
  const GTask& t = *s.t;
  const int k = s.local;
  const c64 v = body::finish(t.partials, t.nblk, k, lds);
  if (threadIdx.x == 0) {
    t.tmp[k] = v;
    body::beta_rule(v, t.rz, t.act, k, t.beta);
  }
}

__global__ __launch_bounds__(kThreads) void kg_refine_due(const GTask* tasks, const int* tab) {
  __shared__ int cnt;
  const Slot s = slot_of(tasks, tab, kShTask);
  const GTask& t = *s.t;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < t.nb; k += blockDim.x) {
    if (!t.act[k]) continue;
    if (body::due_rule(t.tmp, t.rr_upd, t.bb, t.delta2, t.tol2, k)) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) t.count[0] = cnt;
}

__global__ __launch_bounds__(kThreads) void kg_ir_fold(const GTask* tasks, const int* tab) {
  __shared__ double lds[16];
  const Slot s = slot_of(tasks, tab, kShReduce);
  const GTask& t = *s.t;
  const int k = s.local / t.nblk, bx = s.local % t.nblk;
  if (!t.act[k]) return;
  body::ir_fold(t.y, t.x32, t.b, t.n, t.nblk, bx, k, t.partials, lds);
}

__global__ __launch_bounds__(kThreads) void kg_ir_residual(const GTask* tasks, const int* tab) {
  __shared__ double red[16];
  const Slot s = slot_of(tasks, tab, kShStencil);
  const GTask& t = *s.t;
  const int gx = t.ntiles;
  vcb::vc_residual<double, double, float, kGroupStencilCols>(
      t.b, t.y, t.r, t.kl64, t.dg64, t.N, t.nb, t.act, t.partials, nullptr, s.local % gx,
      s.local / gx, gx, red);
}

__global__ __launch_bounds__(kThreads) void kg_refine_rules(const GTask* tasks, const int* tab,
                                                            double factor) {
  __shared__ int cnt;
  const Slot s = slot_of(tasks, tab, kShTask);
  const GTask& t = *s.t;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < t.nb; k += blockDim.x) {
    if (t.act[k]) {
      body::ir_err_rule(t.bd, t.rr_upd, t.rr_new, t.err, k);
      body::restart_rule(t.rr_new, t.tmp, t.rz, factor, k);
      t.rr_upd[k] = t.rr_new[k];
    }
    if (body::mark_rule(t.rr_new, t.bb, t.tol2, t.act, k)) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) t.count[1] = cnt;
}

// ---------------------------------------------------------------------------
// V-cycle stages
// ---------------------------------------------------------------------------
template <int RPW, int HX, int HE, int F>
__device__ __forceinline__ void march(const GStage& g, int item, float* lds) {
  const int bx = item % g.gx, rest = item / g.gx;
  const int by = rest % g.gy, bz = rest / g.gy;
  vcb::vc_march<float, kGroupMarchCols, RPW, HX != 0, HE != 0, F>(
      g.in, g.b, g.out, g.ec, g.ws, g.kl, g.dg, g.N, g.sz, g.nb, g.act, nullptr, bx, by, bz,
      lds);
}

template <int RPW>
__device__ __forceinline__ void march_rpw(const GStage& g, int item, float* lds) {
  // the sweeps of a V-cycle: pre-smoothing from zero (0,0,0) and from x
  // (1,0,0); post-smoothing with the folded correction (1,1,1) and without
  // (1,0,1); other forms are not generated
  if (!g.hx) march<RPW, 0, 0, 0>(g, item, lds);
  else if (!g.f) march<RPW, 1, 0, 0>(g, item, lds);
  else if (g.he) march<RPW, 1, 1, 1>(g, item, lds);
  else march<RPW, 1, 0, 1>(g, item, lds);
}

struct StageLds {
  union {
    float march[vcb::vc_march_lds<float, kGroupMarchCols, 1>()];
    float part[2][4 * 4 * 64];
    double red[2][16];
  };
};

__device__ __forceinline__ void run_stage(const GStage& g, int item, StageLds& sm) {
  const int tid = threadIdx.x;
  switch (g.kind) {
    case kGsMarch:
      if (g.rpw == 1) march_rpw<1>(g, item, sm.march);
      else if (g.rpw == 2) march_rpw<2>(g, item, sm.march);
      else march_rpw<4>(g, item, sm.march);
      break;
    case kGsResRestrict:
      vcb::vc_res_restrict<float, kGroupRrCols, kGroupThreads>(g.b, g.in, g.out, g.kl, g.dg, g.N,
                                                               g.nb, g.act, nullptr,
                                                               item % g.gx, item / g.gx, tid);
      break;
    case kGsDense: {
      // two 256-thread blocks per item
      const int half = tid >> 8;
      const int vb = 2 * item + half;
      const bool live = vb < g.gx * g.gy;
      body::dense_apply_mfma<float>(g.At, g.in, g.out, (int)g.n, g.ld, g.nb, g.act, vb % g.gx,
                                    vb / g.gx, live, sm.part[half], tid & 255);
      break;
    }
    case kGsDot: {
      const int half = tid >> 8;
      const int vb = 2 * item + half;
      const int k = vb / g.nblk;
      const bool live = vb < g.nblk * g.nb && g.act[k];
      body::dot(g.b, g.in, g.n, g.nblk, vb % g.nblk, live ? k : 0, live, g.partials,
                sm.red[half], tid & 255);
      break;
    }
    default: {  // kGsCopy
      const int k = item / g.gx;
      const int64_t i = (int64_t)(item % g.gx) * kGroupThreads + tid;
      if (g.act[k] && i < g.n) g.out[(int64_t)k * g.n + i] = g.in[(int64_t)k * g.n + i];
      break;
    }
  }
}

// One launch runs a set of independent stages: item i of the concatenated
// stages per workgroup.
__global__ __launch_bounds__(kGroupThreads) void kg_stages(const GStage* __restrict__ st, int nst,
                                                         const int* __restrict__ tstart) {
  __shared__ StageLds sm;
  // item and stage indices are uniform over the workgroup
  const int t = blockIdx.x;
  const int s = __builtin_amdgcn_readfirstlane(find_slot(tstart, nst, t));
  run_stage(st[s], __builtin_amdgcn_readfirstlane(t - tstart[s]), sm);
}

}  // namespace

void group_stages(const GStage* st, int nst, const int* tstart, int total, hipStream_t s) {
  if (total <= 0) return;
  MLMC_LAUNCH(kg_stages, dim3((unsigned)total), dim3(kGroupThreads), 0, s, st, nst, tstart);
}

void group_update_apply(const GTask* tasks, const int* tab, int blocks, int old_sel, int new_sel,
                        hipStream_t s) {
  MLMC_LAUNCH(kg_update_apply, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab, old_sel,
              new_sel);
}
void group_finish_alpha(const GTask* tasks, const int* tab, int blocks, hipStream_t s) {
  MLMC_LAUNCH(kg_finish_alpha, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab);
}
void group_cg_xr(const GTask* tasks, const int* tab, int blocks, int new_sel, hipStream_t s) {
  MLMC_LAUNCH(kg_cg_xr, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab, new_sel);
}
void group_finish(const GTask* tasks, const int* tab, int blocks, int which, hipStream_t s) {
  MLMC_LAUNCH(kg_finish, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab, which);
}
void group_finish_beta(const GTask* tasks, const int* tab, int blocks, hipStream_t s) {
  MLMC_LAUNCH(kg_finish_beta, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab);
}
void group_refine_due(const GTask* tasks, const int* tab, int blocks, hipStream_t s) {
  MLMC_LAUNCH(kg_refine_due, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab);
}
void group_ir_fold(const GTask* tasks, const int* tab, int blocks, hipStream_t s) {
  MLMC_LAUNCH(kg_ir_fold, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab);
}
void group_ir_residual(const GTask* tasks, const int* tab, int blocks, hipStream_t s) {
  MLMC_LAUNCH(kg_ir_residual, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab);
}
void group_refine_rules(const GTask* tasks, const int* tab, int blocks, double factor,
                        hipStream_t s) {
  MLMC_LAUNCH(kg_refine_rules, dim3((unsigned)blocks), dim3(kThreads), 0, s, tasks, tab,
              factor);
}

}  // namespace mlmc
