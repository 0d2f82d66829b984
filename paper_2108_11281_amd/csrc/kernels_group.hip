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

// LDS of one 16 x 16 coarsest-solve tile (its partial tiles)
constexpr int kDenseTile = body::kDenseParts * 4 * 64;

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
// One launch runs stages of one kind and form (one kernel instance per kind,
// rows per wave and sweep form, so that each has the registers of its own
// body): item i of the concatenated stages per workgroup.
template <int KIND, int RPW, int HX, int HE, int F>
__global__ __launch_bounds__(kGroupThreads) void kg_stage(const GStage* __restrict__ st, int nst,
                                                        const int* __restrict__ tstart) {
  constexpr int kLds = KIND == kGsMarch ? vcb::vc_march_lds<float, kGroupMarchCols, RPW>()
                                        : (KIND == kGsDense ? 2 * kDenseTile : 64);
  __shared__ __attribute__((aligned(16))) float lds[kLds];
  // item and stage indices are uniform over the workgroup
  const int t = blockIdx.x;
  const int s = __builtin_amdgcn_readfirstlane(find_slot(tstart, nst, t));
  const GStage& g = st[s];
  const int item = __builtin_amdgcn_readfirstlane(t - tstart[s]);
  const int tid = threadIdx.x;
  if constexpr (KIND == kGsMarch) {
    const int bx = item % g.gx, rest = item / g.gx;
    const int by = rest % g.gy, bz = rest / g.gy;
    vcb::vc_march<float, kGroupMarchCols, RPW, HX != 0, HE != 0, F>(
        g.in, g.b, g.out, g.ec, g.ws, g.kl, g.dg, g.N, g.sz, g.nb, g.act, nullptr, bx, by, bz,
        lds);
  } else if constexpr (KIND == kGsResRestrict) {
    vcb::vc_res_restrict<float, kGroupRrCols, kGroupThreads>(g.b, g.in, g.out, g.kl, g.dg, g.N,
                                                             g.nb, g.act, nullptr, item % g.gx,
                                                             item / g.gx, tid);
  } else if constexpr (KIND == kGsDense) {
    // two 256-thread blocks per item
    const int half = tid >> 8;
    const int vb = 2 * item + half;
    const bool live = vb < g.gx * g.gy;
    body::dense_apply_mfma<float>(g.At, g.in, g.out, (int)g.n, g.ld, g.nb, g.act, vb % g.gx,
                                  vb / g.gx, live, lds + half * kDenseTile, tid & 255);
  } else if constexpr (KIND == kGsDot) {
    const int half = tid >> 8;
    const int vb = 2 * item + half;
    const int k = vb / g.nblk;
    const bool live = vb < g.nblk * g.nb && g.act[k];
    body::dot(g.b, g.in, g.n, g.nblk, vb % g.nblk, live ? k : 0, live, g.partials,
              reinterpret_cast<double*>(lds) + 16 * half, tid & 255);
  } else {  // kGsCopy
    const int k = item / g.gx;
    const int64_t i = (int64_t)(item % g.gx) * kGroupThreads + tid;
    if (g.act[k] && i < g.n) g.out[(int64_t)k * g.n + i] = g.in[(int64_t)k * g.n + i];
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// Persistent V-cycle: one workgroup per (problem, column pair) runs every
// stage of that problem's V-cycle for its two columns, stage after stage,
// with nothing shared between workgroups (a stage's items of other column
// pairs belong to other workgroups, and no item reads another pair's columns),
// so stages are ordered by the workgroup's own barriers.  Unit u: stages
// [units[3u], units[3u+1]) of st, column pair units[3u+2].
// ---------------------------------------------------------------------------
template <int RPW, int HX, int HE, int F>
__device__ __forceinline__ void unit_march(const GStage& g, int pair, float* lds) {
  for (int bz = 0; bz < g.gz; ++bz)
    for (int bx = 0; bx < g.gx; ++bx) {
      vcb::vc_march<float, kGroupMarchCols, RPW, HX != 0, HE != 0, F>(
          g.in, g.b, g.out, g.ec, g.ws, g.kl, g.dg, g.N, g.sz, g.nb, g.act, nullptr, bx, pair,
          bz, lds);
      __syncthreads();  // the next tile reuses the LDS rows
    }
}

template <int RPW>
__device__ __forceinline__ void unit_march_rpw(const GStage& g, int pair, float* lds) {
  if (!g.hx) unit_march<RPW, 0, 0, 0>(g, pair, lds);
  else if (!g.f) unit_march<RPW, 1, 0, 0>(g, pair, lds);
  else if (g.he) unit_march<RPW, 1, 1, 1>(g, pair, lds);
  else unit_march<RPW, 1, 0, 1>(g, pair, lds);
}

__global__ __launch_bounds__(kGroupThreads) void kg_vcycle_units(const GStage* __restrict__ st,
                                                               const int* __restrict__ units) {
  constexpr int kMarchLds = vcb::vc_march_lds<float, kGroupMarchCols, 1>();
  __shared__ __attribute__((aligned(16)))
  float lds[kMarchLds > 2 * kDenseTile ? kMarchLds : 2 * kDenseTile];
  const int u = blockIdx.x;
  const int s0 = units[3 * u], s1 = units[3 * u + 1], pair = units[3 * u + 2];
  const int tid = threadIdx.x;
  const int c0 = pair * kGroupMarchCols;
  for (int s = s0; s < s1; ++s) {
    const GStage& g = st[s];
    switch (g.kind) {
      case kGsMarch:
        if (g.rpw == 1) unit_march_rpw<1>(g, pair, lds);
        else if (g.rpw == 2) unit_march_rpw<2>(g, pair, lds);
        else unit_march_rpw<4>(g, pair, lds);
        break;
      case kGsResRestrict:
        // the pair is one column group of the restriction (kGroupRrCols == 2)
        for (int bx = 0; bx < g.gx; ++bx)
          vcb::vc_res_restrict<float, kGroupRrCols, kGroupThreads>(
              g.b, g.in, g.out, g.kl, g.dg, g.N, g.nb, g.act, nullptr, bx, pair, tid);
        break;
      case kGsDense: {
        // 16-column tile of the pair; only the pair's columns are computed
        // and stored (the others belong to other workgroups)
        const int by = c0 / 16;
        const int half = tid >> 8;
        for (int bx0 = 0; bx0 < g.gx; bx0 += 2) {
          const int bx = bx0 + half;
          body::dense_apply_mfma<float>(g.At, g.in, g.out, (int)g.n, g.ld, g.nb, g.act,
                                        bx < g.gx ? bx : 0, by, bx < g.gx,
                                        lds + half * kDenseTile, tid & 255, c0,
                                        c0 + kGroupMarchCols);
          __syncthreads();
        }
        break;
      }
      case kGsDot: {
        const int half = tid >> 8;
        for (int k = c0; k < c0 + kGroupMarchCols && k < g.nb; ++k) {
          const bool on = g.act[k] != 0;
          for (int b0 = 0; b0 < g.nblk; b0 += 2) {
            const int bx = b0 + half;
            const bool live = on && bx < g.nblk;
            body::dot(g.b, g.in, g.n, g.nblk, live ? bx : 0, k, live, g.partials,
                      reinterpret_cast<double*>(lds) + 16 * half, tid & 255);
          }
        }
        break;
      }
      default:  // kGsCopy
        for (int k = c0; k < c0 + kGroupMarchCols && k < g.nb; ++k) {
          if (!g.act[k]) continue;
          for (int64_t i = tid; i < g.n; i += kGroupThreads)
            g.out[(int64_t)k * g.n + i] = g.in[(int64_t)k * g.n + i];
        }
        break;
    }
    // the next stage reads what this one wrote (other waves' stores included)
    __syncthreads();
  }
}

int group_stage_key(const GStage& g) {
  if (g.kind != kGsMarch) return g.kind;
  const int r = g.rpw == 1 ? 0 : (g.rpw == 2 ? 1 : 2);
  const int v = !g.hx ? 0 : (!g.f ? 1 : (g.he ? 2 : 3));
  return 16 + 4 * r + v;
}

void group_stages(const GStage* st, int nst, const int* tstart, int total, int key,
                  hipStream_t s) {
  if (total <= 0) return;
  const dim3 grid((unsigned)total), blk(kGroupThreads);
#define KG(KIND, RPW, HX, HE, F) \
  MLMC_LAUNCH((kg_stage<KIND, RPW, HX, HE, F>), grid, blk, 0, s, st, nst, tstart)
#define KG_MARCH(R, RPW)                      \
  case 16 + 4 * R + 0: KG(kGsMarch, RPW, 0, 0, 0); break; \
  case 16 + 4 * R + 1: KG(kGsMarch, RPW, 1, 0, 0); break; \
  case 16 + 4 * R + 2: KG(kGsMarch, RPW, 1, 1, 1); break; \
  case 16 + 4 * R + 3: KG(kGsMarch, RPW, 1, 0, 1); break;
  switch (key) {
    case kGsResRestrict: KG(kGsResRestrict, 1, 0, 0, 0); break;
    case kGsDense: KG(kGsDense, 1, 0, 0, 0); break;
    case kGsDot: KG(kGsDot, 1, 0, 0, 0); break;
    case kGsCopy: KG(kGsCopy, 1, 0, 0, 0); break;
    KG_MARCH(0, 1)
    KG_MARCH(1, 2)
    KG_MARCH(2, 4)
    default: throw Error(MLMC_EINVAL, "grouped V-cycle: unknown stage kernel");
  }
#undef KG_MARCH
#undef KG
}

void group_vcycle_units(const GStage* st, const int* units, int nunits, hipStream_t s) {
  if (nunits <= 0) return;
  MLMC_LAUNCH(kg_vcycle_units, dim3((unsigned)nunits), dim3(kGroupThreads), 0, s, st, units);
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
