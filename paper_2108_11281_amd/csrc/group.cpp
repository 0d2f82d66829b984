// Level-difference samples of several 3D diffusion problems at once (a batch
// of uneven problems): every problem's two solves per sample batch run in
// lockstep on one stream.  Each step of the refined CG is one launch over all
// problems still iterating, and each application of the preconditioner runs
// the stages of every problem's V-cycle position by position, one launch of
// the stage kernel per position over the (problem, level, stage, tile) items
// of all problems at that position.  The host keeps each
// problem's decisions (refinement due, columns converged) separately, so every
// problem goes through the same operations as its own solve: the samples are
// identical to mlmc_sample_level's.
#include <algorithm>
#include <cstring>

#include "context.h"
#include "group.h"

namespace mlmc {

class GroupSolver {
 public:
  GroupSolver(std::vector<Context*> cs, int mode) : cs_(std::move(cs)), mode_(mode) {}
  ~GroupSolver() { release(); }
  void batch_sample(int level, const uint64_t* seeds, int64_t first, int64_t count,
                    double* out, int* status);

 private:
  struct Task {
    Context* c;
    int p;           // problem index
    int l;           // level solved (1-based)
    const double* b;
    double* y;
    int nb;
    c64* err;
    std::vector<GStage> seq;  // its V-cycle's stages
  };
  // launch tables of a set of tasks on the device
  struct Tab {
    int* dev = nullptr;
    int* host = nullptr;  // pinned staging
    int blocks[4] = {0, 0, 0, 0};
    int count = 0;
  };
  void check_eligible(int level);
  void alloc(int ntasks, int max_stages);
  void release();
  void upload_tab(Tab& T, const std::vector<int>& members);
  void build_stages(Task& t, int l, const float* b, float* x, const c64* rz_dummy, bool top);
  void upload_stages(const std::vector<int>& members);
  void vcycle(const Tab& A);
  void solve(std::vector<Task>& tasks);
  void prologue(Task& t);
  void epilogue(Task& t);

  std::vector<Context*> cs_;
  int mode_;  // 1: persistent V-cycle (a workgroup per problem and column pair), 2: per position
  int* dunits_ = nullptr;  // persistent form: (first stage, end stage, column pair) per unit
  int* hunits_ = nullptr;
  int nunits_ = 0;
  hipStream_t s_ = nullptr;
  std::vector<hipStream_t> saved_;
  GTask* dtasks_ = nullptr;
  GTask* htasks_ = nullptr;  // pinned
  int* dints_ = nullptr;     // counts (2 per task)
  int* hints_ = nullptr;     // pinned copy
  Tab A_, R_;
  GStage* dst_ = nullptr;    // stages, grouped by position in the V-cycle
  GStage* hst_ = nullptr;
  int* dts_ = nullptr;       // item prefix sums
  int* hts_ = nullptr;
  int nst_ = 0, cap_st_ = 0, ntasks_cap_ = 0;
  // launches of a V-cycle: per position, one per stage kernel key; stages
  // [s0, s1) of hst_, their prefix array at hts_[tbeg]
  struct Launch {
    int s0, s1, key, tbeg, total;
  };
  std::vector<Launch> launches_;
  // measurement (the first context's sweep timer on): stage-kernel launches
  // with their events and algorithmic bytes (active columns known on the host:
  // columns change state only at refinements)
  struct Timed {
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Timed> timed_;
  std::vector<int> active_cols_;  // per task of the current solve
  std::vector<int> stage_cols_;   // active columns of each uploaded stage's task
  int64_t launch_seen_ = 0;
  void collect();
  static double stage_bytes(const GStage& g);
  std::vector<Task>* cur_ = nullptr;
};

namespace {
int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }
}  // namespace

void GroupSolver::check_eligible(int level) {
  const Context* c0 = cs_[0];
  for (Context* c : cs_) {
    MLMC_REQUIRE(c->varcoef_, MLMC_EUNSUPPORTED, "grouped solves need VARCOEF3D problems");
    MLMC_REQUIRE(c->opt_.precision == MLMC_FP32_IR64, MLMC_EUNSUPPORTED,
                 "grouped solves need MLMC_FP32_IR64");
    MLMC_REQUIRE(c->opt_.narrow_fp64 == 0 && c->top_cycles_ == 1, MLMC_EUNSUPPORTED,
                 "grouped solves need narrow_fp64 = 0 and one coarse-grid cycle");
    MLMC_REQUIRE(c->opt_.nu_pre >= 1 && c->opt_.nu_post >= 1, MLMC_EUNSUPPORTED,
                 "grouped solves need pre- and post-smoothing");
    MLMC_REQUIRE(c->device_ == c0->device_, MLMC_EINVAL, "grouped problems on different GPUs");
    MLMC_REQUIRE(c->nb_ == c0->nb_ &&
                     c->opt_.max_iter * c->opt_.max_refine ==
                         c0->opt_.max_iter * c0->opt_.max_refine,
                 MLMC_EUNSUPPORTED, "grouped problems need equal nb and iteration limits");
    MLMC_REQUIRE(level >= 1 && level < c->L_, MLMC_EINVAL, "sample level must be in [1, L-1]");
    for (int l = level; l < c->Ls_; ++l)
      MLMC_REQUIRE(c->lv_[l - 1].mcols > 0, MLMC_EUNSUPPORTED,
                   "grouped solves need the fused 3D sweep on every smoothed level");
  }
}

void GroupSolver::alloc(int ntasks, int max_stages) {
  Context* c0 = cs_[0];
  ntasks_cap_ = ntasks;
  cap_st_ = max_stages;
  dtasks_ = c0->dalloc_n<GTask>(ntasks);
  MLMC_HIP(hipHostMalloc((void**)&htasks_, sizeof(GTask) * ntasks));
  dints_ = c0->dalloc_n<int>(2 * ntasks);
  MLMC_HIP(hipHostMalloc((void**)&hints_, sizeof(int) * 2 * ntasks));
  for (Tab* T : {&A_, &R_}) {
    T->dev = c0->dalloc_n<int>(group_table_ints(ntasks));
    MLMC_HIP(hipHostMalloc((void**)&T->host, sizeof(int) * group_table_ints(ntasks)));
  }
  const int max_units = ntasks * ((c0->nb_ + kGroupMarchCols - 1) / kGroupMarchCols);
  dunits_ = c0->dalloc_n<int>(3 * max_units);
  MLMC_HIP(hipHostMalloc((void**)&hunits_, sizeof(int) * 3 * max_units));
  dst_ = c0->dalloc_n<GStage>(max_stages);
  MLMC_HIP(hipHostMalloc((void**)&hst_, sizeof(GStage) * max_stages));
  // prefix arrays: one per launch, together at most 2 max_stages entries
  dts_ = c0->dalloc_n<int>(2 * max_stages + 2);
  MLMC_HIP(hipHostMalloc((void**)&hts_, sizeof(int) * (2 * max_stages + 2)));
}

void GroupSolver::release() {
  if (!cs_.empty() && s_) (void)hipStreamSynchronize(s_);
  Context* c0 = cs_.empty() ? nullptr : cs_[0];
  auto hf = [](void* p) {
    if (p) (void)hipHostFree(p);
  };
  if (c0) {
    for (void* p : {(void*)dtasks_, (void*)dints_, (void*)A_.dev, (void*)R_.dev, (void*)dst_,
                    (void*)dts_, (void*)dunits_})
      if (p) c0->dfree(p);
  }
  hf(htasks_);
  hf(hints_);
  hf(A_.host);
  hf(R_.host);
  hf(hst_);
  hf(hts_);
  hf(hunits_);
  dunits_ = nullptr;
  hunits_ = nullptr;
  dtasks_ = nullptr;
  dints_ = nullptr;
  A_.dev = R_.dev = nullptr;
  dst_ = nullptr;
  dts_ = nullptr;
  htasks_ = nullptr;
  hints_ = nullptr;
  A_.host = R_.host = nullptr;
  hst_ = nullptr;
  hts_ = nullptr;
  // the contexts' own streams back
  for (size_t i = 0; i < saved_.size(); ++i) cs_[i]->s_ = saved_[i];
  saved_.clear();
}

// tables of `members` (indices into the current task list): called only when
// the stream holds no launch that reads T (after a synchronisation)
void GroupSolver::upload_tab(Tab& T, const std::vector<int>& members) {
  const int t = (int)members.size();
  int* h = T.host;
  h[0] = t;
  for (int i = 0; i < t; ++i) h[1 + i] = members[i];
  for (int sh = 0; sh < 4; ++sh) {
    int* start = h + 1 + t + sh * (t + 1);
    int acc = 0;
    for (int i = 0; i < t; ++i) {
      start[i] = acc;
      const GTask& g = htasks_[members[i]];
      int blocks = 1;
      if (sh == kShStencil) blocks = g.ntiles * ceil_div(g.nb, kGroupStencilCols);
      else if (sh == kShReduce) blocks = g.nblk * g.nb;
      else if (sh == kShColumn) blocks = g.nb;
      acc += blocks;
    }
    start[t] = acc;
    T.blocks[sh] = acc;
  }
  T.count = t;
  MLMC_HIP(hipMemcpyAsync(T.dev, h, sizeof(int) * group_table_ints(t), hipMemcpyHostToDevice,
                          s_));
}

// the stages of task t's V-cycle on levels l..L_s in the order of vcycle_vc
// (fused-sweep branch): pre-sweeps, residual restriction, the coarser levels,
// post-sweeps (the first with the folded correction), the final copy; at the
// top level also the partial sums of conj(b)^T x
void GroupSolver::build_stages(Task& t, int l, const float* b, float* x, const c64* rz,
                               bool top) {
  Context* c = t.c;
  Work<float>& w = c->w32_;
  const Level& L = c->lv_[l - 1];
  const int nb = t.nb;
  const int* act = c->act_outer_;
  const int64_t n = L.n;
  auto base = [&](int kind) {
    GStage g;
    std::memset(&g, 0, sizeof(g));
    g.kind = kind;
    g.nb = nb;
    g.N = L.side;
    g.n = n;
    g.act = act;
    return g;
  };
  if (l == c->Ls_) {
    GStage g = base(kGsDense);
    g.At = w.ainvT;
    g.ld = w.ld;
    g.in = b;
    g.out = x;
    g.gx = w.ld / 16;
    g.gy = ceil_div(nb, 16);
    g.tiles = ceil_div((int64_t)g.gx * g.gy, 2);
    t.seq.push_back(g);
  } else {
    const int N = L.side;
    const float* kf = L.kl32;
    const float* dg = L.dg32;
    const int rpw = N <= 32 ? 4 : (N <= 64 ? 2 : 1);
    const int TY = 8 * rpw - 2;
    const int SZ = N >= 32 ? 16 : N;
    const float ws = (float)(c->omega_ * 0.35355339059327373);
    auto march = [&](const float* in, float* out, const float* ec, int f) {
      GStage g = base(kGsMarch);
      g.hx = in != nullptr;
      g.he = ec != nullptr;
      g.f = f;
      g.rpw = rpw;
      g.sz = SZ;
      g.ws = ws;
      g.in = in ? in : b;  // placeholders are never read
      g.b = b;
      g.ec = ec ? ec : b;
      g.kl = kf;
      g.dg = dg;
      g.out = out;
      g.gx = ceil_div(N, TY);
      g.gy = ceil_div(nb, kGroupMarchCols);
      g.gz = ceil_div(N, SZ);
      g.tiles = g.gx * g.gy * g.gz;
      t.seq.push_back(g);
    };
    float* tmp = w.vt[l - 1];
    const int pre = c->opt_.nu_pre, post = c->opt_.nu_post;
    const float* u = nullptr;
    for (int i = 0; i < pre; ++i) {
      float* out = (i % 2 == 0) ? tmp : x;
      march(u, out, nullptr, 0);
      u = out;
    }
    float* bc = w.vb[l];
    float* ec = w.vx[l];
    {
      GStage g = base(kGsResRestrict);
      g.b = b;
      g.in = u;
      g.out = bc;
      g.kl = kf;
      g.dg = dg;
      const int Nc = N / 2;
      g.gx = ceil_div((int64_t)Nc * Nc * Nc, kGroupThreads);
      g.gy = ceil_div(nb, kGroupRrCols);
      g.tiles = g.gx * g.gy;
      t.seq.push_back(g);
    }
    build_stages(t, l + 1, bc, ec, nullptr, false);
    for (int i = 0; i < post; ++i) {
      const int left = post - 1 - i;
      float* out = (left % 2 == 0) ? x : tmp;
      if (out == u) out = (out == x) ? tmp : x;  // never sweep in place
      march(u, out, i == 0 ? ec : nullptr, 1);
      u = out;
    }
    if (u != x) {
      GStage g = base(kGsCopy);
      g.in = u;
      g.out = x;
      g.gx = ceil_div(n, kGroupThreads);
      g.tiles = g.gx * nb;
      t.seq.push_back(g);
    }
  }
  if (top) {
    GStage g = base(kGsDot);
    g.b = b;
    g.in = x;
    g.partials = c->partials_;
    g.nblk = reduce_blocks(n);
    g.tiles = ceil_div((int64_t)g.nblk * nb, 2);
    t.seq.push_back(g);
  }
  (void)rz;
}

// stage arrays of the members' V-cycles: position by position (the stages of
// one position are independent: they belong to different problems), and
// within a position grouped by stage kernel, one launch per group with its own
// prefix array of items
void GroupSolver::upload_stages(const std::vector<int>& members) {
  std::vector<Task>& tasks = *cur_;
  if (mode_ == 1) {
    // every member's stages in V-cycle order, one unit per column pair, the
    // units of larger problems first (they take longest)
    std::vector<int> order(members);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      return htasks_[a].n > htasks_[b].n;
    });
    nst_ = 0;
    nunits_ = 0;
    stage_cols_.assign((size_t)cap_st_, 0);
    for (int m : order) {
      const Task& t = tasks[m];
      const int s0 = nst_;
      for (const GStage& g : t.seq) {
        MLMC_REQUIRE(nst_ < cap_st_, MLMC_EINVAL, "grouped V-cycle: too many stages");
        stage_cols_[(size_t)nst_] = active_cols_[(size_t)m];
        hst_[nst_++] = g;
      }
      for (int p = 0; p * kGroupMarchCols < t.nb; ++p) {
        hunits_[3 * nunits_] = s0;
        hunits_[3 * nunits_ + 1] = nst_;
        hunits_[3 * nunits_ + 2] = p;
        ++nunits_;
      }
    }
    MLMC_HIP(hipMemcpyAsync(dst_, hst_, sizeof(GStage) * nst_, hipMemcpyHostToDevice, s_));
    MLMC_HIP(hipMemcpyAsync(dunits_, hunits_, sizeof(int) * 3 * nunits_, hipMemcpyHostToDevice,
                            s_));
    return;
  }
  size_t maxlen = 0;
  for (int m : members) maxlen = std::max(maxlen, tasks[m].seq.size());
  nst_ = 0;
  launches_.clear();
  stage_cols_.assign((size_t)cap_st_, 0);
  int off = 0;
  for (size_t d = 0; d < maxlen; ++d) {
    std::vector<std::pair<int, int>> pos;  // (key, member)
    for (int m : members)
      if (d < tasks[m].seq.size()) pos.push_back({group_stage_key(tasks[m].seq[d]), m});
    std::stable_sort(pos.begin(), pos.end(),
                     [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
                       return a.first < b.first;
                     });
    for (size_t i = 0; i < pos.size();) {
      Launch L{nst_, nst_, pos[i].first, off, 0};
      int acc = 0;
      for (; i < pos.size() && pos[i].first == L.key; ++i) {
        MLMC_REQUIRE(nst_ < cap_st_, MLMC_EINVAL, "grouped V-cycle: too many stages");
        const int m = pos[i].second;
        stage_cols_[(size_t)nst_] = active_cols_[(size_t)m];
        hst_[nst_] = tasks[m].seq[d];
        hts_[off++] = acc;
        acc += hst_[nst_].tiles;
        ++nst_;
      }
      hts_[off++] = acc;
      L.s1 = nst_;
      L.total = acc;
      launches_.push_back(L);
    }
  }
  MLMC_HIP(hipMemcpyAsync(dst_, hst_, sizeof(GStage) * nst_, hipMemcpyHostToDevice, s_));
  MLMC_HIP(hipMemcpyAsync(dts_, hts_, sizeof(int) * off, hipMemcpyHostToDevice, s_));
}

// algorithmic bytes per active column of a stage (FP32; couplings and
// diagonal shared by the nb columns; the inverse read once per launch is not
// counted)
double GroupSolver::stage_bytes(const GStage& g) {
  const double en = 4.0 * (double)g.n, nb = (double)g.nb;
  switch (g.kind) {
    case kGsMarch: return en * ((g.hx ? 3.0 : 2.0) + (g.he ? 0.125 : 0.0) + 4.0 / nb);
    case kGsResRestrict: return en * (2.0 + 0.125 + 4.0 / nb);
    default: return 2.0 * en;  // dense (B in, Z out), dot (b, x in), copy
  }
}

void GroupSolver::vcycle(const Tab& A) {
  (void)A;
  Context* c0 = cs_[0];
  const bool timing = c0->timing_ && (c0->timing_mask_ & (1u << Context::kTimGs));
  if (mode_ == 1) {
    const bool sample =
        timing && (c0->timing_stride_ <= 1 ||
                   mix64((uint64_t)launch_seen_++) % (uint64_t)c0->timing_stride_ == 0);
    if (!sample) {
      group_vcycle_units(dst_, dunits_, nunits_, s_);
      return;
    }
    double bytes = 0.0;
    for (int s = 0; s < nst_; ++s) bytes += stage_bytes(hst_[s]) * stage_cols_[s];
    LaunchEvents ev;
    ev.start = c0->event();
    ev.stop = c0->event();
    timing_events() = &ev;
    group_vcycle_units(dst_, dunits_, nunits_, s_);
    timing_events() = nullptr;
    timed_.push_back({ev.start, ev.stop, bytes});
    return;
  }
  for (const Launch& L : launches_) {
    const bool sample =
        timing && (c0->timing_stride_ <= 1 ||
                   mix64((uint64_t)launch_seen_++) % (uint64_t)c0->timing_stride_ == 0);
    if (!sample) {
      group_stages(dst_ + L.s0, L.s1 - L.s0, dts_ + L.tbeg, L.total, L.key, s_);
      continue;
    }
    double bytes = 0.0;
    for (int s = L.s0; s < L.s1; ++s) bytes += stage_bytes(hst_[s]) * stage_cols_[s];
    LaunchEvents ev;
    ev.start = c0->event();
    ev.stop = c0->event();
    timing_events() = &ev;
    group_stages(dst_ + L.s0, L.s1 - L.s0, dts_ + L.tbeg, L.total, L.key, s_);
    timing_events() = nullptr;
    timed_.push_back({ev.start, ev.stop, bytes});
  }
}

// timed launches into the first context's sweep timer (FP32 slot, all levels)
void GroupSolver::collect() {
  if (timed_.empty()) return;
  MLMC_HIP(hipStreamSynchronize(s_));
  Context* c0 = cs_[0];
  Context::TimerStat& t = c0->tstat_[2 * Context::kTimGs];
  for (const Timed& x : timed_) {
    float ms = 0.f;
    MLMC_HIP(hipEventElapsedTime(&ms, x.a, x.b));
    t.launches += 1;
    t.ms += ms;
    t.bytes += x.bytes;
    c0->ev_pool_.push_back(x.a);
    c0->ev_pool_.push_back(x.b);
  }
  timed_.clear();
}

// solve(): the FP64 |b|^2, flags and stated errors; then pcg_refined's start
void GroupSolver::prologue(Task& t) {
  Context* c = t.c;
  const int64_t n = c->lv_[t.l - 1].n;
  const int nb = t.nb;
  vec_dot_partials<double>(t.b, t.b, n, nb, nullptr, c->partials_, s_);
  finish_sums(c->partials_, reduce_blocks(n), nb, c->scal_[Context::kBb], s_);
  set_all_active(c->act_outer_, nb, s_);
  vec_zero<c64>(t.err, 1, nb, nullptr, s_);
  vec_copy<c64>(c->scal_[Context::kBb], c->scal_[Context::kRres], 1, nb, nullptr, s_);
  vec_zero<double>(t.y, n, nb, nullptr, s_);
  vec_zero<float>(c->d32_, n, nb, nullptr, s_);
  vec_convert<float, double>(t.b, c->w32_.r, n, nb, nullptr, s_);
}

// solve()'s final check: the FP64 relative residual of every column
void GroupSolver::epilogue(Task& t) {
  Context* c = t.c;
  const int nb = t.nb;
  MLMC_HIP(hipMemcpyAsync(c->host_c64_, c->scal_[Context::kRres], sizeof(c64) * nb,
                          hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipMemcpyAsync(c->host_c64_ + nb, c->scal_[Context::kBb], sizeof(c64) * nb,
                          hipMemcpyDeviceToHost, s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  const double tol = c->opt_.solve_tol;
  c->col_ok_.assign((size_t)nb, 1);
  for (int k = 0; k < nb; ++k) {
    const double bn = c->host_c64_[nb + k].re;
    const double rel =
        bn > 0 ? std::sqrt(c->host_c64_[k].re / bn) : std::sqrt(c->host_c64_[k].re);
    if (!(rel <= tol)) c->col_ok_[(size_t)k] = 0;
  }
}

// pcg_refined of every task in lockstep (the same iteration and refinement
// rules, decided per task)
void GroupSolver::solve(std::vector<Task>& tasks) {
  cur_ = &tasks;
  const int nt = (int)tasks.size();
  // tasks on the coarsest solver level: their own direct solve
  std::vector<int> act_set;
  for (int i = 0; i < nt; ++i) {
    Task& t = tasks[i];
    if (t.l == t.c->Ls_) {
      bool ok = true;
      t.c->solve(t.l, t.b, t.y, t.nb, t.err, nullptr, &ok);
      continue;
    }
    act_set.push_back(i);
  }
  if (act_set.empty()) return;
  for (int i : act_set) {
    Task& t = tasks[i];
    Context* c = t.c;
    const Level& L = c->lv_[t.l - 1];
    GTask& g = htasks_[i];
    std::memset(&g, 0, sizeof(g));
    g.N = L.side;
    g.nb = t.nb;
    g.n = L.n;
    g.ntiles = varcoef_blocks(L.side);
    g.nblk = reduce_blocks(L.n);
    g.kl32 = L.kl32;
    g.dg32 = L.dg32;
    g.kl64 = L.kl64;
    g.dg64 = L.dg64;
    g.x32 = c->d32_;
    g.r = c->w32_.r;
    g.z = c->w32_.z;
    g.P1 = c->w32_.p;
    g.P2 = c->w32_.p2;
    g.q = c->w32_.q;
    g.b = t.b;
    g.y = t.y;
    g.rz = c->scal_[Context::kRz];
    g.tmp = c->scal_[Context::kTmp];
    g.alpha = c->scal_[Context::kAlpha];
    g.beta = c->scal_[Context::kBeta];
    g.bb = c->scal_[Context::kBb];
    g.bd = c->scal_[Context::kBd];
    g.rr_upd = c->scal_[Context::kRres];
    g.rr_new = c->scal_[Context::kRres2];
    g.err = t.err;
    g.act = c->act_outer_;
    g.partials = c->partials_;
    g.count = dints_ + 2 * i;
    g.delta2 = c->opt_.inner_tol * c->opt_.inner_tol;
    g.tol2 = c->opt_.solve_tol * c->opt_.solve_tol;
    t.seq.clear();
    build_stages(t, t.l, c->w32_.r, c->w32_.z, c->partials_, true);
  }
  MLMC_HIP(hipMemcpyAsync(dtasks_, htasks_, sizeof(GTask) * nt, hipMemcpyHostToDevice, s_));
  active_cols_.assign((size_t)nt, 0);
  for (int i : act_set) active_cols_[(size_t)i] = tasks[i].nb;
  for (int i : act_set) prologue(tasks[i]);
  upload_tab(A_, act_set);
  upload_stages(act_set);
  // z = M r, rz, beta = 0
  vcycle(A_);
  group_finish(dtasks_, A_.dev, A_.blocks[kShColumn], 1, s_);
  for (int i : act_set) vec_zero<c64>(tasks[i].c->scal_[Context::kBeta], 1, tasks[i].nb, nullptr, s_);
  const int max_it = tasks[act_set[0]].c->opt_.max_iter * tasks[act_set[0]].c->opt_.max_refine;
  std::vector<int> cur = act_set;
  auto core = [&](int old_sel, int new_sel, bool checked) {
    group_update_apply(dtasks_, A_.dev, A_.blocks[kShStencil], old_sel, new_sel, s_);
    group_finish_alpha(dtasks_, A_.dev, A_.blocks[kShColumn], s_);
    group_cg_xr(dtasks_, A_.dev, A_.blocks[kShReduce], new_sel, s_);
    if (checked) group_finish(dtasks_, A_.dev, A_.blocks[kShColumn], 0, s_);
    for (int i : cur) tasks[i].c->counters[0] += 1;
  };
  auto tail = [&] {
    vcycle(A_);
    group_finish_beta(dtasks_, A_.dev, A_.blocks[kShColumn], s_);
  };
  auto due = [&] { group_refine_due(dtasks_, A_.dev, A_.blocks[kShTask], s_); };
  // after due(): refine the tasks that need it; true when every task is done
  auto refine = [&](bool force) {
    MLMC_HIP(hipMemcpyAsync(hints_, dints_, sizeof(int) * 2 * ntasks_cap_, hipMemcpyDeviceToHost,
                            s_));
    MLMC_HIP(hipStreamSynchronize(s_));
    std::vector<int> sub;
    for (int i : cur)
      if (force || hints_[2 * i] > 0) sub.push_back(i);
    if (sub.empty()) return false;
    upload_tab(R_, sub);
    group_ir_fold(dtasks_, R_.dev, R_.blocks[kShReduce], s_);
    group_finish(dtasks_, R_.dev, R_.blocks[kShColumn], 2, s_);
    group_ir_residual(dtasks_, R_.dev, R_.blocks[kShStencil], s_);
    group_finish(dtasks_, R_.dev, R_.blocks[kShColumn], 3, s_);
    group_refine_rules(dtasks_, R_.dev, R_.blocks[kShTask], 100.0, s_);
    MLMC_HIP(hipMemcpyAsync(hints_, dints_, sizeof(int) * 2 * ntasks_cap_, hipMemcpyDeviceToHost,
                            s_));
    MLMC_HIP(hipStreamSynchronize(s_));
    std::vector<int> keep;
    bool cols_changed = false;
    for (int i : cur) {
      const bool refined = std::find(sub.begin(), sub.end(), i) != sub.end();
      if (refined) {
        tasks[i].c->counters[1] += 1;
        cols_changed = cols_changed || active_cols_[(size_t)i] != hints_[2 * i + 1];
        active_cols_[(size_t)i] = hints_[2 * i + 1];
      }
      if (refined && hints_[2 * i + 1] == 0) continue;  // every column converged
      keep.push_back(i);
    }
    if (keep.size() != cur.size()) {
      cur = keep;
      if (cur.empty()) return true;
      upload_tab(A_, cur);
      upload_stages(cur);
    } else if (cols_changed) {
      upload_stages(cur);  // the measurement's column counts only
    }
    return false;
  };
  int it = 1;
  core(0, 1, it == max_it);
  if (it == max_it) {
    due();
    refine(true);
    return;
  }
  tail();
  core(1, 2, true);
  it = 2;
  due();
  if (refine(it == max_it)) return;
  while (it < max_it && !cur.empty()) {
    if (it + 2 <= max_it) {
      tail();
      core(2, 1, false);
      tail();
      core(1, 2, true);
      due();
      it += 2;
      if (refine(it == max_it)) return;
    } else {
      tail();
      core(2, 1, true);
      it += 1;
      due();
      refine(true);
      return;
    }
  }
}

void GroupSolver::batch_sample(int level, const uint64_t* seeds, int64_t first, int64_t count,
                               double* out, int* status) {
  check_eligible(level);
  const int np = (int)cs_.size();
  // every problem's work on the first problem's stream, after its own queue
  s_ = cs_[0]->s_;
  for (Context* c : cs_) MLMC_HIP(hipStreamSynchronize(c->s_));
  for (Context* c : cs_) {
    saved_.push_back(c->s_);
    c->s_ = s_;
    std::memset(c->counters, 0, sizeof(c->counters));
  }
  // stage capacity: every problem's V-cycle of its sample level
  int max_stages = 0;
  for (Context* c : cs_) {
    const int depth = c->Ls_ - level + 1;
    max_stages += depth * (c->opt_.nu_pre + c->opt_.nu_post + 2) + 2;
  }
  alloc(np, max_stages);
  const int nb = cs_[0]->nb_;
  std::vector<c64> buf((size_t)nb);
  std::vector<double> eb((size_t)nb);
  for (int i = 0; i < np; ++i) status[i] = MLMC_OK;
  for (int64_t j = 0; j < count; j += nb) {
    const int nbt = (int)std::min<int64_t>(nb, count - j);
    const uint64_t f = (uint64_t)(first + j);
    // problems that have not failed: this batch's level and level + 1 solves
    std::vector<Task> A, B;
    for (int i = 0; i < np; ++i) {
      if (status[i] != MLMC_OK) continue;  // a failed problem takes no more batches
      Context* c = cs_[i];
      c->write_probes(level, seeds[i], kStreamProbe, f, nbt, c->b1_);
      A.push_back(Task{c, i, level, c->b1_, c->y1_, nbt, c->scal_[Context::kErr1], {}});
      B.push_back(Task{c, i, level + 1, c->b2_, c->y2_, nbt, c->scal_[Context::kErr2], {}});
    }
    if (A.empty()) break;
    solve(A);
    const int na = (int)A.size();
    std::vector<std::vector<char>> ok1(na), ok2(na);
    for (int a = 0; a < na; ++a) {
      Context* c = A[a].c;
      if (A[a].l != c->Ls_) epilogue(A[a]);
      ok1[a] = c->col_ok_;
      c->restrict64(level, c->b1_, c->b2_, nbt);
    }
    solve(B);
    for (int a = 0; a < na; ++a) {
      Context* c = B[a].c;
      const int i = B[a].p;
      if (B[a].l != c->Ls_) epilogue(B[a]);
      ok2[a] = c->col_ok_;
      c->probe_quad(level, seeds[i], kStreamProbe, f, nbt, c->y1_, c->scal_[Context::kQa]);
      const int64_t n2 = c->lv_[level].n;
      vec_dot_partials<double>(c->b2_, c->y2_, n2, nbt, nullptr, c->partials_, s_);
      finish_sums(c->partials_, reduce_blocks(n2), nbt, c->scal_[Context::kQb], s_);
      double* o = out + (size_t)i * (size_t)count * 2;
      try {
        c->finish_samples(level, nbt, ok1[a].data(), ok2[a].data(), f, buf.data(), eb.data());
      } catch (const Error& e) {
        status[i] = e.code;
        c->last_error = e.what();
      }
      for (int k = 0; k < nbt; ++k) {
        o[2 * (j + k)] = buf[(size_t)k].re;
        o[2 * (j + k) + 1] = buf[(size_t)k].im;
      }
    }
  }
  collect();
  release();
}

// entry from the C ABI.  mode 1: one persistent launch per V-cycle, a
// workgroup per (problem, column pair) running all stages of its pair; mode 2:
// one stage-kernel launch per V-cycle position and stage kernel.  (A form with
// one workgroup per item of a shared queue, waiting on device-scope completion
// counts of the previous stage, did not finish on the GPU within the tests'
// time limits and was removed.)
void group_batch_sample(const std::vector<Context*>& cs, int level, const uint64_t* seeds,
                        int64_t first, int64_t count, int mode, double* out, int* status) {
  MLMC_REQUIRE(mode == 1 || mode == 2, MLMC_EINVAL, "grouped solves: mode must be 1 or 2");
  GroupSolver g(cs, mode);
  g.batch_sample(level, seeds, first, count, out, status);
}

}  // namespace mlmc
