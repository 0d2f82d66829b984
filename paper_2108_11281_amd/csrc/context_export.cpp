// Export of the hierarchy (Sec. 4.1: A_{l+1} = R_l A_l P_l, R_l = P_l^H) as
// sparse matrices in canonical compressed-row form, for every operator kind:
// the level operators A_l and the prolongations P_l as the library holds them.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "context.h"

namespace mlmc {

namespace {

// rows of (column, value) pairs -> canonical CSR: columns ascending, repeated
// columns summed, exact zeros dropped
struct Triplets {
  int64_t rows = 0, cols = 0;
  bool cplx = false;
  std::vector<int64_t> rp;
  std::vector<int> ci;
  std::vector<double> v;  // cplx: interleaved (re, im)
};

void canonical_row(std::vector<std::pair<int, c64>>& row, Triplets& out) {
  std::sort(row.begin(), row.end(),
            [](const std::pair<int, c64>& a, const std::pair<int, c64>& b) {
              return a.first < b.first;
            });
  for (size_t i = 0; i < row.size();) {
    const int c = row[i].first;
    c64 s = {0.0, 0.0};
    for (; i < row.size() && row[i].first == c; ++i) {
      s.re += row[i].second.re;
      s.im += row[i].second.im;
    }
    if (s.re == 0.0 && s.im == 0.0) continue;
    out.ci.push_back(c);
    out.v.push_back(s.re);
    if (out.cplx) out.v.push_back(s.im);
  }
  out.rp.push_back((int64_t)out.ci.size());
}

// 2D grid aggregation: fine (x, y) on side N -> coarse (x / 2, y / 2), value w
void agg_grid_2d(int N, double w, Triplets& t) {
  const int Nc = N / 2;
  t.rows = (int64_t)N * N;
  t.cols = (int64_t)Nc * Nc;
  t.rp.assign(1, 0);
  for (int y = 0; y < N; ++y)
    for (int x = 0; x < N; ++x) {
      t.ci.push_back((y / 2) * Nc + x / 2);
      t.v.push_back(w);
      t.rp.push_back((int64_t)t.ci.size());
    }
}

}  // namespace

void Context::export_level(int level, int which, int64_t* rows, int64_t* cols, int64_t* nnz,
                           int64_t* row_ptr, int32_t* col_idx, double* vals) {
  MLMC_REQUIRE(which == 0 || which == 1, MLMC_EINVAL, "which must be 0 (A_l) or 1 (P_l)");
  MLMC_REQUIRE(level >= 1 && level <= Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(which == 0 || level < Ls_, MLMC_EINVAL, "the coarsest level has no prolongation");
  const Level& L = lv_[level - 1];
  Triplets t;
  t.cplx = complex_;
  if (which == 0) {
    t.rows = t.cols = L.n;
    t.rp.assign(1, 0);
    std::vector<std::pair<int, c64>> row;
    if (csr_) {
      for (int64_t i = 0; i < L.n; ++i) {
        row.clear();
        for (int64_t e = L.h_rp[i]; e < L.h_rp[i + 1]; ++e)
          row.push_back({L.h_ci[e], c64{L.h_v[e], 0.0}});
        canonical_row(row, t);
      }
    } else if (complex_) {
      // the level's blocks (or the Wilson operator from its links) listed on the
      // device by the stencil kernels' own coupling rule
      const int per = 5 * L.dof;
      int* dc = dalloc_n<int>(L.n * per);
      c64* dv = dalloc_n<c64>(L.n * per);
      stencil_entries(L.wilson ? nullptr : L.B64, L.U64, op_.mass + 2.0, L.side, L.dof, dc, dv,
                      s_);
      std::vector<int> hc((size_t)L.n * per);
      std::vector<c64> hv((size_t)L.n * per);
      MLMC_HIP(hipMemcpyAsync(hc.data(), dc, sizeof(int) * hc.size(), hipMemcpyDeviceToHost, s_));
      MLMC_HIP(hipMemcpyAsync(hv.data(), dv, sizeof(c64) * hv.size(), hipMemcpyDeviceToHost, s_));
      MLMC_HIP(hipStreamSynchronize(s_));
      dfree(dv);
      dfree(dc);
      for (int64_t i = 0; i < L.n; ++i) {
        row.clear();
        for (int e = 0; e < per; ++e)
          row.push_back({hc[(size_t)i * per + e], hv[(size_t)i * per + e]});
        canonical_row(row, t);
      }
    } else if (varcoef_) {
      // 7-point: diagonal dg, -k on each interior face (k[3][N][N][N+1]:
      // x-faces [z][y][f], y-faces [z][x][f], z-faces [y][x][f])
      const int N = L.side;
      const int64_t nf = 3LL * N * N * (N + 1);
      std::vector<double> kf((size_t)nf), dg((size_t)L.n);
      MLMC_HIP(hipMemcpyAsync(kf.data(), L.kf64, sizeof(double) * kf.size(), hipMemcpyDeviceToHost,
                              s_));
      MLMC_HIP(hipMemcpyAsync(dg.data(), L.dg64, sizeof(double) * dg.size(), hipMemcpyDeviceToHost,
                              s_));
      MLMC_HIP(hipStreamSynchronize(s_));
      const int64_t NN = (int64_t)N * N, F = N + 1;
      auto kx = [&](int z, int y, int f) { return kf[(size_t)((z * (int64_t)N + y) * F + f)]; };
      auto ky = [&](int z, int x, int f) {
        return kf[(size_t)(NN * F + (z * (int64_t)N + x) * F + f)];
      };
      auto kz = [&](int y, int x, int f) {
        return kf[(size_t)(2 * NN * F + (y * (int64_t)N + x) * F + f)];
      };
      for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
          for (int x = 0; x < N; ++x) {
            const int64_t i = (z * (int64_t)N + y) * N + x;
            row.clear();
            row.push_back({(int)i, c64{dg[(size_t)i], 0.0}});
            if (x > 0) row.push_back({(int)(i - 1), c64{-kx(z, y, x), 0.0}});
            if (x + 1 < N) row.push_back({(int)(i + 1), c64{-kx(z, y, x + 1), 0.0}});
            if (y > 0) row.push_back({(int)(i - N), c64{-ky(z, x, y), 0.0}});
            if (y + 1 < N) row.push_back({(int)(i + N), c64{-ky(z, x, y + 1), 0.0}});
            if (z > 0) row.push_back({(int)(i - NN), c64{-kz(y, x, z), 0.0}});
            if (z + 1 < N) row.push_back({(int)(i + NN), c64{-kz(y, x, z + 1), 0.0}});
            canonical_row(row, t);
          }
    } else {
      // 2D Poisson level: d I - c (grid neighbours), Dirichlet
      const int N = L.side;
      for (int y = 0; y < N; ++y)
        for (int x = 0; x < N; ++x) {
          const int i = y * N + x;
          row.clear();
          row.push_back({i, c64{L.d, 0.0}});
          if (x > 0) row.push_back({i - 1, c64{-L.c, 0.0}});
          if (x + 1 < N) row.push_back({i + 1, c64{-L.c, 0.0}});
          if (y > 0) row.push_back({i - N, c64{-L.c, 0.0}});
          if (y + 1 < N) row.push_back({i + N, c64{-L.c, 0.0}});
          canonical_row(row, t);
        }
    }
  } else {
    const Level& C = lv_[level];
    if (csr_ && general_) {
      t.rows = L.n;
      t.cols = L.pcols;
      t.rp.assign(L.hp_rp.begin(), L.hp_rp.end());
      t.ci.assign(L.hp_ci.begin(), L.hp_ci.end());
      t.v.assign(L.hp_v.begin(), L.hp_v.end());
    } else if (csr_) {
      // orthonormal piecewise constants: 1/sqrt(|J|) on the aggregate J of i
      std::vector<int64_t> size((size_t)C.n, 0);
      for (int64_t i = 0; i < L.n; ++i) size[(size_t)L.h_agg[(size_t)i]] += 1;
      t.rows = L.n;
      t.cols = C.n;
      t.rp.assign(1, 0);
      for (int64_t i = 0; i < L.n; ++i) {
        const int a = L.h_agg[(size_t)i];
        t.ci.push_back(a);
        t.v.push_back(1.0 / std::sqrt((double)size[(size_t)a]));
        t.rp.push_back((int64_t)t.ci.size());
      }
    } else if (complex_) {
      // fine unknown i = s * dof + a of site s = (sx, sy) lies in aggregate
      // (sx / blk, sy / blk); its row holds the aggregate basis coefficients q[i]
      const int nv = C.dof, Nc = L.side / L.blk;
      std::vector<c64> q((size_t)L.n * nv);
      MLMC_HIP(hipMemcpyAsync(q.data(), L.q64, sizeof(c64) * q.size(), hipMemcpyDeviceToHost, s_));
      MLMC_HIP(hipStreamSynchronize(s_));
      t.rows = L.n;
      t.cols = C.n;
      t.rp.assign(1, 0);
      std::vector<std::pair<int, c64>> row;
      for (int64_t i = 0; i < L.n; ++i) {
        const int s = (int)(i / L.dof), sy = s / L.side, sx = s - sy * L.side;
        const int agg = (sy / L.blk) * Nc + sx / L.blk;
        row.clear();
        for (int v = 0; v < nv; ++v) row.push_back({agg * nv + v, q[(size_t)i * nv + v]});
        canonical_row(row, t);
      }
    } else if (varcoef_) {
      const int N = L.side, Nc = N / 2;
      const double w = 1.0 / std::sqrt(8.0);
      t.rows = L.n;
      t.cols = C.n;
      t.rp.assign(1, 0);
      for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
          for (int x = 0; x < N; ++x) {
            t.ci.push_back(((z / 2) * Nc + y / 2) * Nc + x / 2);
            t.v.push_back(w);
            t.rp.push_back((int64_t)t.ci.size());
          }
    } else {
      agg_grid_2d(L.side, 0.5, t);
    }
  }
  if (rows) *rows = t.rows;
  if (cols) *cols = t.cols;
  if (nnz) *nnz = t.rp.back();
  if (row_ptr) std::copy(t.rp.begin(), t.rp.end(), row_ptr);
  if (col_idx) std::copy(t.ci.begin(), t.ci.end(), col_idx);
  if (vals) std::copy(t.v.begin(), t.v.end(), vals);
}

}  // namespace mlmc
