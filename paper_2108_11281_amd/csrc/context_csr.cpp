// Operators given as a sparse matrix (MLMC_CSR): hierarchy construction on the
// host (canonical rows, symmetry check, greedy aggregation of the matrix graph,
// first-fit colouring, Galerkin products with orthonormal piecewise-constant
// aggregation, Sec. 4.1), upload of every level, the autotuner of the sweep
// and the V-cycle.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "context.h"

namespace mlmc {
namespace {

struct HostCsr {
  int n = 0;     // rows
  int cols = 0;  // columns
  std::vector<int64_t> rp;
  std::vector<int> ci;
  std::vector<double> v;
};

// rows sorted by column, repeated entries summed, zero entries dropped; n rows,
// ncols columns (ncols 0: square)
HostCsr canonical(int64_t n, const int64_t* rp, const int32_t* ci, const double* v,
                  int64_t ncols = 0) {
  if (ncols == 0) ncols = n;
  MLMC_REQUIRE(n >= 1 && n < (int64_t)1 << 31, MLMC_EINVAL, "CSR needs 1 <= n < 2^31");
  MLMC_REQUIRE(ncols >= 1 && ncols < (int64_t)1 << 31, MLMC_EINVAL,
               "CSR needs 1 <= cols < 2^31");
  MLMC_REQUIRE(rp != nullptr && ci != nullptr && v != nullptr, MLMC_EINVAL,
               "CSR needs row_ptr, col_idx and vals");
  MLMC_REQUIRE(rp[0] == 0, MLMC_EINVAL, "row_ptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    MLMC_REQUIRE(rp[i + 1] >= rp[i], MLMC_EINVAL, "row_ptr must be non-decreasing");
  MLMC_REQUIRE(rp[n] < (int64_t)1 << 31, MLMC_EINVAL, "CSR needs nnz < 2^31");
  HostCsr A;
  A.n = (int)n;
  A.cols = (int)ncols;
  A.rp.assign(n + 1, 0);
  A.ci.reserve(rp[n]);
  A.v.reserve(rp[n]);
  std::vector<std::pair<int, double>> row;
  for (int64_t i = 0; i < n; ++i) {
    row.clear();
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      MLMC_REQUIRE(ci[e] >= 0 && ci[e] < ncols, MLMC_EINVAL, "column index out of range");
      MLMC_REQUIRE(std::isfinite(v[e]), MLMC_EINVAL, "CSR values must be finite");
      row.push_back({ci[e], v[e]});
    }
    std::stable_sort(row.begin(), row.end(),
                     [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
                       return a.first < b.first;
                     });
    for (size_t k = 0; k < row.size();) {
      const int j = row[k].first;
      double sum = 0.0;
      for (; k < row.size() && row[k].first == j; ++k) sum += row[k].second;
      if (sum != 0.0) {
        A.ci.push_back(j);
        A.v.push_back(sum);
      }
    }
    A.rp[i + 1] = (int64_t)A.ci.size();
  }
  return A;
}

// value of entry (i, j), or 0 (rows sorted)
double entry(const HostCsr& A, int i, int j) {
  const int* lo = A.ci.data() + A.rp[i];
  const int* hi = A.ci.data() + A.rp[i + 1];
  const int* p = std::lower_bound(lo, hi, j);
  return (p != hi && *p == j) ? A.v[p - A.ci.data()] : 0.0;
}

void check_spd_shape(const HostCsr& A, int level) {
  const std::string at = " (level " + std::to_string(level) + ")";
  for (int i = 0; i < A.n; ++i) {
    MLMC_REQUIRE(entry(A, i, i) > 0, MLMC_EINVAL, "every row needs a positive diagonal" + at);
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.ci[e];
      const double a = A.v[e], b = entry(A, j, i);
      MLMC_REQUIRE(std::fabs(a - b) <= 1e-12 * std::max(std::fabs(a), std::fabs(b)), MLMC_EINVAL,
                   "the matrix must be symmetric" + at);
    }
  }
}

// Greedy aggregation of the matrix graph: pass 1 visits unknowns in index
// order and one whose neighbours are all unassigned founds an aggregate with
// them; pass 2 puts every unknown left over into the pass-1 aggregate of its
// neighbour with the largest |a_ij| (the smallest j among equal ones; the
// columns are ascending, so the first maximum wins).
std::vector<int> greedy_aggregates(const HostCsr& A, int* nc_out) {
  std::vector<int> agg(A.n, -1);
  int nc = 0;
  for (int i = 0; i < A.n; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int64_t e = A.rp[i]; e < A.rp[i + 1] && free; ++e)
      if (A.ci[e] != i && agg[A.ci[e]] >= 0) free = false;
    if (!free) continue;
    agg[i] = nc;
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) agg[A.ci[e]] = nc;
    ++nc;
  }
  const std::vector<int> first = agg;
  for (int i = 0; i < A.n; ++i) {
    if (agg[i] >= 0) continue;
    double best = -1.0;
    int to = -1;
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.ci[e];
      if (j == i || first[j] < 0) continue;
      if (std::fabs(A.v[e]) > best) {
        best = std::fabs(A.v[e]);
        to = first[j];
      }
    }
    MLMC_REQUIRE(to >= 0, MLMC_EINVAL, "greedy aggregation left an unknown unassigned");
    agg[i] = to;
  }
  *nc_out = nc;
  return agg;
}

// first-fit colouring in index order: the smallest colour that no neighbour
// with a smaller index holds
std::vector<int> first_fit_colours(const HostCsr& A) {
  std::vector<int> colour(A.n, 0);
  std::vector<int> mark;
  for (int i = 0; i < A.n; ++i) {
    for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
      const int j = A.ci[e];
      if (j >= i) continue;
      const int c = colour[j];
      if ((int)mark.size() <= c) mark.resize(c + 1, -1);
      mark[c] = i;
    }
    int c = 0;
    while (c < (int)mark.size() && mark[c] == i) ++c;
    colour[i] = c;
  }
  return colour;
}

// A_c = P^T A P with P(i, J) = 1/sqrt|J| for J = agg[i]
HostCsr galerkin(const HostCsr& A, const std::vector<int>& agg, int nc) {
  std::vector<int> size(nc, 0);
  for (int i = 0; i < A.n; ++i) ++size[agg[i]];
  std::vector<int> aptr(nc + 1, 0), arows(A.n);
  for (int J = 0; J < nc; ++J) aptr[J + 1] = aptr[J] + size[J];
  {
    std::vector<int> fill(aptr.begin(), aptr.end() - 1);
    for (int i = 0; i < A.n; ++i) arows[fill[agg[i]]++] = i;
  }
  HostCsr C;
  C.n = nc;
  C.cols = nc;
  C.rp.assign(nc + 1, 0);
  std::vector<double> acc(nc, 0.0);
  std::vector<int> seen(nc, -1), touched;
  for (int I = 0; I < nc; ++I) {
    touched.clear();
    for (int m = aptr[I]; m < aptr[I + 1]; ++m) {
      const int i = arows[m];
      for (int64_t e = A.rp[i]; e < A.rp[i + 1]; ++e) {
        const int J = agg[A.ci[e]];
        if (seen[J] != I) {
          seen[J] = I;
          acc[J] = 0.0;
          touched.push_back(J);
        }
        acc[J] += A.v[e];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int J : touched) {
      const double val = acc[J] / std::sqrt((double)size[I] * (double)size[J]);
      if (val != 0.0) {
        C.ci.push_back(J);
        C.v.push_back(val);
      }
    }
    C.rp[I + 1] = (int64_t)C.ci.size();
  }
  return C;
}

// X^T (cols x rows), rows of the result in ascending column order
HostCsr transpose(const HostCsr& X) {
  HostCsr T;
  T.n = X.cols;
  T.cols = X.n;
  T.rp.assign(T.n + 1, 0);
  for (int c : X.ci) ++T.rp[c + 1];
  for (int i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(X.ci.size());
  T.v.resize(X.v.size());
  std::vector<int64_t> fill(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < X.n; ++i)
    for (int64_t e = X.rp[i]; e < X.rp[i + 1]; ++e) {
      const int64_t d = fill[X.ci[e]]++;
      T.ci[d] = i;
      T.v[d] = X.v[e];
    }
  return T;
}

// X Y (X.n x Y.cols), rows with ascending columns, exact zeros dropped
HostCsr spgemm(const HostCsr& X, const HostCsr& Y) {
  MLMC_REQUIRE(X.cols == Y.n, MLMC_EINVAL, "sparse product: inner dimensions differ");
  HostCsr C;
  C.n = X.n;
  C.cols = Y.cols;
  C.rp.assign(C.n + 1, 0);
  std::vector<double> acc(Y.cols, 0.0);
  std::vector<int> seen(Y.cols, -1), touched;
  for (int i = 0; i < X.n; ++i) {
    touched.clear();
    for (int64_t e = X.rp[i]; e < X.rp[i + 1]; ++e) {
      const int k = X.ci[e];
      const double a = X.v[e];
      for (int64_t f = Y.rp[k]; f < Y.rp[k + 1]; ++f) {
        const int j = Y.ci[f];
        if (seen[j] != i) {
          seen[j] = i;
          acc[j] = 0.0;
          touched.push_back(j);
        }
        acc[j] += a * Y.v[f];
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int j : touched)
      if (acc[j] != 0.0) {
        C.ci.push_back(j);
        C.v.push_back(acc[j]);
      }
    C.rp[i + 1] = (int64_t)C.ci.size();
  }
  return C;
}

// SELL-64 copy (see CsrMat) of the rows `rows` of (rp, ci, v) (row -1: an
// empty padding position): slice offsets, column indices and values; with
// skip_diag the diagonal entry of each row is left out.  Padding entries hold
// value 0 and, for square matrices (own_pad), the row itself as column,
// otherwise column 0, so they add nothing and read in bounds.
void sell_build(const std::vector<int64_t>& rp, const std::vector<int>& ci,
                const std::vector<double>& v, const std::vector<int>& rows, bool skip_diag,
                bool own_pad, std::vector<int>& sptr, std::vector<int>& sci,
                std::vector<double>& sv) {
  const int m = (int)rows.size();
  const int ns = (m + 63) / 64;
  sptr.assign(ns + 1, 0);
  for (int sl = 0; sl < ns; ++sl) {
    int w = 0;
    for (int l = 0; l < 64 && sl * 64 + l < m; ++l) {
      const int i = rows[sl * 64 + l];
      if (i < 0) continue;
      const int len = (int)(rp[i + 1] - rp[i]) - (skip_diag ? 1 : 0);
      w = std::max(w, len);
    }
    MLMC_REQUIRE((int64_t)sptr[sl] + 64LL * w < (int64_t)1 << 31, MLMC_EINVAL,
                 "sliced matrix copy exceeds 2^31 entries");
    sptr[sl + 1] = sptr[sl] + 64 * w;
  }
  sci.assign(sptr[ns], 0);
  sv.assign(sptr[ns], 0.0);
  for (int sl = 0; sl < ns; ++sl) {
    const int w = (sptr[sl + 1] - sptr[sl]) / 64;
    for (int l = 0; l < 64; ++l) {
      const int pos = sl * 64 + l;
      const int i = pos < m ? rows[pos] : -1;
      int e = 0;
      if (i >= 0) {
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
          if (skip_diag && ci[q] == i) continue;
          sci[sptr[sl] + e * 64 + l] = ci[q];
          sv[sptr[sl] + e * 64 + l] = v[q];
          ++e;
        }
      }
      for (; e < w; ++e) sci[sptr[sl] + e * 64 + l] = (own_pad && i >= 0) ? i : 0;
    }
  }
}

}  // namespace

template <> const CsrMat<float>& Context::csr_mat<float>(int l) const { return lv_[l - 1].A32; }
template <> const CsrMat<double>& Context::csr_mat<double>(int l) const { return lv_[l - 1].A64; }
template <> const CsrSweep<float>& Context::csr_sweep<float>(int l) const {
  return lv_[l - 1].S32;
}
template <> const CsrSweep<double>& Context::csr_sweep<double>(int l) const {
  return lv_[l - 1].S64;
}
template <> const CsrMat<float>& Context::csr_P<float>(int l) const { return lv_[l - 1].P32; }
template <> const CsrMat<double>& Context::csr_P<double>(int l) const { return lv_[l - 1].P64; }
template <> const CsrMat<float>& Context::csr_R<float>(int l) const { return lv_[l - 1].R32; }
template <> const CsrMat<double>& Context::csr_R<double>(int l) const { return lv_[l - 1].R64; }
template <> const CsrAgg<float>& Context::csr_agg<float>(int l) const { return lv_[l - 1].G32; }
template <> const CsrAgg<double>& Context::csr_agg<double>(int l) const { return lv_[l - 1].G64; }

// device copies of level L's matrix, colour-sorted sweep arrays and (unless it
// is the coarsest level) its aggregation, from the host copies in L
void Context::csr_upload(Level& L, bool last) {
  const int n = (int)L.n;
  auto up = [&](const auto& h) {
    using V = typename std::decay<decltype(h)>::type::value_type;
    V* d = dalloc_n<V>(std::max<int64_t>((int64_t)h.size(), 1));
    if (!h.empty()) {  // h may be a temporary: wait for the copy
      MLMC_HIP(hipMemcpyAsync(d, h.data(), sizeof(V) * h.size(), hipMemcpyHostToDevice, s_));
      MLMC_HIP(hipStreamSynchronize(s_));
    }
    return d;
  };
  auto to_f32 = [](const std::vector<double>& a) {
    return std::vector<float>(a.begin(), a.end());
  };
  auto sell = [&](const std::vector<int>& rows, bool skip_diag, std::vector<int>& sptr,
                  std::vector<int>& sci, std::vector<double>& sv) {
    sell_build(L.h_rp, L.h_ci, L.h_v, rows, skip_diag, true, sptr, sci, sv);
  };
  // the matrix by rows: plain CSR (dense build) and its SELL-64 copy
  std::vector<int> rp32(L.h_rp.begin(), L.h_rp.end());
  const int* rp = up(rp32);
  const int* ci = up(L.h_ci);
  std::vector<int> all(n), sptr, sci;
  std::vector<double> sv;
  std::iota(all.begin(), all.end(), 0);
  sell(all, false, sptr, sci, sv);
  const int* dsptr = up(sptr);
  const int* dsci = up(sci);
  L.A64 = {n, n, rp, ci, up(L.h_v), dsptr, dsci, up(sv)};
  L.A32 = {n, n, rp, ci, up(to_f32(L.h_v)), dsptr, dsci, up(to_f32(sv))};
  // the off-diagonal part by colour class (ascending rows within a class), each
  // class padded to whole slices, and the inverted diagonal per position
  const int ncol = n ? *std::max_element(L.h_colour.begin(), L.h_colour.end()) + 1 : 0;
  std::vector<int> cnt(ncol, 0);
  for (int i = 0; i < n; ++i) ++cnt[L.h_colour[i]];
  std::vector<int> soff(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) soff[c + 1] = soff[c] + (cnt[c] + 63) / 64;
  std::vector<int> srow(64 * (size_t)soff[ncol], -1);
  {
    std::vector<int> fill(ncol);
    for (int c = 0; c < ncol; ++c) fill[c] = 64 * soff[c];
    for (int i = 0; i < n; ++i) srow[fill[L.h_colour[i]]++] = i;
  }
  std::vector<double> sdi(srow.size(), 0.0);
  for (size_t k = 0; k < srow.size(); ++k)
    if (srow[k] >= 0) {
      const int i = srow[k];
      for (int64_t q = L.h_rp[i]; q < L.h_rp[i + 1]; ++q)
        if (L.h_ci[q] == i) sdi[k] = 1.0 / L.h_v[q];
    }
  std::vector<int> gptr, gci;
  std::vector<double> gv;
  sell(srow, true, gptr, gci, gv);
  const int* dsrow = up(srow);
  const int* dgptr = up(gptr);
  const int* dgci = up(gci);
  L.S64.srow = L.S32.srow = dsrow;
  L.S64.sptr = L.S32.sptr = dgptr;
  L.S64.sci = L.S32.sci = dgci;
  L.S64.sv = up(gv);
  L.S64.sdi = up(sdi);
  L.S32.sv = up(to_f32(gv));
  L.S32.sdi = up(to_f32(sdi));
  L.S64.soff = L.S32.soff = soff;
  if (last) return;
  if (general_) {
    // given prolongation P (n x pcols) and R = P^T, SELL-64 copies of both
    HostCsr Ph;
    Ph.n = n;
    Ph.cols = L.pcols;
    Ph.rp = L.hp_rp;
    Ph.ci = L.hp_ci;
    Ph.v = L.hp_v;
    const HostCsr Rh = transpose(Ph);
    auto put = [&](const HostCsr& M, CsrMat<float>& m32, CsrMat<double>& m64) {
      std::vector<int> rows(M.n), sp, sc;
      std::vector<double> sw;
      std::iota(rows.begin(), rows.end(), 0);
      sell_build(M.rp, M.ci, M.v, rows, false, false, sp, sc, sw);
      const int* dsp = up(sp);
      const int* dsc = up(sc);
      m64 = {M.n, M.cols, nullptr, nullptr, nullptr, dsp, dsc, up(sw)};
      m32 = {M.n, M.cols, nullptr, nullptr, nullptr, dsp, dsc, up(to_f32(sw))};
    };
    put(Ph, L.P32, L.P64);
    put(Rh, L.R32, L.R64);
    return;
  }
  // aggregation: member lists (ascending) and the scales 1/sqrt|J|
  const int nc = *std::max_element(L.h_agg.begin(), L.h_agg.end()) + 1;
  std::vector<int> aptr(nc + 1, 0), arows(n);
  for (int i = 0; i < n; ++i) ++aptr[L.h_agg[i] + 1];
  for (int J = 0; J < nc; ++J) aptr[J + 1] += aptr[J];
  {
    std::vector<int> fill(aptr.begin(), aptr.end() - 1);
    for (int i = 0; i < n; ++i) arows[fill[L.h_agg[i]]++] = i;
  }
  std::vector<double> cs(nc), fs(n);
  for (int J = 0; J < nc; ++J) cs[J] = 1.0 / std::sqrt((double)(aptr[J + 1] - aptr[J]));
  for (int i = 0; i < n; ++i) fs[i] = cs[L.h_agg[i]];
  const int* dagg = up(L.h_agg);
  const int* daptr = up(aptr);
  const int* darows = up(arows);
  L.G64 = {nc, dagg, daptr, darows, up(fs), up(cs)};
  L.G32 = {nc, dagg, daptr, darows, up(to_f32(fs)), up(to_f32(cs))};
}

void Context::build_csr(const mlmc_operator& A, const int32_t* const* aggs, const mlmc_csr* P) {
  MLMC_REQUIRE(!(aggs && P), MLMC_EINVAL, "give aggregate maps or prolongations, not both");
  general_ = P != nullptr;
  lv_.resize(Ls_);
  HostCsr cur = canonical(A.n, A.row_ptr, A.col_idx, A.vals);
  for (int l = 0; l < Ls_; ++l) {
    check_spd_shape(cur, l + 1);
    Level& L = lv_[l];
    L.index = l + 1;
    L.side = 0;
    L.dof = 1;
    L.n = cur.n;
    L.h_colour = first_fit_colours(cur);
    if (l + 1 < Ls_ && P) {
      // given prolongation: A_{l+1} = P^T A_l P (Sec. 4.1, R = P^T)
      const mlmc_csr& Pl = P[l];
      MLMC_REQUIRE(Pl.rows == cur.n, MLMC_EINVAL,
                   "P[" + std::to_string(l) + "] must have n_l rows");
      MLMC_REQUIRE(Pl.cols >= 1 && Pl.cols <= Pl.rows, MLMC_EINVAL,
                   "P[" + std::to_string(l) + "] needs 1 <= cols <= rows");
      HostCsr Ph = canonical(Pl.rows, Pl.row_ptr, Pl.col_idx, Pl.vals, Pl.cols);
      HostCsr next = spgemm(transpose(Ph), spgemm(cur, Ph));
      L.pcols = Ph.cols;
      L.hp_rp = std::move(Ph.rp);
      L.hp_ci = std::move(Ph.ci);
      L.hp_v = std::move(Ph.v);
      L.h_rp = std::move(cur.rp);
      L.h_ci = std::move(cur.ci);
      L.h_v = std::move(cur.v);
      cur = std::move(next);
    } else if (l + 1 < Ls_) {
      int nc = 0;
      if (aggs) {
        MLMC_REQUIRE(aggs[l] != nullptr, MLMC_EINVAL, "agg[" + std::to_string(l) + "] is null");
        L.h_agg.assign(aggs[l], aggs[l] + cur.n);
        int mx = -1;
        for (int a : L.h_agg) {
          MLMC_REQUIRE(a >= 0 && a < cur.n, MLMC_EINVAL, "aggregate number out of range");
          mx = std::max(mx, a);
        }
        nc = mx + 1;
        std::vector<char> used(nc, 0);
        for (int a : L.h_agg) used[a] = 1;
        MLMC_REQUIRE(std::all_of(used.begin(), used.end(), [](char u) { return u != 0; }),
                     MLMC_EINVAL, "aggregate numbers must cover 0..nc-1 without gaps");
      } else {
        L.h_agg = greedy_aggregates(cur, &nc);
      }
      HostCsr next = galerkin(cur, L.h_agg, nc);
      L.h_rp = std::move(cur.rp);
      L.h_ci = std::move(cur.ci);
      L.h_v = std::move(cur.v);
      cur = std::move(next);
    } else {
      L.h_rp = std::move(cur.rp);
      L.h_ci = std::move(cur.ci);
      L.h_v = std::move(cur.v);
    }
  }
  MLMC_REQUIRE(lv_[Ls_ - 1].n <= 16384, MLMC_EINVAL,
               "coarsest solver level larger than 16384 unknowns (add levels)");
  for (int l = 0; l < Ls_; ++l) csr_upload(lv_[l], l + 1 == Ls_);
  MLMC_HIP(hipStreamSynchronize(s_));
  finish_real_build();
  if (general_) {
    gA_ = dalloc_n<double>(lv_[1].n * nb_);
    gB_ = dalloc_n<double>(lv_[1].n * nb_);
    csr_general_coarse_trace();
  }
  tune_csr();
}

// Coarsest term of the general decomposition (Remark 4.2): tr(A_L^{-1} M) with
// M = Rhat_L Phat_L, formed level by level as M_{l+1} = P_l^T M_l P_l from
// M_2 = P_1^T P_1 (sparse, on the host); the FP64 inverse of A_L comes from
// the device.
void Context::csr_general_coarse_trace() {
  auto hp = [&](int l) {  // P_l as a host matrix (l 1-based)
    HostCsr Ph;
    Ph.n = (int)lv_[l - 1].n;
    Ph.cols = lv_[l - 1].pcols;
    Ph.rp = lv_[l - 1].hp_rp;
    Ph.ci = lv_[l - 1].hp_ci;
    Ph.v = lv_[l - 1].hp_v;
    return Ph;
  };
  HostCsr P1 = hp(1);
  HostCsr M = spgemm(transpose(P1), P1);
  for (int l = 2; l < L_; ++l) {
    HostCsr Pl = hp(l);
    M = spgemm(transpose(Pl), spgemm(M, Pl));
  }
  const int nL = (int)lv_[L_ - 1].n;
  MLMC_REQUIRE(M.n == nL && M.cols == nL, MLMC_EINVAL, "coarsest product has the wrong shape");
  std::vector<double> inv((size_t)nL * nL);
  const double* dinv = (L_ == Ls_) ? ainv_solver_ : ainv_mlmc_;
  MLMC_HIP(hipMemcpyAsync(inv.data(), dinv, sizeof(double) * inv.size(), hipMemcpyDeviceToHost,
                          s_));
  MLMC_HIP(hipStreamSynchronize(s_));
  // tr(A^{-1} M) = sum_{i,j} inv[i][j] M[j][i], over M's entries
  double tr = 0.0;
  for (int j = 0; j < nL; ++j)
    for (int64_t e = M.rp[j]; e < M.rp[j + 1]; ++e) tr += inv[(size_t)M.ci[e] * nL + j] * M.v[e];
  coarse_trace_ = {tr, 0.0};
}

// Level-l samples of the general decomposition: x on the finest level (probe
// stream keyed by level l), b_l = Rhat_l x by l-1 restrictions (FP64), y =
// A_l^{-1} b_l and z = A_{l+1}^{-1} R_l b_l; with R = P^T the two quadratic forms
// x^T Phat y and x^T Phat_{l+1} z are b_l^T y and b_{l+1}^T z.
void Context::samples_batch_general(int level, uint64_t seed, uint64_t first, int nbatch,
                                    c64* out, double* err_out) {
  const int64_t n1 = lv_[0].n;
  probes_write<double>(b1_, n1, nbatch, seed, 0, first, (uint64_t)level, kStreamProbe, s_);
  double* bl = b1_;
  for (int l = 1; l < level; ++l) {
    double* nxt = (bl == gA_) ? gB_ : gA_;
    op_restrict<double>(l, bl, nxt, nbatch, nullptr);
    bl = nxt;
  }
  bool ok1 = true, ok2 = true;
  c64 *e1 = scal_[kErr1], *e2 = scal_[kErr2], *qa = scal_[kQa], *qb = scal_[kQb];
  solve(level, bl, y1_, nbatch, e1, nullptr, &ok1);
  const std::vector<char> okc1 = col_ok_;
  op_restrict<double>(level, bl, b2_, nbatch, nullptr);
  solve(level + 1, b2_, y2_, nbatch, e2, nullptr, &ok2);
  const std::vector<char> okc2 = col_ok_;
  const int64_t nl = lv_[level - 1].n, nl1 = lv_[level].n;
  vec_dot_partials<double>(bl, y1_, nl, nbatch, nullptr, partials_, s_);
  finish_sums(partials_, reduce_blocks(nl), nbatch, qa, s_);
  vec_dot_partials<double>(b2_, y2_, nl1, nbatch, nullptr, partials_, s_);
  finish_sums(partials_, reduce_blocks(nl1), nbatch, qb, s_);
  finish_samples(level, nbatch, okc1.data(), okc2.data(), first, out, err_out);
}

// Autotuner of the CSR kernels: per smoothed level, time one Gauss-Seidel
// sweep with 1, 2, 4 and 8 right-hand sides per thread (the results are
// identical; only the reuse of the row's indices and values and the
// parallelism differ), once over all nb columns and once over a narrow batch
// of 16, and keep the fastest of each for every CSR kernel of that level; then,
// with that choice, the sweep's schedule of its trailing small colour classes
// (a launch per class, or the trailing classes of at most 4, 16 or 64 slices
// in shared launches: fewer launches, fewer compute units per class; the
// results are identical).  Each candidate is timed as the best of five sweeps
// after a warm-up.  Runs once at setup on the library's own work vectors.
void Context::tune_csr() {
  const bool fp32 = opt_.precision == MLMC_FP32_IR64;
  hipEvent_t a = event(), b = event();
  auto time_sweep = [&](const Level& L, int ncols, int cols, int tail) {
    float ms = 1e30f;  // best of 5 after a warm-up run (robust to noise)
    for (int rep = 0; rep < 6; ++rep) {
      MLMC_HIP(hipEventRecord(a, s_));
      if (fp32)
        csr_gs_sweep<float>(w32_.r, w32_.x, L.S32, (int)L.n, ncols, cols, tail, nullptr, false,
                            s_);
      else
        csr_gs_sweep<double>(w64_.r, w64_.x, L.S64, (int)L.n, ncols, cols, tail, nullptr, false,
                             s_);
      MLMC_HIP(hipEventRecord(b, s_));
      MLMC_HIP(hipEventSynchronize(b));
      float t = 0.f;
      MLMC_HIP(hipEventElapsedTime(&t, a, b));
      if (rep > 0) ms = std::min(ms, t);  // the first run warms caches and code
    }
    return ms;
  };
  for (int l = 1; l < Ls_; ++l) {
    Level& L = lv_[l - 1];
    const std::vector<int>& soff = L.S32.soff;
    for (int narrow = 0; narrow < 2; ++narrow) {
      const int ncols = narrow ? std::min(nb_, 16) : nb_;
      float best = 1e30f;
      int best_cols = 4;
      for (int cols : {1, 2, 4, 8}) {
        const float ms = time_sweep(L, ncols, cols, 0);
        if (ms < best) {
          best = ms;
          best_cols = cols;
        }
      }
      (narrow ? L.cols_narrow : L.cols) = best_cols;
      // shared launches only where they are at least 5% faster than a launch
      // per class, so that the choice does not follow timing noise
      const float t_classes = best;
      int best_tail = 0, last_start = csr_tail_start(soff, 0);
      for (int tail : {4, 16, 64}) {
        const int start = csr_tail_start(soff, tail);
        if (start == last_start) continue;  // the same schedule as a smaller bound
        last_start = start;
        const float ms = time_sweep(L, ncols, best_cols, tail);
        if (ms < best && ms < 0.95f * t_classes) {
          best = ms;
          best_tail = tail;
        }
      }
      (narrow ? L.tail_slices_narrow : L.tail_slices) = best_tail;
    }
  }
  ev_pool_.push_back(a);
  ev_pool_.push_back(b);
}

// V-cycle of a CSR level: in-place multicolour Gauss-Seidel sweeps (classes in
// ascending order before the coarse correction, descending after it, so the
// preconditioner is symmetric), residual + restriction, prolongation +
// omega-scaled correction.
template <typename T>
void Context::vcycle_csr(int l, const T* b, T* x, int nb, const int* act, c64* rz_partials,
                         bool top) {
  Work<T>& w = work<T>();
  if (l == 1) counters[2] += 1;
  const Level& L = lv_[l - 1];
  const int64_t n = L.n;
  const double en = (double)sizeof(T) * (double)n;
  if (l == Ls_) {
    dense_apply<T>(w.ainvT, b, x, (int)n, nb, act, s_, w.ld);
  } else {
    const CsrMat<T>& A = csr_mat<T>(l);
    const CsrSweep<T>& S = csr_sweep<T>(l);
    const CsrAgg<T>& G = csr_agg<T>(l);
    const int64_t nnz = L.h_rp[n];
    // matrix bytes of a sweep (off-diagonal entries, row ids, offsets, inverted
    // diagonal) and of a residual (all entries, offsets), shared by the columns
    const double sweep_mat = (double)(nnz - n) * (4.0 + sizeof(T)) + (double)n * (8.0 + sizeof(T));
    const double res_mat = (double)nnz * (4.0 + sizeof(T)) + 4.0 * (double)n;
    const double enc = (double)sizeof(T) * (double)lv_[l].n;
    const int pre = opt_.nu_pre, post = opt_.nu_post;
    const int cols = csr_cols(L, nb), tail = csr_tail(L, nb);
    if (pre > 0) vec_zero<T>(x, n, nb, act, s_);
    for (int i = 0; i < pre; ++i)
      timed<T>(l, kTimGs, 3.0 * en + sweep_mat / nb, act, nb,
               [&] { csr_gs_sweep<T>(b, x, S, (int)n, nb, cols, tail, act, false, s_); });
    T* bc = w.vb[l];
    T* ec = w.vx[l];
    if (general_) {  // given P and R = P^T
      const CsrMat<T>& Pm = csr_P<T>(l);
      const CsrMat<T>& Rm = csr_R<T>(l);
      if (pre == 0) {
        csr_spmm<T>(b, bc, Rm, 1.0, 0.0, nb, cols, act, s_);
      } else {
        timed<T>(l, kTimResRestrict, 2.0 * en + enc + res_mat / nb, act, nb, [&] {
          csr_residual<T, T, T>(b, x, w.vt[l - 1], A, nb, cols, act, nullptr, s_);
          csr_spmm<T>(w.vt[l - 1], bc, Rm, 1.0, 0.0, nb, cols, act, s_);
        });
      }
      vcycle_csr<T>(l + 1, bc, ec, nb, act, nullptr);
      second_coarse_cycle<T>(l, bc, ec, nb, act, top);
      timed<T>(l, kTimProlong, (pre == 0 ? 1.0 : 2.0) * en + enc, act, nb, [&] {
        csr_spmm<T>(ec, x, Pm, omega_, pre == 0 ? 0.0 : 1.0, nb, cols, act, s_);
      });
    } else {
      if (pre == 0)
        csr_restrict<T>(nullptr, b, bc, nullptr, A, G, nb, cols, act, s_);
      else  // the residual passes through the level's scratch vector
        timed<T>(l, kTimResRestrict, 2.0 * en + enc + res_mat / nb, act, nb,
                 [&] { csr_restrict<T>(b, x, bc, w.vt[l - 1], A, G, nb, cols, act, s_); });
      vcycle_csr<T>(l + 1, bc, ec, nb, act, nullptr);
      second_coarse_cycle<T>(l, bc, ec, nb, act, top);
      timed<T>(l, kTimProlong, (pre == 0 ? 1.0 : 2.0) * en + enc, act, nb, [&] {
        csr_prolong<T>(ec, x, G, (int)n, omega_, pre == 0 ? 0.0 : 1.0, nb, act, s_);
      });
    }
    for (int i = 0; i < post; ++i)
      timed<T>(l, kTimGs, 3.0 * en + sweep_mat / nb, act, nb,
               [&] { csr_gs_sweep<T>(b, x, S, (int)n, nb, cols, tail, act, true, s_); });
  }
  if (rz_partials) vec_dot_partials<T>(b, x, n, nb, act, rz_partials, s_);
}

template void Context::vcycle_csr<float>(int, const float*, float*, int, const int*, c64*, bool);
template void Context::vcycle_csr<double>(int, const double*, double*, int, const int*, c64*,
                                          bool);

// the matrix of a level in canonical CSR form (nnz always; every array
// nullable), its aggregate map (levels below L_s) and its colours
void Context::export_csr(int level, int64_t* nnz, int64_t* row_ptr, int32_t* col_idx,
                         double* vals, int32_t* agg, int32_t* colour) {
  MLMC_REQUIRE(csr_, MLMC_EUNSUPPORTED, "export_csr is for CSR operators");
  MLMC_REQUIRE(level >= 1 && level <= Ls_, MLMC_EINVAL, "level out of range");
  MLMC_REQUIRE(nnz != nullptr, MLMC_EINVAL, "nnz must not be null");
  const Level& L = lv_[level - 1];
  *nnz = L.h_rp.back();
  if (row_ptr) std::copy(L.h_rp.begin(), L.h_rp.end(), row_ptr);
  if (col_idx) std::copy(L.h_ci.begin(), L.h_ci.end(), col_idx);
  if (vals) std::copy(L.h_v.begin(), L.h_v.end(), vals);
  if (agg) {
    MLMC_REQUIRE(level < Ls_, MLMC_EINVAL, "the coarsest level has no aggregates");
    MLMC_REQUIRE(!general_, MLMC_EINVAL, "a hierarchy with given prolongations has no aggregates");
    std::copy(L.h_agg.begin(), L.h_agg.end(), agg);
  }
  if (colour) std::copy(L.h_colour.begin(), L.h_colour.end(), colour);
}

}  // namespace mlmc
