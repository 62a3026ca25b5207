// ILU(0) factorisation and level schedules of the Darcy block (host).
// Compiled without floating-point contraction: the factors equal the
// oracle's bit for bit (same operations in the same order).
#include <algorithm>
#include <cstring>

#include "solver.h"

namespace sd {

namespace {

// Level of every row: forward (lower == true) over the strict lower entries
// in ascending row order, backward over the strict upper entries in
// descending row order.  Returns the level pointers and the rows in level
// order (ascending within a level).
void schedule(const HostCSR& A, const std::vector<int64_t>& diag, bool lower,
              std::vector<int32_t>& ptr, std::vector<int32_t>& ord) {
  const int64_t n = A.n_rows;
  std::vector<int32_t> lev((size_t)n, 0);
  int32_t top = -1;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = lower ? t : n - 1 - t;
    int32_t l = 0;
    const int64_t b = lower ? A.rowptr[i] : diag[i] + 1;
    const int64_t e = lower ? diag[i] : A.rowptr[i + 1];
    for (int64_t k = b; k < e; ++k) l = std::max(l, lev[A.col[k]] + 1);
    lev[i] = l;
    top = std::max(top, l);
  }
  const int32_t nl = top + 1;
  if (nl > kIluMaxLevels)
    throw Error(SD_E_INVALID, "ILU(0): more substitution levels than the device solve supports");
  ptr.assign((size_t)nl + 1, 0);
  for (int64_t i = 0; i < n; ++i) ++ptr[(size_t)lev[i] + 1];
  for (int32_t l = 0; l < nl; ++l) ptr[(size_t)l + 1] += ptr[(size_t)l];
  std::vector<int32_t> next(ptr.begin(), ptr.end() - 1);
  ord.assign((size_t)n, 0);
  for (int64_t i = 0; i < n; ++i) ord[(size_t)next[lev[i]]++] = (int32_t)i;
}

}  // namespace

void ilu0_host(const HostCSR& A, HostIlu& out) {
  const int64_t n = A.n_rows;
  if (A.n_cols != n) throw Error(SD_E_INVALID, "ILU(0) needs a square matrix");
  std::vector<double> f = A.val;
  std::vector<int64_t> diag((size_t)n, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e)
      if (A.col[e] == i) diag[i] = e;
    if (diag[i] < 0) throw Error(SD_E_INVALID, "ILU(0): a row has no diagonal entry");
    if (diag[i] - A.rowptr[i] > kIluWidth || A.rowptr[i + 1] - diag[i] - 1 > kIluWidth)
      throw Error(SD_E_INVALID, "ILU(0): a triangle row is wider than the device solve supports");
  }
  // pos[j] = entry of column j in the current row i (or -1)
  std::vector<int64_t> pos((size_t)n, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) pos[A.col[e]] = e;
    for (int64_t e = A.rowptr[i]; e < diag[i]; ++e) {
      const int32_t k = A.col[e];
      const double ukk = f[diag[k]];
      if (ukk == 0.0) throw Error(SD_E_BREAKDOWN, "ILU(0): zero pivot");
      const double lik = f[e] / ukk;
      f[e] = lik;
      for (int64_t g = diag[k] + 1; g < A.rowptr[k + 1]; ++g) {
        const int64_t h = pos[A.col[g]];
        if (h >= 0) f[h] = f[h] - lik * f[g];
      }
    }
    if (f[diag[i]] == 0.0) throw Error(SD_E_BREAKDOWN, "ILU(0): zero pivot");
    for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e) pos[A.col[e]] = -1;
  }
  out = HostIlu();
  out.n = n;
  schedule(A, diag, true, out.lev_l, out.ord_l);
  schedule(A, diag, false, out.lev_u, out.ord_u);
  const size_t w = (size_t)kIluWidth * (size_t)n;
  out.col_l.assign(w, -1);
  out.col_u.assign(w, -1);
  out.val_l.assign(w, 0.0);
  out.val_u.assign(w, 0.0);
  out.diag_u.assign((size_t)n, 0.0);
  for (int64_t q = 0; q < n; ++q) {
    const int64_t i = out.ord_l[q];
    int k = 0;
    for (int64_t e = A.rowptr[i]; e < diag[i]; ++e, ++k) {
      out.col_l[(size_t)k * n + q] = A.col[e];
      out.val_l[(size_t)k * n + q] = f[e];
    }
    const int64_t u = out.ord_u[q];
    k = 0;
    for (int64_t e = diag[u] + 1; e < A.rowptr[u + 1]; ++e, ++k) {
      out.col_u[(size_t)k * n + q] = A.col[e];
      out.val_u[(size_t)k * n + q] = f[e];
    }
    out.diag_u[q] = f[diag[u]];
  }
}

}  // namespace sd
