// Host setup of the aggregation AMG hierarchy.
//
// The paper's velocity and Darcy sub-solves are one V-cycle of an aggregation
// AMG (Sec. 5, solver setup).  Setup steps, all deterministic:
//   strength   j strong for i iff j != i, same component, and
//              (a_ij*a_ij) >= (theta*theta) * |a_ii*a_jj|; graph symmetrised;
//   roots      maximal independent set of the strength graph (distance 1) or
//              of its square (distance 2) by synchronous Luby rounds, priority
//              (fmix32(i ^ seed(level)), i), seed(level) = 0x9E3779B9 (level+1);
//   aggregates roots numbered in index order; a node with a root neighbour
//              joins the root of largest |a_ij| (ties: smallest index); for
//              distance-2 roots the leftover nodes join, in one synchronous
//              sweep, the aggregate of their aggregated strong neighbour of
//              largest |a_ij| (ties: smallest index);
//   transfer   tentative P[i, agg(i)] = 1, or smoothed
//              P = (I - w D_F^-1 A_F) P_t, A_F = strong entries + a diagonal
//              with the weak entries lumped in (equal row sums),
//              w = 4 / (3 rho), rho = max_i sum_j |a_F,ij| / |a_F,ii|; rows
//              whose lumped diagonal vanishes keep P_t;
//              R = P^T; A_c = R (A P) with Gustavson-ordered sums;
//   coarsest   dense blocked LU with partial pivoting and explicit inverse.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <thread>

#include "sd_internal.h"

namespace sd {

namespace {

thread_local int tl_host_threads = 0;   // set_host_threads of this thread

// Run f(begin, end) over [r0, r1) split into contiguous chunks on threads,
// at least `grain` rows per thread (small ranges run inline: thread start-up
// would cost more than the rows, and concurrent setups share the host).
template <typename F>
void parallel_rows(int64_t r0, int64_t r1, F&& f, int64_t grain = 8192) {
  const int64_t cnt = r1 - r0;
  if (cnt <= 0) return;
  const unsigned cap = tl_host_threads > 0 ? (unsigned)tl_host_threads : 16u;
  const unsigned hw = std::max(1u, std::min(cap, std::thread::hardware_concurrency()));
  const int64_t nt = std::min<int64_t>(hw, cnt / std::max<int64_t>(grain, 1));
  if (nt <= 1) {
    f(r0, r1);
    return;
  }
  std::vector<std::thread> th;
  const int64_t chunk = (cnt + nt - 1) / nt;
  for (int64_t t = 1; t < nt; ++t) {
    const int64_t a = r0 + t * chunk, b = std::min(r1, a + chunk);
    if (a < b) th.emplace_back(f, a, b);
  }
  f(r0, std::min(r1, r0 + chunk));
  for (auto& x : th) x.join();
}

enum : int8_t { UND = 0, ROOT = 1, NONROOT = 2 };

struct Graph {  // adjacency lists with sorted neighbours, no self loops
  std::vector<int64_t> ptr;
  std::vector<int32_t> adj;
};

double diag_of(const HostCSR& A, int64_t r) {
  for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
    if (A.col[k] == r) return A.val[k];
  throw Error(SD_E_INVALID, "AMG: missing diagonal entry");
}

std::vector<uint8_t> strong_mask(const HostCSR& A, const std::vector<int32_t>& comp,
                                 const std::vector<double>& d, double theta) {
  const double th2 = theta * theta;
  std::vector<uint8_t> m((size_t)A.nnz(), 0);
  parallel_rows(0, A.n_rows, [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i) {
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
        const int64_t j = A.col[k];
        const double a = A.val[k];
        m[k] = (j != i) && (comp[i] == comp[j]) && ((a * a) >= th2 * std::fabs(d[i] * d[j]));
      }
    }
  });
  return m;
}

// Rows of a graph built in parallel: build(i, out) appends row i's sorted
// neighbours; row ranges run on threads and are concatenated in order.
template <typename B>
Graph build_graph(int64_t n, B build) {
  struct Part {
    int64_t r0 = 0;
    std::vector<int64_t> len;
    std::vector<int32_t> adj;
  };
  std::vector<Part> parts;
  std::mutex mu;
  parallel_rows(0, n, [&](int64_t r0, int64_t r1) {
    Part pt;
    pt.r0 = r0;
    std::vector<int32_t> tmp;
    for (int64_t i = r0; i < r1; ++i) {
      tmp.clear();
      build(i, tmp);
      pt.len.push_back((int64_t)tmp.size());
      pt.adj.insert(pt.adj.end(), tmp.begin(), tmp.end());
    }
    std::lock_guard<std::mutex> lk(mu);
    parts.push_back(std::move(pt));
  });
  std::sort(parts.begin(), parts.end(), [](const Part& a, const Part& b) { return a.r0 < b.r0; });
  Graph G;
  G.ptr.assign(1, 0);
  for (const Part& pt : parts) {
    for (int64_t l : pt.len) G.ptr.push_back(G.ptr.back() + l);
    G.adj.insert(G.adj.end(), pt.adj.begin(), pt.adj.end());
  }
  return G;
}

Graph symmetric_strength(const HostCSR& A, const std::vector<uint8_t>& m) {
  const int64_t n = A.n_rows;
  // transpose of the strong pattern (counting sort: rows of S^T ascending)
  std::vector<int64_t> tp((size_t)n + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k)
    if (m[k]) ++tp[(size_t)A.col[k] + 1];
  for (int64_t i = 0; i < n; ++i) tp[i + 1] += tp[i];
  std::vector<int32_t> tadj((size_t)tp[n]);
  std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (m[k]) tadj[(size_t)fill[A.col[k]]++] = (int32_t)i;
  return build_graph(n, [&](int64_t i, std::vector<int32_t>& v) {
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (m[k]) v.push_back(A.col[k]);
    for (int64_t k = tp[i]; k < tp[i + 1]; ++k) v.push_back(tadj[k]);
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
  });
}

// Synchronous Luby rounds for a maximal set of nodes at pairwise distance
// greater than dist (1 or 2) in the symmetric graph G: in a round every
// undecided node whose key exceeds the keys of all undecided nodes within
// dist becomes a root, then every undecided node within dist of a new root
// leaves.  Every decision reads the state at the round's start, so the row
// ranges of a phase run on threads.  For dist = 2 the two-hop neighbourhoods
// are never formed: with top[v] the largest undecided key of v's closed
// neighbourhood, node i (undecided) beats everything within two hops iff it
// beats its undecided neighbours and top[j] <= key[i] for each neighbour j;
// and i is within two hops of a new root iff a neighbour j is one or has one
// as a neighbour.
std::vector<int8_t> luby_mis(const Graph& G, int level, int dist) {
  const int64_t n = (int64_t)G.ptr.size() - 1;
  const uint32_t seed = (uint32_t)(0x9E3779B9ull * (uint64_t)(level + 1));
  std::vector<uint64_t> key((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    key[i] = ((uint64_t)fmix32((uint32_t)i ^ seed) << 32) | (uint64_t)i;
  std::vector<int8_t> state((size_t)n, UND);
  std::vector<uint8_t> new_root((size_t)n, 0), near((size_t)n, 0);
  std::vector<uint64_t> top(dist == 2 ? (size_t)n : 0, 0);
  int64_t undecided = n;
  while (undecided > 0) {
    if (dist == 2) {
      // top[v] = max undecided key over v and its neighbours (0: none; every
      // key is positive: fmix32 maps only 0 to 0, and i ^ seed = 0 leaves the
      // index i = seed > 0 in the low half)
      parallel_rows(0, n, [&](int64_t r0, int64_t r1) {
        for (int64_t v = r0; v < r1; ++v) {
          uint64_t t = state[v] == UND ? key[v] : 0;
          for (int64_t k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
            const int32_t u = G.adj[k];
            if (state[u] == UND && key[u] > t) t = key[u];
          }
          top[v] = t;
        }
      });
    }
    parallel_rows(0, n, [&](int64_t r0, int64_t r1) {
      for (int64_t i = r0; i < r1; ++i) {
        new_root[i] = 0;
        if (state[i] != UND) continue;
        bool lost = false;
        for (int64_t k = G.ptr[i]; k < G.ptr[i + 1] && !lost; ++k) {
          const int32_t j = G.adj[k];
          if (dist == 2 ? top[j] > key[i] : (state[j] == UND && key[j] > key[i])) lost = true;
        }
        new_root[i] = !lost;
      }
    });
    for (int64_t i = 0; i < n; ++i)
      if (new_root[i]) state[i] = ROOT;
    if (dist == 2) {
      parallel_rows(0, n, [&](int64_t r0, int64_t r1) {
        for (int64_t v = r0; v < r1; ++v) {
          uint8_t f = new_root[v];
          for (int64_t k = G.ptr[v]; k < G.ptr[v + 1] && !f; ++k) f = new_root[G.adj[k]];
          near[v] = f;
        }
      });
    }
    const std::vector<uint8_t>& hit = dist == 2 ? near : new_root;
    parallel_rows(0, n, [&](int64_t r0, int64_t r1) {
      for (int64_t i = r0; i < r1; ++i) {
        if (state[i] != UND) continue;
        for (int64_t k = G.ptr[i]; k < G.ptr[i + 1]; ++k)
          if (hit[G.adj[k]]) {
            state[i] = NONROOT;
            break;
          }
      }
    });
    undecided = 0;
    for (int64_t i = 0; i < n; ++i) undecided += state[i] == UND;
  }
  return state;
}

// |a_ij| if (i, j) is stored, else 0.
double abs_entry(const HostCSR& A, int64_t i, int32_t j) {
  const int32_t* b = A.col.data() + A.rowptr[i];
  const int32_t* e = A.col.data() + A.rowptr[i + 1];
  const int32_t* p = std::lower_bound(b, e, j);
  if (p != e && *p == j) return std::fabs(A.val[(size_t)(p - A.col.data())]);
  return 0.0;
}

// One synchronous joining sweep (see header comment).
void join_sweep(const HostCSR& A, const Graph& S, const std::vector<uint8_t>& src_ok,
                std::vector<int32_t>& agg) {
  const std::vector<int32_t> before = agg;
  const int64_t n = A.n_rows;
  for (int64_t i = 0; i < n; ++i) {
    if (before[i] >= 0) continue;
    double best_w = -1.0;
    int32_t best_c = -1;
    for (int64_t k = S.ptr[i]; k < S.ptr[i + 1]; ++k) {
      const int32_t c = S.adj[k];
      if (!src_ok[c]) continue;
      const double w = abs_entry(A, i, c);
      if (best_c < 0 || w > best_w) {  // ascending c: ties keep the smaller
        best_w = w;
        best_c = c;
      }
    }
    if (best_c >= 0) agg[i] = before[best_c];
  }
}

HostCSR tentative(const std::vector<int32_t>& agg, int64_t n_c) {
  HostCSR P;
  P.n_rows = (int64_t)agg.size();
  P.n_cols = n_c;
  P.rowptr.resize(agg.size() + 1);
  P.col.resize(agg.size());
  P.val.assign(agg.size(), 1.0);
  for (size_t i = 0; i < agg.size(); ++i) {
    P.rowptr[i] = (int64_t)i;
    P.col[i] = agg[i];
  }
  P.rowptr[agg.size()] = (int64_t)agg.size();
  return P;
}

HostCSR smoothed(const HostCSR& A, const std::vector<uint8_t>& strong,
                 const std::vector<double>& d, const std::vector<int32_t>& agg,
                 int64_t n_c) {
  const int64_t n = A.n_rows;
  // filtered diagonal: a_ii plus the row's weak entries in stored order
  std::vector<double> dF(d);
  std::vector<uint8_t> valid((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (!strong[k] && A.col[k] != i) dF[i] = dF[i] + A.val[k];
    valid[i] = std::fabs(dF[i]) > 1e-8 * std::fabs(d[i]);
  }
  double rho = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (!valid[i]) continue;
    double s = 0.0;
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      if (A.col[k] == i)
        s = s + std::fabs(dF[i]);
      else if (strong[k])
        s = s + std::fabs(A.val[k]);
    }
    const double q = s / std::fabs(dF[i]);
    if (q > rho) rho = q;
  }
  const double wp = rho > 0.0 ? 4.0 / (3.0 * rho) : 0.0;
  HostCSR P;
  P.n_rows = n;
  P.n_cols = n_c;
  P.rowptr.assign(1, 0);
  std::vector<std::pair<int32_t, double>> acc;   // (aggregate, running sum), few per row
  for (int64_t i = 0; i < n; ++i) {
    if (!valid[i]) {
      P.col.push_back(agg[i]);
      P.val.push_back(1.0);
      P.rowptr.push_back((int64_t)P.col.size());
      continue;
    }
    acc.clear();
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      const bool diag = A.col[k] == i;
      if (!(strong[k] || diag)) continue;
      const double v = diag ? dF[i] : A.val[k];
      const int32_t J = agg[A.col[k]];
      size_t q = 0;
      while (q < acc.size() && acc[q].first != J) ++q;
      if (q == acc.size())
        acc.emplace_back(J, 0.0 + v);
      else
        acc[q].second = acc[q].second + v;
    }
    std::sort(acc.begin(), acc.end());
    const double coef = wp / dF[i];
    for (auto& e : acc) {
      const double base = (e.first == agg[i]) ? 1.0 : 0.0;
      P.col.push_back(e.first);
      P.val.push_back(base - coef * e.second);
    }
    P.rowptr.push_back((int64_t)P.col.size());
  }
  return P;
}

HostCSR transpose(const HostCSR& P) {
  HostCSR R;
  R.n_rows = P.n_cols;
  R.n_cols = P.n_rows;
  R.rowptr.assign((size_t)R.n_rows + 1, 0);
  for (int32_t c : P.col) R.rowptr[(size_t)c + 1]++;
  for (int64_t r = 0; r < R.n_rows; ++r) R.rowptr[r + 1] += R.rowptr[r];
  R.col.resize(P.col.size());
  R.val.resize(P.val.size());
  std::vector<int64_t> pos(R.rowptr.begin(), R.rowptr.end() - 1);
  for (int64_t i = 0; i < P.n_rows; ++i)  // ascending i keeps R's columns sorted
    for (int64_t k = P.rowptr[i]; k < P.rowptr[i + 1]; ++k) {
      const int64_t dst = pos[P.col[k]]++;
      R.col[dst] = (int32_t)i;
      R.val[dst] = P.val[k];
    }
  return R;
}



// Gustavson product: (XY)[i, J] accumulates x_ik * y_kJ over ascending k,
// then over Y's row k in ascending J.  Structural pattern, zeros kept.  Rows
// are independent: contiguous row ranges run on threads, each row summed in
// the same order as a serial loop, so the result does not depend on the
// thread count.  The rows per thread follow the work: products with few,
// long rows (the Galerkin and fused-transfer products on coarse levels) get
// small row ranges.
HostCSR spgemm(const HostCSR& X, const HostCSR& Y) {
  struct Part {
    int64_t r0 = 0;
    std::vector<int64_t> len;
    std::vector<int32_t> col;
    std::vector<double> val;
  };
  int64_t products = 0;
  for (int64_t k = 0; k < X.nnz(); ++k) products += Y.rowptr[X.col[k] + 1] - Y.rowptr[X.col[k]];
  constexpr int64_t kProductsPerThread = 1 << 18;
  const int64_t grain = std::max<int64_t>(
      64, std::min<int64_t>(8192, X.n_rows * kProductsPerThread / std::max<int64_t>(products, 1)));
  std::vector<Part> parts;
  std::mutex mu;
  parallel_rows(0, X.n_rows, [&](int64_t r0, int64_t r1) {
    Part pt;
    pt.r0 = r0;
    std::vector<double> acc((size_t)Y.n_cols, 0.0);
    std::vector<int64_t> mark((size_t)Y.n_cols, -1);
    std::vector<int32_t> cols;
    for (int64_t i = r0; i < r1; ++i) {
      cols.clear();
      for (int64_t k = X.rowptr[i]; k < X.rowptr[i + 1]; ++k) {
        const int32_t kk = X.col[k];
        const double xv = X.val[k];
        for (int64_t l = Y.rowptr[kk]; l < Y.rowptr[kk + 1]; ++l) {
          const int32_t J = Y.col[l];
          const double prod = xv * Y.val[l];
          if (mark[J] != i) {
            mark[J] = i;
            acc[J] = 0.0 + prod;
            cols.push_back(J);
          } else {
            acc[J] = acc[J] + prod;
          }
        }
      }
      std::sort(cols.begin(), cols.end());
      for (int32_t J : cols) {
        pt.col.push_back(J);
        pt.val.push_back(acc[J]);
      }
      pt.len.push_back((int64_t)cols.size());
    }
    std::lock_guard<std::mutex> lk(mu);
    parts.push_back(std::move(pt));
  }, grain);
  std::sort(parts.begin(), parts.end(), [](const Part& a, const Part& b) { return a.r0 < b.r0; });
  HostCSR Z;
  Z.n_rows = X.n_rows;
  Z.n_cols = Y.n_cols;
  Z.rowptr.assign(1, 0);
  for (const Part& pt : parts) {
    for (int64_t l : pt.len) Z.rowptr.push_back(Z.rowptr.back() + l);
    Z.col.insert(Z.col.end(), pt.col.begin(), pt.col.end());
    Z.val.insert(Z.val.end(), pt.val.begin(), pt.val.end());
  }
  return Z;
}

// Blocked right-looking LU with partial pivoting (row interchanges), then the
// explicit inverse from L U X = P I.  Rows of each update are independent, so
// the result does not depend on the thread count.
void dense_inverse(std::vector<double>& M, int64_t n, std::vector<double>& inv) {
  // rows of the dense updates are long: small chunks pay off above n ~ 512
  const int64_t dense_grain = n >= 512 ? 64 : n + 1;
  const int64_t NB = 64;
  std::vector<int64_t> piv((size_t)n);
  for (int64_t kb = 0; kb < n; kb += NB) {
    const int64_t ke = std::min(n, kb + NB);
    for (int64_t k = kb; k < ke; ++k) {
      int64_t p = k;
      double best = std::fabs(M[k * n + k]);
      for (int64_t r = k + 1; r < n; ++r)
        if (std::fabs(M[r * n + k]) > best) {
          best = std::fabs(M[r * n + k]);
          p = r;
        }
      if (!(best > 0.0) || !std::isfinite(best))
        throw Error(SD_E_BREAKDOWN, "AMG: singular coarsest operator");
      piv[k] = p;
      if (p != k)
        for (int64_t c = 0; c < n; ++c) std::swap(M[k * n + c], M[p * n + c]);
      const double inv_piv = 1.0 / M[k * n + k];
      for (int64_t r = k + 1; r < n; ++r) {
        const double l = M[r * n + k] * inv_piv;
        M[r * n + k] = l;
        if (l != 0.0)
          for (int64_t c = k + 1; c < ke; ++c) M[r * n + c] -= l * M[k * n + c];
      }
    }
    // U12 = L11^-1 A12 (unit lower triangular)
    for (int64_t k = kb; k < ke; ++k)
      for (int64_t r = k + 1; r < ke; ++r) {
        const double l = M[r * n + k];
        if (l != 0.0)
          for (int64_t c = ke; c < n; ++c) M[r * n + c] -= l * M[k * n + c];
      }
    // A22 -= L21 U12
    parallel_rows(ke, n, [&](int64_t a, int64_t b) {
      for (int64_t r = a; r < b; ++r)
        for (int64_t k = kb; k < ke; ++k) {
          const double l = M[r * n + k];
          if (l == 0.0) continue;
          double* dst = &M[r * n];
          const double* src = &M[k * n];
          for (int64_t c = ke; c < n; ++c) dst[c] -= l * src[c];
        }
    }, dense_grain);
  }
  std::vector<int64_t> perm((size_t)n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t k = 0; k < n; ++k) std::swap(perm[k], perm[piv[k]]);
  // A^-1 = U^-1 L^-1 P: B = U^-1 L^-1 column block by column block (columns
  // are independent), rows in blocks of NB so that each source row is applied
  // to a block of rows held in cache; then the columns are permuted.
  std::vector<double> B((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i) B[i * n + i] = 1.0;
  parallel_rows(0, n, [&](int64_t c0, int64_t c1) {
    // forward: unit lower L; column c of L^-1 vanishes above row c
    for (int64_t rb0 = c0; rb0 < n; rb0 += NB) {
      const int64_t rb1 = std::min(n, rb0 + NB);
      for (int64_t k = c0; k < rb1; ++k) {
        const int64_t ce = std::min(c1, k + 1);
        const double* src = &B[k * n];
        for (int64_t r = std::max(rb0, k + 1); r < rb1; ++r) {
          const double l = M[r * n + k];
          if (l == 0.0) continue;
          double* dst = &B[r * n];
          for (int64_t c = c0; c < ce; ++c) dst[c] -= l * src[c];
        }
      }
    }
    // backward: U, rows in descending blocks
    for (int64_t rb1 = n; rb1 > 0; rb1 -= NB) {
      const int64_t rb0 = std::max<int64_t>(0, rb1 - NB);
      for (int64_t k = n - 1; k >= rb1; --k) {
        const double* src = &B[k * n];
        for (int64_t r = rb0; r < rb1; ++r) {
          const double u = M[r * n + k];
          if (u == 0.0) continue;
          double* dst = &B[r * n];
          for (int64_t c = c0; c < c1; ++c) dst[c] -= u * src[c];
        }
      }
      for (int64_t r = rb1 - 1; r >= rb0; --r) {
        double* dst = &B[r * n];
        for (int64_t k = r + 1; k < rb1; ++k) {
          const double u = M[r * n + k];
          if (u == 0.0) continue;
          const double* src = &B[k * n];
          for (int64_t c = c0; c < c1; ++c) dst[c] -= u * src[c];
        }
        const double d = M[r * n + r];
        for (int64_t c = c0; c < c1; ++c) dst[c] /= d;
      }
    }
  }, dense_grain);
  inv.assign((size_t)(n * n), 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t r = 0; r < n; ++r) inv[i * n + perm[r]] = B[i * n + r];
}

}  // namespace

namespace {

// X + alpha Y (union pattern, rows sorted by column).
HostCSR add_scaled(const HostCSR& X, const HostCSR& Y, double alpha) {
  HostCSR Z;
  Z.n_rows = X.n_rows;
  Z.n_cols = X.n_cols;
  Z.rowptr.assign(1, 0);
  for (int64_t i = 0; i < X.n_rows; ++i) {
    int64_t a = X.rowptr[i], ae = X.rowptr[i + 1], b = Y.rowptr[i], be = Y.rowptr[i + 1];
    while (a < ae || b < be) {
      if (b >= be || (a < ae && X.col[a] < Y.col[b])) {
        Z.col.push_back(X.col[a]);
        Z.val.push_back(X.val[a]);
        ++a;
      } else if (a >= ae || Y.col[b] < X.col[a]) {
        Z.col.push_back(Y.col[b]);
        Z.val.push_back(alpha * Y.val[b]);
        ++b;
      } else {
        Z.col.push_back(X.col[a]);
        Z.val.push_back(X.val[a] + alpha * Y.val[b]);
        ++a;
        ++b;
      }
    }
    Z.rowptr.push_back((int64_t)Z.col.size());
  }
  return Z;
}

// diag(s) X (rows scaled) or X diag(s) (columns scaled).
HostCSR scale_rows(HostCSR X, const std::vector<double>& s) {
  for (int64_t i = 0; i < X.n_rows; ++i)
    for (int64_t k = X.rowptr[i]; k < X.rowptr[i + 1]; ++k) X.val[k] = s[i] * X.val[k];
  return X;
}
HostCSR scale_cols(HostCSR X, const std::vector<double>& s) {
  for (size_t k = 0; k < X.col.size(); ++k) X.val[k] = X.val[k] * s[X.col[k]];
  return X;
}

std::vector<double> jacobi_weights(const HostCSR& A, double omega) {
  std::vector<double> w((size_t)A.n_rows);
  for (int64_t i = 0; i < A.n_rows; ++i) w[i] = omega / diag_of(A, i);
  return w;
}

}  // namespace

HostCSR scaled_product(const HostCSR& X, const std::vector<double>& s, const HostCSR& Y) {
  return spgemm(scale_cols(X, s), Y);
}

HostCSR sparse_product(const HostCSR& X, const HostCSR& Y) { return spgemm(X, Y); }

HostCSR presmoothed_restriction(const HostCSR& A, const HostCSR& R, const HostCSR& RA,
                                double omega) {
  const std::vector<double> w = jacobi_weights(A, omega);
  const HostCSR T = scale_cols(A, w);                 // A W
  // R (I - A M2) = R - 2 R A W + (R A W)(A W), the product with R first
  const HostCSR RAW = scale_cols(RA, w);
  return add_scaled(add_scaled(R, RAW, -2.0), spgemm(RAW, T), 1.0);
}

HostCSR presmoothed_restriction(const HostCSR& A, const HostCSR& R, double omega) {
  return presmoothed_restriction(A, R, spgemm(R, A), omega);
}

HostCSR smoothed_correction(const HostCSR& A, const HostCSR& P, const HostCSR& AP,
                            double omega) {
  const std::vector<double> w = jacobi_weights(A, omega);
  return add_scaled(P, scale_rows(AP, w), -1.0);
}

void parallel_ranges(int64_t r0, int64_t r1, const std::function<void(int64_t, int64_t)>& f) {
  parallel_rows(r0, r1, f);
}

void set_host_threads(int n) { tl_host_threads = std::max(0, n); }

HostCSR residual_restriction(const HostCSR& A, const HostCSR& R) {
  return residual_restriction(A, R, spgemm(R, A));
}

HostCSR residual_restriction(const HostCSR& A, const HostCSR& R, const HostCSR& RA) {
  HostCSR Q;
  Q.n_rows = R.n_rows;
  Q.n_cols = 2 * A.n_cols;
  Q.rowptr.assign(1, 0);
  Q.col.reserve((size_t)(R.nnz() + RA.nnz()));
  Q.val.reserve((size_t)(R.nnz() + RA.nnz()));
  for (int64_t i = 0; i < R.n_rows; ++i) {
    for (int64_t k = R.rowptr[i]; k < R.rowptr[i + 1]; ++k) {
      Q.col.push_back(R.col[k]);
      Q.val.push_back(R.val[k]);
    }
    for (int64_t k = RA.rowptr[i]; k < RA.rowptr[i + 1]; ++k) {
      Q.col.push_back((int32_t)(A.n_cols + RA.col[k]));
      Q.val.push_back(-RA.val[k]);
    }
    Q.rowptr.push_back((int64_t)Q.col.size());
  }
  return Q;
}

void amg_setup_host(const HostCSR& A0, const std::vector<int32_t>& comp0, bool singular,
                    const AMGOpts& o, HostHierarchy& h) {
  if (o.mis != 1 && o.mis != 2) throw Error(SD_E_INVALID, "AMG: mis must be 1 or 2");
  if (!(o.theta >= 0.0) || !(o.omega > 0.0) || o.coarse_max < 1 || o.max_levels < 1 ||
      o.nu_pre < 0 || o.nu_post < 0)
    throw Error(SD_E_INVALID, "AMG: bad options");
  h.levels.clear();
  h.levels.emplace_back();
  h.levels[0].A = A0;
  h.levels[0].comp = comp0;
  // Strength threshold of the current level: halved for this level and the
  // coarser ones whenever aggregation would shrink a level by less than a
  // factor of 2 (the level-dependent threshold of smoothed aggregation, Vanek,
  // Mandel, Brezina 1996, applied where coarsening stalls, as on the wide
  // Galerkin stencils of 3-D hierarchies); at most 6 halvings; below
  // min_ratio the hierarchy ends.
  double theta = o.theta;
  while (h.levels.back().A.n_rows > o.coarse_max && (int)h.levels.size() < o.max_levels) {
    const int lev = (int)h.levels.size() - 1;
    const HostCSR& A = h.levels.back().A;
    const std::vector<int32_t>& comp = h.levels.back().comp;
    const int64_t n = A.n_rows;
    std::vector<double> d((size_t)n);
    for (int64_t i = 0; i < n; ++i) d[i] = diag_of(A, i);
    std::vector<uint8_t> strong = strong_mask(A, comp, d, theta);
    Graph S = symmetric_strength(A, strong);
    std::vector<int8_t> state = luby_mis(S, lev, o.mis);
    std::vector<int32_t> agg((size_t)n, -1);
    std::vector<int32_t> roots;
    for (int64_t i = 0; i < n; ++i)
      if (state[i] == ROOT) {
        agg[i] = (int32_t)roots.size();
        roots.push_back((int32_t)i);
      }
    std::vector<uint8_t> ok((size_t)n);
    for (int64_t i = 0; i < n; ++i) ok[i] = state[i] == ROOT;
    join_sweep(A, S, ok, agg);
    if (o.mis == 2) {
      for (int64_t i = 0; i < n; ++i) ok[i] = agg[i] >= 0;
      join_sweep(A, S, ok, agg);
    }
    for (int64_t i = 0; i < n; ++i)
      if (agg[i] < 0) throw Error(SD_E_INVALID, "AMG: node left without an aggregate");
    const int64_t n_c = (int64_t)roots.size();
    if ((double)n < 2.0 * (double)n_c && theta > o.theta / 64.0) {
      theta = theta / 2.0;
      continue;
    }
    if ((double)n < o.min_ratio * (double)n_c) break;
    HostLevel& L = h.levels.back();
    L.P = o.smoothed ? smoothed(A, strong, d, agg, n_c) : tentative(agg, n_c);
    L.R = transpose(L.P);
    L.AP = spgemm(A, L.P);
    HostLevel next;
    next.A = spgemm(L.R, L.AP);
    next.comp.resize((size_t)n_c);
    for (int64_t c = 0; c < n_c; ++c) next.comp[c] = comp[roots[c]];
    L.agg = std::move(agg);
    h.levels.push_back(std::move(next));
  }
  const HostCSR& Ac = h.levels.back().A;
  const int64_t nc = Ac.n_rows;
  if (nc > 4096) throw Error(SD_E_INVALID, "AMG: coarsest level too large for a dense solve");
  std::vector<double> M((size_t)(nc * nc), 0.0);
  for (int64_t r = 0; r < nc; ++r)
    for (int64_t k = Ac.rowptr[r]; k < Ac.rowptr[r + 1]; ++k) M[r * nc + Ac.col[k]] = Ac.val[k];
  if (singular) {
    double tr = 0.0;
    for (int64_t r = 0; r < nc; ++r) tr += M[r * nc + r];
    const double s = tr / (double)(nc * nc);
    for (auto& m : M) m = m + s;
  }
  dense_inverse(M, nc, h.Ainv);
  h.n_coarse = nc;
}

}  // namespace sd
