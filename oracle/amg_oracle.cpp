// FP64 CPU oracle for smoothed-aggregation AMG-preconditioned CG and
// BiCGSTAB and their adjoints.  TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check
// and the benchmark's CPU-baseline leg load this library; the product path
// never does.  It shares no code, header or table with the HIP library.
//
// Plain and slow on purpose; the setup is sequential, and the solve loops
// run on one thread unless or_set_threads asks for more (OpenMP over rows
// and over fixed dot-product blocks, so results never depend on the thread
// count).  Every step follows the method as the
// paper fixes it where it speaks (adjoint, Eq. (1); matrix-value and RHS
// gradients, Eq. (2); setup reuse on a fixed pattern, Section 2.1 "C++/CUDA
// backend"; iteration count / final residual / status diagnostics, Section
// 2.2) and, where the paper delegates the numerical method to its backend,
// the smoothed-aggregation definition written out below (strength graph,
// distance-2 maximal independent set roots in decreasing-key order,
// aggregates, smoothed prolongator, Galerkin product, damped-Jacobi V(1,1),
// PCG; for a nonsymmetric A: an LU coarse solve, right-preconditioned
// BiCGSTAB -- the paper's default solver, Section 2.1 -- and an adjoint on the
// explicit transpose, Section 2.1 with Eq. (1)).
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC (no FMA
// contraction: every product and sum is rounded on its own).
//
// Parity pins: see the oracle tests (closed-form Laplacian spectrum,
// manufactured eigenvector solutions, brute-force MIS-2 characterisation,
// dense Galerkin products, dense V-cycle symmetry/SPD, SciPy CG iterates,
// dense adjoint gradients and central finite differences; SciPy BiCGSTAB
// iterates, LAPACK LU and inverses, dense nonsymmetric adjoints).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

enum {
  OR_OK = 0,
  OR_NOT_CONVERGED = 1,
  OR_ERR_INVALID_ARG = -1,
  OR_ERR_ZERO_DIAG = -2,
  OR_ERR_PATTERN_MISMATCH = -3,
  OR_ERR_BREAKDOWN = -4,
  OR_ERR_COARSE_TOO_LARGE = -7,
};

// Largest coarsest level that gets a dense factorization; a hierarchy whose
// coarsening stalls above this size is rejected instead.
constexpr int kMaxDenseCoarse = 2048;

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
  int64_t nnz() const { return (int64_t)ci.size(); }
};

struct Params {
  double theta;
  int max_coarse;
  int max_levels;
  int smoother;  // 0 damped Jacobi, 1 L1-Jacobi
  double omega;
  int nu_pre, nu_post;
  int symmetric;  // 1: Cholesky coarse factor; 0: LU with partial pivoting
};

struct Level {
  Csr A;
  std::vector<double> dinv;   // 1 / a_ii
  std::vector<double> sw;     // smoother weight per row: omega*dinv (Jacobi) or 1/sum|a_ij| (L1); see smooth_weight()
  Csr G;                      // strength graph (no diagonal, symmetric)
  std::vector<int> agg;       // fine node -> aggregate (only if not coarsest)
  int nagg = 0;
  double rho = 0.0, omegaP = 0.0;
  Csr P, R;
};

struct Hier {
  Params prm;
  std::vector<Level> lv;        // lv.back() is the coarsest level
  std::vector<double> L;        // dense factor of the coarsest A, row-major: Cholesky (lower) or packed LU
  std::vector<int> piv;         // LU only: row exchanged with row k at elimination step k
  int nL = 0;
};

// ---------------------------------------------------------------- utilities

// MurmurHash3 32-bit finalizer (public domain, Appleby).
uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Node priority for the maximal independent set: hash in the high word,
// index in the low word, so keys are distinct.
uint64_t node_key(int i) { return ((uint64_t)fmix32((uint32_t)i) << 32) | (uint64_t)(uint32_t)i; }

int validate_csr(int n, const int* rp, const int* ci) {
  if (n <= 0 || !rp || !ci) return OR_ERR_INVALID_ARG;
  if (rp[0] != 0) return OR_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return OR_ERR_INVALID_ARG;
    bool has_diag = false;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= n) return OR_ERR_INVALID_ARG;
      if (k > rp[i] && ci[k] <= ci[k - 1]) return OR_ERR_INVALID_ARG;  // unsorted or duplicate
      if (ci[k] == i) has_diag = true;
    }
    if (!has_diag) return OR_ERR_ZERO_DIAG;
  }
  return OR_OK;
}

double diag_of(const Csr& A, int i) {
  for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
    if (A.ci[k] == i) return A.v[k];
  return 0.0;
}

// Threads of the solve loops (or_set_threads; default 1).  Only loops whose
// results do not depend on how rows are shared out run in parallel: row-wise
// products and element-wise updates, and dot products over fixed blocks.
int g_threads = 1;
constexpr int kParMin = 16384;  // shorter loops stay on one thread

// y = A x, each row summed in stored order from +0.0.
void spmv(const Csr& A, const double* x, double* y) {
#pragma omp parallel for schedule(static) num_threads(g_threads) if (A.nrows >= kParMin)
  for (int i = 0; i < A.nrows; ++i) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * x[A.ci[k]];
    y[i] = s;
  }
}

// <a, b> over fixed blocks of kDotBlock elements: each block summed in index
// order from +0.0, then the block sums in block order.  The blocks do not
// depend on the thread count, so neither does the result; a vector of at
// most kDotBlock elements is one block (the plain sequential sum).
constexpr int kDotBlock = 8192;
double dot(const std::vector<double>& a, const std::vector<double>& b) {
  const int64_t n = (int64_t)a.size();
  const int64_t nb = (n + kDotBlock - 1) / kDotBlock;
  std::vector<double> part(std::max<int64_t>(nb, 1), 0.0);
#pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
  for (int64_t k = 0; k < nb; ++k) {
    double s = 0.0;
    const int64_t e = std::min(n, (k + 1) * kDotBlock);
    for (int64_t i = k * kDotBlock; i < e; ++i) s += a[i] * b[i];
    part[k] = s;
  }
  double s = 0.0;
  for (int64_t k = 0; k < nb; ++k) s += part[k];
  return s;
}

// ------------------------------------------------------------- setup steps

// Strength graph: off-diagonal entries (all of them when theta == 0, else
// |a_ij| >= theta*sqrt(|a_ii a_jj|)), then symmetrised (G union G^T), rows
// sorted, no duplicates.
Csr strength_graph(const Csr& A, double theta) {
  int n = A.nrows;
  std::vector<std::vector<int>> adj(n);
  for (int i = 0; i < n; ++i) {
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int j = A.ci[k];
      if (j == i) continue;
      bool strong = true;
      if (theta > 0.0) strong = std::fabs(A.v[k]) >= theta * std::sqrt(std::fabs(diag_of(A, i) * diag_of(A, j)));
      if (strong) {
        adj[i].push_back(j);
        adj[j].push_back(i);
      }
    }
  }
  Csr G;
  G.nrows = G.ncols = n;
  G.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    std::sort(adj[i].begin(), adj[i].end());
    adj[i].erase(std::unique(adj[i].begin(), adj[i].end()), adj[i].end());
    G.rp[i + 1] = G.rp[i] + (int)adj[i].size();
  }
  G.ci.reserve(G.rp[n]);
  for (int i = 0; i < n; ++i) G.ci.insert(G.ci.end(), adj[i].begin(), adj[i].end());
  return G;
}

// Aggregation.  Roots: greedy maximal distance-2 independent set in
// decreasing key order (a node is a root iff no root within graph distance 2
// has a larger key).  Aggregate numbers: roots ranked by ascending index.
// Every non-root adjacent to a root joins that root (unique: roots are at
// least 3 apart).  Every remaining node joins the smallest aggregate number
// among its neighbours assigned in the previous step.
int aggregate(const Csr& G, std::vector<int>& agg) {
  int n = G.nrows;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [](int a, int b) { return node_key(a) > node_key(b); });
  std::vector<char> excluded(n, 0), root(n, 0);
  for (int t = 0; t < n; ++t) {
    int i = order[t];
    if (excluded[i]) continue;
    root[i] = 1;
    excluded[i] = 1;
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      int j = G.ci[k];
      excluded[j] = 1;
      for (int m = G.rp[j]; m < G.rp[j + 1]; ++m) excluded[G.ci[m]] = 1;
    }
  }
  agg.assign(n, -1);
  int nagg = 0;
  for (int i = 0; i < n; ++i)
    if (root[i]) agg[i] = nagg++;
  std::vector<int> agg2 = agg;  // after the neighbour-of-root step
  for (int i = 0; i < n; ++i) {
    if (root[i]) continue;
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k)
      if (root[G.ci[k]]) { agg2[i] = agg[G.ci[k]]; break; }
  }
  std::vector<int> agg3 = agg2;
  for (int i = 0; i < n; ++i) {
    if (agg2[i] >= 0) continue;
    int best = -1;
    for (int k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      int a = agg2[G.ci[k]];
      if (a >= 0 && (best < 0 || a < best)) best = a;
    }
    agg3[i] = best;  // maximality guarantees best >= 0
  }
  agg = agg3;
  return nagg;
}

// Gershgorin bound of rho(D^-1 A): max_i (sum_j |a_ij|) / |a_ii|.
double gershgorin_rho(const Csr& A) {
  double rho = 0.0;
  for (int i = 0; i < A.nrows; ++i) {
    double s = 0.0, d = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      s += std::fabs(A.v[k]);
      if (A.ci[k] == i) d = A.v[k];
    }
    double r = s / std::fabs(d);
    if (r > rho) rho = r;
  }
  return rho;
}

// Smoothed prolongator P = (I - omegaP D^-1 A) T with T the 0/1 aggregate
// indicator.  Row i: w = omegaP / a_ii; for every aggregate J touched by
// row i, s_J = sum over j in row i with agg(j) == J (stored order, from
// +0.0); P_iJ = [J == agg(i)] - w*s_J.  Columns ascending; every touched
// aggregate is kept.
Csr smoothed_prolongator(const Csr& A, const std::vector<int>& agg, int nagg, double omegaP) {
  int n = A.nrows;
  Csr P;
  P.nrows = n;
  P.ncols = nagg;
  P.rp.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    std::vector<int> Js;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) Js.push_back(agg[A.ci[k]]);
    std::sort(Js.begin(), Js.end());
    Js.erase(std::unique(Js.begin(), Js.end()), Js.end());
    double w = omegaP / diag_of(A, i);
    for (int J : Js) {
      double s = 0.0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (agg[A.ci[k]] == J) s += A.v[k];
      double delta = (J == agg[i]) ? 1.0 : 0.0;
      double ws = w * s;
      P.ci.push_back(J);
      P.v.push_back(delta - ws);
    }
    P.rp[i + 1] = (int)P.ci.size();
  }
  return P;
}

// Explicit transpose; each row of the result lists source rows ascending.
Csr transpose(const Csr& P) {
  Csr R;
  R.nrows = P.ncols;
  R.ncols = P.nrows;
  R.rp.assign(R.nrows + 1, 0);
  for (int k = 0; k < (int)P.ci.size(); ++k) R.rp[P.ci[k] + 1]++;
  for (int I = 0; I < R.nrows; ++I) R.rp[I + 1] += R.rp[I];
  R.ci.resize(P.ci.size());
  R.v.resize(P.v.size());
  std::vector<int> fill(R.rp.begin(), R.rp.end() - 1);
  for (int i = 0; i < P.nrows; ++i)
    for (int k = P.rp[i]; k < P.rp[i + 1]; ++k) {
      int J = P.ci[k];
      R.ci[fill[J]] = i;
      R.v[fill[J]] = P.v[k];
      fill[J]++;
    }
  return R;
}

// C = X * Y in canonical order: row i of C accumulates, for every k of row i
// of X in ascending order and every J of row k of Y in ascending order,
// acc[J] += x_ik * y_kJ (product rounded, then sum rounded, acc from +0.0).
// Every touched column is stored, ascending.
Csr spgemm(const Csr& X, const Csr& Y) {
  Csr C;
  C.nrows = X.nrows;
  C.ncols = Y.ncols;
  C.rp.assign(C.nrows + 1, 0);
  std::vector<double> acc(Y.ncols, 0.0);
  std::vector<int> mark(Y.ncols, -1);
  for (int i = 0; i < X.nrows; ++i) {
    std::vector<int> cols;
    for (int a = X.rp[i]; a < X.rp[i + 1]; ++a) {
      int k = X.ci[a];
      double xv = X.v[a];
      for (int b = Y.rp[k]; b < Y.rp[k + 1]; ++b) {
        int J = Y.ci[b];
        if (mark[J] != i) {
          mark[J] = i;
          acc[J] = 0.0;
          cols.push_back(J);
        }
        acc[J] += xv * Y.v[b];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int J : cols) {
      C.ci.push_back(J);
      C.v.push_back(acc[J]);
    }
    C.rp[i + 1] = (int)C.ci.size();
  }
  return C;
}

void level_numerics(Level& L, const Params& prm) {
  const Csr& A = L.A;
  int n = A.nrows;
  L.dinv.resize(n);
  L.sw.resize(n);
  for (int i = 0; i < n; ++i) {
    L.dinv[i] = 1.0 / diag_of(A, i);
    if (prm.smoother == 1) {
      double s = 0.0;
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
      L.sw[i] = 1.0 / s;
    } else {
      L.sw[i] = prm.omega * L.dinv[i];
    }
  }
}

// Dense Cholesky of the coarsest matrix, right-looking, column by column.
int coarse_factor(Hier& H) {
  const Csr& A = H.lv.back().A;
  int n = A.nrows;
  if (n > kMaxDenseCoarse) return OR_ERR_COARSE_TOO_LARGE;
  H.nL = n;
  std::vector<double> W((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) W[(size_t)i * n + A.ci[k]] = A.v[k];
  for (int k = 0; k < n; ++k) {
    double d = W[(size_t)k * n + k];
    if (!(d > 0.0)) return OR_ERR_BREAKDOWN;
    double lkk = std::sqrt(d);
    W[(size_t)k * n + k] = lkk;
    for (int i = k + 1; i < n; ++i) W[(size_t)i * n + k] /= lkk;
    for (int j = k + 1; j < n; ++j)
      for (int i = j; i < n; ++i) W[(size_t)i * n + j] -= W[(size_t)i * n + k] * W[(size_t)j * n + k];
  }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) W[(size_t)i * n + j] = 0.0;
  H.L = W;
  return OR_OK;
}

// Dense LU with partial pivoting of the coarsest matrix (Gaussian
// elimination with row interchanges, one column at a time): at step k the
// pivot is the first row i >= k of largest |w_ik|; rows k and pivot are
// exchanged over the full width, the multipliers w_ik / w_kk are stored below
// the diagonal, and every w_ij with i, j > k loses multiplier times w_kj.
int coarse_lu(Hier& H) {
  const Csr& A = H.lv.back().A;
  int n = A.nrows;
  if (n > kMaxDenseCoarse) return OR_ERR_COARSE_TOO_LARGE;
  H.nL = n;
  std::vector<double> W((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) W[(size_t)i * n + A.ci[k]] = A.v[k];
  H.piv.assign(n, 0);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::fabs(W[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double a = std::fabs(W[(size_t)i * n + k]);
      if (a > best) { best = a; p = i; }
    }
    if (!(best > 0.0)) return OR_ERR_BREAKDOWN;  // singular (or NaN) coarse matrix
    H.piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(W[(size_t)k * n + j], W[(size_t)p * n + j]);
    double ukk = W[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) W[(size_t)i * n + k] = W[(size_t)i * n + k] / ukk;
    for (int i = k + 1; i < n; ++i) {
      double l = W[(size_t)i * n + k];
      for (int j = k + 1; j < n; ++j) W[(size_t)i * n + j] = W[(size_t)i * n + j] - l * W[(size_t)k * n + j];
    }
  }
  H.L = W;
  return OR_OK;
}

void coarse_solve(const Hier& H, const double* b, double* x) {
  int n = H.nL;
  const std::vector<double>& L = H.L;
  if (!H.prm.symmetric) {
    // P A = L U: y = P b, L y' = y (unit lower), U x = y'
    std::vector<double> y(b, b + n);
    for (int k = 0; k < n; ++k) std::swap(y[k], y[H.piv[k]]);
    for (int i = 0; i < n; ++i) {
      double s = y[i];
      for (int j = 0; j < i; ++j) s -= L[(size_t)i * n + j] * y[j];
      y[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = y[i];
      for (int j = i + 1; j < n; ++j) s -= L[(size_t)i * n + j] * x[j];
      x[i] = s / L[(size_t)i * n + i];
    }
    return;
  }
  std::vector<double> y(n);
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int j = 0; j < i; ++j) s -= L[(size_t)i * n + j] * y[j];
    y[i] = s / L[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = y[i];
    for (int j = i + 1; j < n; ++j) s -= L[(size_t)j * n + i] * x[j];
    x[i] = s / L[(size_t)i * n + i];
  }
}

// Build (or, with frozen aggregates, rebuild the values of) the hierarchy.
int build_levels(Hier& H, bool refresh) {
  const Params& prm = H.prm;
  size_t l = 0;
  for (;;) {
    Level& L = H.lv[l];
    level_numerics(L, prm);
    bool last;
    if (refresh) {
      last = (l + 1 == H.lv.size());
    } else {
      last = L.A.nrows <= prm.max_coarse || (int)(l + 1) >= prm.max_levels;
      if (!last) {
        L.G = strength_graph(L.A, prm.theta);
        L.nagg = aggregate(L.G, L.agg);
        if (10LL * L.nagg > 9LL * L.A.nrows) last = true;
      }
    }
    if (last) {
      L.agg.clear();
      L.nagg = 0;
      L.P = Csr();
      L.R = Csr();
      break;
    }
    L.rho = gershgorin_rho(L.A);
    L.omegaP = (4.0 / 3.0) / L.rho;
    L.P = smoothed_prolongator(L.A, L.agg, L.nagg, L.omegaP);
    L.R = transpose(L.P);
    Csr AP = spgemm(L.A, L.P);
    Csr Ac = spgemm(L.R, AP);
    if (refresh) {
      if (Ac.ci != H.lv[l + 1].A.ci || Ac.rp != H.lv[l + 1].A.rp) return OR_ERR_PATTERN_MISMATCH;
      H.lv[l + 1].A.v = Ac.v;
    } else {
      H.lv.emplace_back();
      H.lv.back().A = std::move(Ac);
    }
    ++l;
  }
  return prm.symmetric ? coarse_factor(H) : coarse_lu(H);
}

// ---------------------------------------------------------------- solve

// Damped-Jacobi (or L1) V(nu_pre, nu_post) cycle, recursive.
void vcycle(const Hier& H, size_t l, const double* b, double* x) {
  if (l + 1 == H.lv.size()) {
    coarse_solve(H, b, x);
    return;
  }
  const Level& L = H.lv[l];
  int n = L.A.nrows;
  std::vector<double> Ax(n), r(n);
  const bool par = n >= kParMin;
  (void)par;
  for (int i = 0; i < n; ++i) x[i] = 0.0;
  for (int s = 0; s < H.prm.nu_pre; ++s) {
    spmv(L.A, x, Ax.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (par)
    for (int i = 0; i < n; ++i) x[i] = x[i] + L.sw[i] * (b[i] - Ax[i]);
  }
  spmv(L.A, x, Ax.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (par)
  for (int i = 0; i < n; ++i) r[i] = b[i] - Ax[i];
  int nc = L.nagg;
  std::vector<double> bc(nc), xc(nc), Pxc(n);
  spmv(L.R, r.data(), bc.data());
  vcycle(H, l + 1, bc.data(), xc.data());
  spmv(L.P, xc.data(), Pxc.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (par)
  for (int i = 0; i < n; ++i) x[i] = x[i] + Pxc[i];
  for (int s = 0; s < H.prm.nu_post; ++s) {
    spmv(L.A, x, Ax.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (par)
    for (int i = 0; i < n; ++i) x[i] = x[i] + L.sw[i] * (b[i] - Ax[i]);
  }
}

// use_prec: 0 identity, 1 V-cycle, 2 V-cycle followed by a positive diagonal
// scaling that changes with the iteration (a deliberately variable
// preconditioner; test hook for the flexible recurrence).
void apply_prec(const Hier& H, int use_prec, const std::vector<double>& r, std::vector<double>& z, int it) {
  if (use_prec == 0) { z = r; return; }
  vcycle(H, 0, r.data(), z.data());
  if (use_prec == 2)
    for (size_t i = 0; i < z.size(); ++i) z[i] *= 1.0 + 0.5 * std::sin((double)i + 1.7 * it);
}

// Preconditioned CG from x0 = 0.  Standard beta = <r,z>/<r_old,z_old>, or the
// flexible (Polak-Ribiere) beta = <z, r - r_old>/<r_old, z_old>.  Iterations
// count products A p.  Stops when ||r||^2 <= tol^2 ||b||^2 (recursive
// residual); then the true residual b - A x is formed, and if it misses the
// tolerance the recursion restarts from it (at most 5 times).
// hist (optional, maxiter entries): recursive relative residual per
// iteration.  conj (optional, maxiter entries): cosine between the new search
// direction and A times the previous one (local A-conjugacy).
int pcg(const Hier& H, const double* bptr, double* xptr, double tol, int maxiter, int flexible, int use_prec,
        int* iters_out, double* relres_out, double* hist, double* conj) {
  const Csr& A = H.lv[0].A;
  int n = A.nrows;
  std::vector<double> b(bptr, bptr + n), x(n, 0.0), r(n), z(n), p(n), q(n), rold;
  double bb = dot(b, b);
  *iters_out = 0;
  if (!(bb == bb)) { std::copy(x.begin(), x.end(), xptr); *relres_out = NAN; return OR_ERR_BREAKDOWN; }
  if (bb == 0.0) {
    std::copy(x.begin(), x.end(), xptr);
    *relres_out = 0.0;
    return OR_OK;
  }
  double thresh = (tol * tol) * bb;
  r = b;
  int iters = 0, replacements = 0, status = OR_NOT_CONVERGED;
  bool breakdown = false;
  for (;;) {
    apply_prec(H, use_prec, r, z, iters);
    double rz = dot(r, z);
    if (!(rz > 0.0)) { breakdown = true; break; }
    p = z;
    bool conv = false;
    while (iters < maxiter) {
      spmv(A, p.data(), q.data());
      double pq = dot(p, q);
      if (!(pq > 0.0)) { breakdown = true; break; }
      double alpha = rz / pq;
      if (flexible) rold = r;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
      for (int i = 0; i < n; ++i) {
        x[i] = x[i] + alpha * p[i];
        r[i] = r[i] - alpha * q[i];
      }
      ++iters;
      double rr = dot(r, r);
      if (hist) hist[iters - 1] = std::sqrt(rr / bb);
      if (rr <= thresh) { conv = true; break; }
      if (!(rr == rr)) { breakdown = true; break; }
      apply_prec(H, use_prec, r, z, iters);
      double rzn = dot(r, z);
      if (!(rzn > 0.0)) { breakdown = true; break; }
      double beta;
      if (flexible) {
        double zro = dot(z, rold);
        beta = (rzn - zro) / rz;
      } else {
        beta = rzn / rz;
      }
      rz = rzn;
#pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
      for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
      if (conj) conj[iters - 1] = dot(p, q) / std::sqrt(dot(p, p) * dot(q, q));
    }
    if (breakdown) break;
    if (!conv) break;  // iteration limit
    std::vector<double> Ax(n);
    spmv(A, x.data(), Ax.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
    for (int i = 0; i < n; ++i) r[i] = b[i] - Ax[i];
    double trr = dot(r, r);
    if (trr <= thresh) { status = OR_OK; break; }
    if (replacements >= 5 || iters >= maxiter) break;
    ++replacements;
  }
  std::vector<double> Ax(n), d(n);
  spmv(A, x.data(), Ax.data());
#pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
  for (int i = 0; i < n; ++i) d[i] = b[i] - Ax[i];
  const double trr = dot(d, d);
  *relres_out = std::sqrt(trr / bb);
  *iters_out = iters;
  std::copy(x.begin(), x.end(), xptr);
  if (breakdown) return OR_ERR_BREAKDOWN;
  return status == OR_OK || trr <= thresh ? OR_OK : OR_NOT_CONVERGED;
}

// Right-preconditioned BiCGSTAB (van der Vorst, 1992) from x0 = 0, the
// paper's default Krylov method (Section 2.1).  Shadow residual r^ = r0.
// One iteration:
//   rho = <r^, r>;  p = r (first) or r + beta (p - omega v),
//                   beta = (rho / rho_old) (alpha / omega)
//   y = M p;  v = A y;  alpha = rho / <r^, v>
//   x = x + alpha y;  s = r - alpha v        (stop here if ||s|| is small)
//   z = M s;  t = A z;  omega = <t, s> / <t, t>
//   x = x + omega z;  r = s - omega t
// Iterations count full steps (a stop at s counts its step).  Stops when
// ||s||^2 or ||r||^2 <= tol^2 ||b||^2; then the true residual b - A x is
// formed and, if it misses the tolerance, the method restarts from it
// (r^ = r = b - A x; at most 5 times).  Breakdown: rho, <r^, v>, <t, t> or
// omega zero or NaN.  hist (optional, maxiter entries): relative recursive
// residual at the end of each step.
int bicgstab(const Hier& H, const double* bptr, double* xptr, double tol, int maxiter, int use_prec,
             int* iters_out, double* relres_out, double* hist) {
  const Csr& A = H.lv[0].A;
  int n = A.nrows;
  std::vector<double> b(bptr, bptr + n), x(n, 0.0), r(n), rh(n), p(n, 0.0), v(n, 0.0), y(n), s(n), z(n), t(n);
  double bb = dot(b, b);
  *iters_out = 0;
  if (!(bb == bb)) { std::copy(x.begin(), x.end(), xptr); *relres_out = NAN; return OR_ERR_BREAKDOWN; }
  if (bb == 0.0) {
    std::copy(x.begin(), x.end(), xptr);
    *relres_out = 0.0;
    return OR_OK;
  }
  double thresh = (tol * tol) * bb;
  r = b;
  int iters = 0, replacements = 0, status = OR_NOT_CONVERGED;
  bool breakdown = false;
  for (;;) {
    rh = r;
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    bool first = true, conv = false;
    while (iters < maxiter) {
      double rho = dot(rh, r);
      if (!(rho != 0.0) || !(rho == rho)) { breakdown = true; break; }
      if (first) {
        p = r;
        first = false;
      } else {
        double beta = (rho / rho_old) * (alpha / omega);
        #pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
        for (int i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
      }
      apply_prec(H, use_prec, p, y, iters);
      spmv(A, y.data(), v.data());
      double rv = dot(rh, v);
      if (!(rv != 0.0) || !(rv == rv)) { breakdown = true; break; }
      alpha = rho / rv;
      #pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
      for (int i = 0; i < n; ++i) {
        x[i] = x[i] + alpha * y[i];
        s[i] = r[i] - alpha * v[i];
      }
      ++iters;
      double ss = dot(s, s);
      if (ss <= thresh) {
        r = s;
        if (hist) hist[iters - 1] = std::sqrt(ss / bb);
        conv = true;
        break;
      }
      apply_prec(H, use_prec, s, z, iters);
      spmv(A, z.data(), t.data());
      double tt = dot(t, t), ts = dot(t, s);
      if (!(tt > 0.0)) { breakdown = true; break; }
      omega = ts / tt;
      if (!(omega != 0.0) || !(omega == omega)) { breakdown = true; break; }
      #pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
      for (int i = 0; i < n; ++i) {
        x[i] = x[i] + omega * z[i];
        r[i] = s[i] - omega * t[i];
      }
      double rr = dot(r, r);
      if (hist) hist[iters - 1] = std::sqrt(rr / bb);
      if (rr <= thresh) { conv = true; break; }
      if (!(rr == rr)) { breakdown = true; break; }
      rho_old = rho;
    }
    if (breakdown || !conv) break;
    std::vector<double> Ax(n);
    spmv(A, x.data(), Ax.data());
    #pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
    for (int i = 0; i < n; ++i) r[i] = b[i] - Ax[i];
    double trr = dot(r, r);
    if (trr <= thresh) { status = OR_OK; break; }
    if (replacements >= 5 || iters >= maxiter) break;
    ++replacements;
  }
  std::vector<double> Ax(n), d(n);
  spmv(A, x.data(), Ax.data());
  #pragma omp parallel for schedule(static) num_threads(g_threads) if (n >= kParMin)
  for (int i = 0; i < n; ++i) d[i] = b[i] - Ax[i];
  const double trr = dot(d, d);
  *relres_out = std::sqrt(trr / bb);
  *iters_out = iters;
  std::copy(x.begin(), x.end(), xptr);
  if (breakdown) return OR_ERR_BREAKDOWN;
  return status == OR_OK || trr <= thresh ? OR_OK : OR_NOT_CONVERGED;
}

}  // namespace

// ================================================================ C API
extern "C" {

// Threads of the solve loops (spmv, element-wise updates, fixed-block dot
// products); the results do not depend on it.  k < 1 is taken as 1.
void or_set_threads(int k) { g_threads = k < 1 ? 1 : k; }
int or_get_threads(void) { return g_threads; }

void* or_setup(int n, const int* rp, const int* ci, const double* v, double theta, int max_coarse, int max_levels,
               int smoother, double omega, int nu_pre, int nu_post, int symmetric, int* status) {
  int st = validate_csr(n, rp, ci);
  if (st == OR_OK && (max_levels < 1 || max_coarse < 1 || nu_pre < 1 || nu_post < 1 || (symmetric != 0 && symmetric != 1)))
    st = OR_ERR_INVALID_ARG;
  if (st != OR_OK) { *status = st; return nullptr; }
  Hier* H = new Hier;
  H->prm = Params{theta, max_coarse, max_levels, smoother, omega, nu_pre, nu_post, symmetric};
  H->lv.emplace_back();
  Csr& A = H->lv[0].A;
  A.nrows = A.ncols = n;
  A.rp.assign(rp, rp + n + 1);
  A.ci.assign(ci, ci + rp[n]);
  A.v.assign(v, v + rp[n]);
  for (int i = 0; i < n; ++i)
    if (diag_of(A, i) == 0.0) { delete H; *status = OR_ERR_ZERO_DIAG; return nullptr; }
  st = build_levels(*H, false);
  if (st != OR_OK) { delete H; *status = st; return nullptr; }
  *status = OR_OK;
  return H;
}

// New values on the same pattern.  theta == 0: the strength graph is A's
// pattern, so aggregates and patterns are kept and only the values of every
// level are recomputed.  theta > 0: the strength graph depends on the values,
// so the whole hierarchy is built again (it never depends on earlier values).
int or_update_values(void* h, const double* v) {
  Hier* H = (Hier*)h;
  Csr& A = H->lv[0].A;
  std::copy(v, v + A.nnz(), A.v.begin());
  for (int i = 0; i < A.nrows; ++i)
    if (diag_of(A, i) == 0.0) return OR_ERR_ZERO_DIAG;
  if (H->prm.theta > 0.0) {
    H->lv.resize(1);
    return build_levels(*H, false);
  }
  return build_levels(*H, true);
}

void or_destroy(void* h) { delete (Hier*)h; }

int or_num_levels(void* h) { return (int)((Hier*)h)->lv.size(); }

// out: n, nnz(A), nnz(P) (0 on the coarsest), nagg (0 on the coarsest), nnz(G)
int or_level_sizes(void* h, int l, int64_t* out) {
  Hier* H = (Hier*)h;
  if (l < 0 || l >= (int)H->lv.size()) return OR_ERR_INVALID_ARG;
  const Level& L = H->lv[l];
  out[0] = L.A.nrows;
  out[1] = L.A.nnz();
  out[2] = L.P.nnz();
  out[3] = L.nagg;
  out[4] = L.G.nnz();
  return OR_OK;
}

// Any output pointer may be null.  scal: rho, omegaP.
int or_export_level(void* h, int l, int* agg, int* A_rp, int* A_ci, double* A_v, double* dinv, int* P_rp, int* P_ci,
                    double* P_v, int* R_rp, int* R_ci, double* R_v, int* G_rp, int* G_ci, double* scal) {
  Hier* H = (Hier*)h;
  if (l < 0 || l >= (int)H->lv.size()) return OR_ERR_INVALID_ARG;
  const Level& L = H->lv[l];
  auto cp_i = [](int* dst, const std::vector<int>& s) { if (dst) std::copy(s.begin(), s.end(), dst); };
  auto cp_d = [](double* dst, const std::vector<double>& s) { if (dst) std::copy(s.begin(), s.end(), dst); };
  cp_i(agg, L.agg);
  cp_i(A_rp, L.A.rp); cp_i(A_ci, L.A.ci); cp_d(A_v, L.A.v);
  cp_d(dinv, L.dinv);
  cp_i(P_rp, L.P.rp); cp_i(P_ci, L.P.ci); cp_d(P_v, L.P.v);
  cp_i(R_rp, L.R.rp); cp_i(R_ci, L.R.ci); cp_d(R_v, L.R.v);
  cp_i(G_rp, L.G.rp); cp_i(G_ci, L.G.ci);
  if (scal) { scal[0] = L.rho; scal[1] = L.omegaP; }
  return OR_OK;
}

// Smoother weights of level l (n_l entries): omega/a_ii for damped Jacobi,
// 1/sum_j |a_ij| for L1-Jacobi.
int or_export_sw(void* h, int l, double* sw) {
  Hier* H = (Hier*)h;
  if (l < 0 || l >= (int)H->lv.size()) return OR_ERR_INVALID_ARG;
  std::copy(H->lv[l].sw.begin(), H->lv[l].sw.end(), sw);
  return OR_OK;
}

int or_coarse_factor(void* h, double* Lout) {
  Hier* H = (Hier*)h;
  std::copy(H->L.begin(), H->L.end(), Lout);
  return H->nL;
}

// LU pivots of the coarsest level (nonsymmetric hierarchies; returns nL, or
// 0 for a Cholesky factor).
int or_coarse_pivots(void* h, int* piv) {
  Hier* H = (Hier*)h;
  if (H->prm.symmetric) return 0;
  std::copy(H->piv.begin(), H->piv.end(), piv);
  return H->nL;
}

int or_bicgstab(void* h, const double* b, double* x, double tol, int maxiter, int use_prec, int* iters,
                double* relres, double* hist) {
  return bicgstab(*(Hier*)h, b, x, tol, maxiter, use_prec, iters, relres, hist);
}

// Explicit transpose of an n x n CSR matrix (rows of the result list source
// rows ascending): the operator of the nonsymmetric adjoint, Eq. (1).
void or_transpose(int n, const int* rp, const int* ci, const double* v, int* rpT, int* ciT, double* vT) {
  Csr A;
  A.nrows = A.ncols = n;
  A.rp.assign(rp, rp + n + 1);
  A.ci.assign(ci, ci + rp[n]);
  A.v.assign(v, v + rp[n]);
  Csr T = transpose(A);
  std::copy(T.rp.begin(), T.rp.end(), rpT);
  std::copy(T.ci.begin(), T.ci.end(), ciT);
  std::copy(T.v.begin(), T.v.end(), vT);
}

int or_vcycle(void* h, const double* b, double* x) {
  vcycle(*(Hier*)h, 0, b, x);
  return OR_OK;
}

int or_pcg(void* h, const double* b, double* x, double tol, int maxiter, int flexible, int use_prec, int* iters,
           double* relres, double* hist, double* conj) {
  return pcg(*(Hier*)h, b, x, tol, maxiter, flexible, use_prec, iters, relres, hist, conj);
}

// Adjoint (Eq. (1)) of a symmetric A: A^T lambda = g is solved by PCG with
// A's own hierarchy and the same settings.  (A nonsymmetric A's adjoint is
// solved on the hierarchy of its explicit transpose, or_transpose.)
int or_solve_adjoint(void* h, const double* g, double* lam, double tol, int maxiter, int flexible, int* iters,
                     double* relres) {
  return pcg(*(Hier*)h, g, lam, tol, maxiter, flexible, 1, iters, relres, nullptr, nullptr);
}

// Matrix-value gradient restricted to the stored pattern (Eq. (2)):
// grad_val[k] = -(lambda[row k] * x[col k]).  The RHS gradient is lambda.
void or_pattern_grad(int n, const int* rp, const int* ci, const double* lam, const double* x, double* grad) {
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) grad[k] = -(lam[i] * x[ci[k]]);
}

void or_spmv(int n, const int* rp, const int* ci, const double* v, const double* x, double* y) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    y[i] = s;
  }
}

// ||b - A x||_2 / ||b||_2 in FP64.
double or_rel_residual(int n, const int* rp, const int* ci, const double* v, const double* b, const double* x) {
  double rr = 0.0, bb = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s += v[k] * x[ci[k]];
    double d = b[i] - s;
    rr += d * d;
    bb += b[i] * b[i];
  }
  return std::sqrt(rr / bb);
}

// ------------------------------------------------ matrix-free assembly
// Graph-colored probing (Section 2.1, "Matrix-free operator support";
// Curtis, Powell and Reid 1974): a partition of the columns into groups in
// which no two columns share a row, so that one operator application to the
// 0/1 sum of a group's unit vectors yields every entry of those columns.

// Greedy coloring in decreasing node-key order (the same keys as the
// aggregation): each column takes the smallest color not used by any
// already colored column that shares a row with it.  Returns the number of
// colors.
int or_color_columns(int n, const int* rp, const int* ci, int* color) {
  Csr A;
  A.nrows = A.ncols = n;
  A.rp.assign(rp, rp + n + 1);
  A.ci.assign(ci, ci + rp[n]);
  A.v.assign(rp[n], 0.0);
  Csr T = transpose(A);  // column j -> its rows
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::sort(order.begin(), order.end(), [](int a, int b) { return node_key(a) > node_key(b); });
  for (int j = 0; j < n; ++j) color[j] = -1;
  std::vector<int> seen(n + 1, -1);  // seen[c] == j: color c is used next to column j
  int ncolors = 0;
  for (int j : order) {
    for (int a = T.rp[j]; a < T.rp[j + 1]; ++a) {
      int i = T.ci[a];
      for (int b = A.rp[i]; b < A.rp[i + 1]; ++b) {
        int c = color[A.ci[b]];
        if (c >= 0) seen[c] = j;
      }
    }
    int c = 0;
    while (seen[c] == j) ++c;
    color[j] = c;
    ncolors = std::max(ncolors, c + 1);
  }
  return ncolors;
}

// val[k] = Y[color(col k)][row k]: Y = A V with probe c = sum of the unit
// vectors of the columns of color c, stored [ncolors][n].
void or_probe_assemble(int n, const int* rp, const int* ci, const int* color, const double* Y, double* val) {
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) val[k] = Y[(size_t)color[ci[k]] * n + i];
}

// Adjoint of the assembly: dY = 0, then dY[color(col k)][row k] = dval[k].
void or_probe_scatter(int n, const int* rp, const int* ci, const int* color, int ncolors, const double* dval,
                      double* dY) {
  std::fill(dY, dY + (size_t)ncolors * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = rp[i]; k < rp[i + 1]; ++k) dY[(size_t)color[ci[k]] * n + i] = dval[k];
}

uint64_t or_node_key(int i) { return node_key(i); }

int or_validate(int n, const int* rp, const int* ci) { return validate_csr(n, rp, ci); }

}  // extern "C"
