// Host-side (FP64) construction of the 1D spectral-element operators and their
// generalised eigendecomposition.
//
// Paper: Liu, Shen & Zhang, arXiv 2310.00226.
//   Sec. 2.1       Q^k Lagrange basis on (k+1) Gauss-Lobatto points; 1D stiffness
//                  <phi_i', phi_j'> and lumped (diagonal) mass <phi_i, phi_j>.
//   Sec. 2.3       robust eigen-solve through the symmetric M^{-1/2} K M^{-1/2}.
//   Appendix       SEGenerator1D: uniform mesh, element half-width h, gluing of
//                  shared end nodes; LegendreD: GLL rule and derivative matrix.
//
// Everything here runs once per plan ("offline" in the paper's terms).
#include "plan_host.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <stdexcept>
#include <thread>
#include <vector>

namespace semfd {

// ----------------------------------------------------------------------------
// Symmetric tridiagonal eigen-solver: implicit symmetric QR steps with the
// Wilkinson shift and deflation of negligible off-diagonal entries (Golub & Van
// Loan, Matrix Computations, 4th ed., Algorithms 8.3.2 and 8.3.3).
// d[0..n-1] diagonal, e[0..n-2] off-diagonal (e[i] couples i and i+1).  If
// z != nullptr (n x n, row-major, leading dimension ldz) the Givens rotations are
// accumulated into z's columns: on exit column j of z holds the eigenvector of
// d[j] in z's original basis.  The rotations of one bulge chase are recorded and
// then applied to the rows of z in parallel.
// ----------------------------------------------------------------------------
namespace {
struct Givens {
  double c, s;
};

// z[:, j] <- c z[:, j] + s z[:, j+1];  z[:, j+1] <- -s z[:, j] + c z[:, j+1]
// for j = first, first + 1, ... in the order recorded
void rotate_columns(double* z, int nrows, int ldz, int first, const std::vector<Givens>& g, int nthreads) {
  auto rows = [&](int r0, int r1) {
    for (int r = r0; r < r1; ++r) {
      double* row = z + (size_t)r * ldz;
      for (size_t t = 0; t < g.size(); ++t) {
        const int j = first + (int)t;
        const double a = row[j], b = row[j + 1];
        row[j] = g[t].c * a + g[t].s * b;
        row[j + 1] = -g[t].s * a + g[t].c * b;
      }
    }
  };
  const long cost = (long)nrows * (long)g.size();
  if (nthreads <= 1 || cost < 200000) {
    rows(0, nrows);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back(rows, (int)((long)nrows * t / nthreads), (int)((long)nrows * (t + 1) / nthreads));
  for (auto& x : th) x.join();
}
}  // namespace

void tridiag_qr(int n, double* d, double* e_in, double* z, int ldz, int nthreads) {
  if (n <= 1) return;
  std::vector<double> e(e_in, e_in + (n - 1));
  std::vector<Givens> chase;
  chase.reserve(n);
  const double tol = 0.5 * std::numeric_limits<double>::epsilon();
  int hi = n - 1, steps = 0;
  while (hi > 0) {
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= tol * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    if (e[hi - 1] == 0.0) {  // d[hi] has converged
      --hi;
      steps = 0;
      continue;
    }
    int lo = hi - 1;  // the unreduced block [lo, hi]
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++steps > 60) throw std::runtime_error("tridiagonal QR did not converge");
    // Wilkinson shift: the eigenvalue of the trailing 2x2 closer to d[hi]
    const double half = 0.5 * (d[hi - 1] - d[hi]), b = e[hi - 1];
    const double mu = d[hi] - b * b / (half + (half >= 0.0 ? 1.0 : -1.0) * std::hypot(half, b));
    // bulge chase: the first rotation acts on the shifted first column, each
    // later one annihilates the bulge the previous one left below e[k-1]
    chase.clear();
    double x = d[lo] - mu, y = e[lo], bulge = 0.0;
    for (int k = lo; k < hi; ++k) {
      if (k > lo) {
        x = e[k - 1];
        y = bulge;
      }
      const double r = std::hypot(x, y);
      const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : y / r;
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
      if (k + 1 < hi) {
        bulge = s * e[k + 1];
        e[k + 1] *= c;
      }
      chase.push_back({c, s});
    }
    if (z) rotate_columns(z, n, ldz, lo, chase, nthreads);
  }
}

// ----------------------------------------------------------------------------
// Householder reduction of a dense symmetric matrix a (n x n, row-major) to
// tridiagonal form a = Q T Q^T.  On exit a holds Q, d the diagonal, e the
// off-diagonal (e[i] couples i and i+1).
// ----------------------------------------------------------------------------
void householder_tridiag(int n, double* a, double* d, double* e, int nthreads) {
  std::vector<double> v(n), w(n);
  std::vector<double> hv;  // Householder vectors, stored in the lower part of a
  for (int k = 0; k < n - 2; ++k) {
    // column k below the diagonal: x = a[k+1..n-1][k]
    double alpha2 = 0.0;
    for (int i = k + 1; i < n; ++i) alpha2 += a[(size_t)i * n + k] * a[(size_t)i * n + k];
    double x0 = a[(size_t)(k + 1) * n + k];
    double alpha = (x0 >= 0 ? -1.0 : 1.0) * std::sqrt(alpha2);
    if (alpha2 == 0.0 || std::fabs(alpha2 - x0 * x0) <= 1e-300) {
      // column already reduced: identity reflector, flagged by a zero vector
      e[k] = x0;
      for (int i = k + 1; i < n; ++i) a[(size_t)i * n + k] = 0.0;
      continue;
    }
    // v = x - alpha e1, normalised so that H = I - 2 v v^T / (v^T v)
    for (int i = k + 1; i < n; ++i) v[i] = a[(size_t)i * n + k];
    v[k + 1] -= alpha;
    double vnorm2 = 0.0;
    for (int i = k + 1; i < n; ++i) vnorm2 += v[i] * v[i];
    const double beta = 2.0 / vnorm2;
    // w = beta * A v on the trailing block (rows/cols k+1..n-1)
    auto mv = [&](int r0, int r1) {
      for (int i = r0; i < r1; ++i) {
        const double* row = a + (size_t)i * n;
        double s = 0.0;
        for (int j = k + 1; j < n; ++j) s += row[j] * v[j];
        w[i] = beta * s;
      }
    };
    const int m = n - k - 1;
    if (nthreads > 1 && (long)m * m > 400000) {
      std::vector<std::thread> th;
      for (int t = 0; t < nthreads; ++t)
        th.emplace_back(mv, k + 1 + (int)((long)m * t / nthreads), k + 1 + (int)((long)m * (t + 1) / nthreads));
      for (auto& x : th) x.join();
    } else {
      mv(k + 1, n);
    }
    // w <- w - (beta/2)(v^T w) v  ; A <- A - v w^T - w v^T
    double vw = 0.0;
    for (int i = k + 1; i < n; ++i) vw += v[i] * w[i];
    const double kk = 0.5 * beta * vw;
    for (int i = k + 1; i < n; ++i) w[i] -= kk * v[i];
    auto upd = [&](int r0, int r1) {
      for (int i = r0; i < r1; ++i) {
        double* row = a + (size_t)i * n;
        const double vi = v[i], wi = w[i];
        for (int j = k + 1; j < n; ++j) row[j] -= vi * w[j] + wi * v[j];
      }
    };
    if (nthreads > 1 && (long)m * m > 400000) {
      std::vector<std::thread> th;
      for (int t = 0; t < nthreads; ++t)
        th.emplace_back(upd, k + 1 + (int)((long)m * t / nthreads), k + 1 + (int)((long)m * (t + 1) / nthreads));
      for (auto& x : th) x.join();
    } else {
      upd(k + 1, n);
    }
    e[k] = alpha;
    // store v (scaled to unit norm) in column k below the diagonal for the accumulation
    const double inv = 1.0 / std::sqrt(vnorm2);
    for (int i = k + 1; i < n; ++i) a[(size_t)i * n + k] = v[i] * inv;
  }
  if (n >= 2) e[n - 2] = a[(size_t)(n - 1) * n + (n - 2)];
  for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
  // Accumulate Q = H_0 H_1 ... H_{n-3} into a fresh matrix q (backward accumulation).
  std::vector<double> q((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) q[(size_t)i * n + i] = 1.0;
  for (int k = n - 3; k >= 0; --k) {
    // u = unit Householder vector in rows k+1..n-1 of column k; H = I - 2 u u^T
    bool zero = true;
    for (int i = k + 1; i < n; ++i) {
      v[i] = a[(size_t)i * n + k];
      if (v[i] != 0.0) zero = false;
    }
    if (zero) continue;
    // q[k+1.., k+1..] <- H q  : q -= 2 u (u^T q)
    const int m = n - k - 1;
    std::fill(w.begin(), w.end(), 0.0);
    auto colsum = [&](int c0, int c1) {
      for (int j = c0; j < c1; ++j) {
        double s = 0.0;
        for (int i = k + 1; i < n; ++i) s += v[i] * q[(size_t)i * n + j];
        w[j] = s;
      }
    };
    auto upd = [&](int c0, int c1) {
      for (int i = k + 1; i < n; ++i) {
        double* row = q.data() + (size_t)i * n;
        const double vi = 2.0 * v[i];
        for (int j = c0; j < c1; ++j) row[j] -= vi * w[j];
      }
    };
    if (nthreads > 1 && (long)m * m > 400000) {
      std::vector<std::thread> th;
      for (int t = 0; t < nthreads; ++t)
        th.emplace_back(colsum, k + 1 + (int)((long)m * t / nthreads), k + 1 + (int)((long)m * (t + 1) / nthreads));
      for (auto& x : th) x.join();
      th.clear();
      for (int t = 0; t < nthreads; ++t)
        th.emplace_back(upd, k + 1 + (int)((long)m * t / nthreads), k + 1 + (int)((long)m * (t + 1) / nthreads));
      for (auto& x : th) x.join();
    } else {
      colsum(k + 1, n);
      upd(k + 1, n);
    }
  }
  std::memcpy(a, q.data(), sizeof(double) * (size_t)n * n);
}

// Symmetric eigen-decomposition a = Q diag(w) Q^T, ascending; a is overwritten by Q.
void sym_eig(int n, double* a, double* w, int nthreads) {
  std::vector<double> e(std::max(n, 1), 0.0);
  if (n == 1) {
    w[0] = a[0];
    a[0] = 1.0;
    return;
  }
  householder_tridiag(n, a, w, e.data(), nthreads);
  tridiag_qr(n, w, e.data(), a, n, nthreads);
  // sort ascending, permuting columns
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int i, int j) { return w[i] < w[j]; });
  std::vector<double> ws(n), as((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    ws[c] = w[idx[c]];
    for (int r = 0; r < n; ++r) as[(size_t)r * n + c] = a[(size_t)r * n + idx[c]];
  }
  std::memcpy(w, ws.data(), sizeof(double) * n);
  std::memcpy(a, as.data(), sizeof(double) * (size_t)n * n);
}

// ----------------------------------------------------------------------------
// GLL rule.  Interior nodes are the zeros of P_k', i.e. of the Jacobi polynomial
// P^{(1,1)}_{k-1}: the eigenvalues of its symmetric Jacobi matrix (zero diagonal,
// off-diagonal sqrt(j(j+2)/((2j+1)(2j+3))), j = 1..k-2)  [Golub-Welsch].
// Weights 2/(k(k+1) P_k(x)^2).
// ----------------------------------------------------------------------------
static double legendre_p(int k, double x) {
  double p0 = 1.0, p1 = x;
  if (k == 0) return p0;
  for (int j = 1; j < k; ++j) {
    double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

void gll_rule(int k, std::vector<double>& x, std::vector<double>& w) {
  x.assign(k + 1, 0.0);
  w.assign(k + 1, 0.0);
  x[0] = -1.0;
  x[k] = 1.0;
  if (k >= 2) {
    const int m = k - 1;
    std::vector<double> d(m, 0.0), e(std::max(m, 1), 0.0);
    for (int j = 1; j <= m - 1; ++j) e[j - 1] = std::sqrt((double)j * (j + 2) / ((2.0 * j + 1) * (2.0 * j + 3)));
    tridiag_qr(m, d.data(), e.data(), nullptr, 0, 1);
    std::sort(d.begin(), d.end());
    // the eigenvalues carry errors of a few ulps; two Newton steps on P_k' in long
    // double (P_k'' from Legendre's equation) round them correctly
    for (int j = 0; j < m; ++j) {
      long double t = d[j];
      for (int it = 0; it < 2; ++it) {
        long double p0 = 1.0L, p1 = t;
        for (int q = 1; q < k; ++q) {
          const long double p2 = ((2.0L * q + 1.0L) * t * p1 - (long double)q * p0) / (long double)(q + 1);
          p0 = p1;
          p1 = p2;
        }
        const long double dp = k * (t * p1 - p0) / (t * t - 1.0L);
        const long double d2p = (2.0L * t * dp - (long double)k * (k + 1) * p1) / (1.0L - t * t);
        t -= dp / d2p;
      }
      x[j + 1] = (double)t;
    }
    // enforce the exact symmetry of the rule
    for (int j = 1; j < k; ++j) {
      double s = 0.5 * (x[j] - x[k - j]);
      x[j] = s;
      x[k - j] = -s;
    }
    if (k % 2 == 0) x[k / 2] = 0.0;
  }
  for (int j = 0; j <= k; ++j) {
    double p = legendre_p(k, x[j]);
    w[j] = 2.0 / (k * (k + 1.0) * p * p);
  }
}

// Derivative matrix D[i][j] = l_j'(x_i): closed form for Legendre-Gauss-Lobatto
// off the diagonal, P_k(x_i) / (P_k(x_j) (x_i - x_j)); diagonal = minus the row sum
// (so that constants are differentiated to zero exactly).
static void gll_derivative(int k, const std::vector<double>& x, std::vector<double>& D) {
  const int np = k + 1;
  D.assign((size_t)np * np, 0.0);
  std::vector<double> p(np);
  for (int i = 0; i < np; ++i) p[i] = legendre_p(k, x[i]);
  for (int i = 0; i < np; ++i) {
    double s = 0.0;
    for (int j = 0; j < np; ++j) {
      if (i == j) continue;
      D[(size_t)i * np + j] = p[i] / (p[j] * (x[i] - x[j]));
      s += D[(size_t)i * np + j];
    }
    D[(size_t)i * np + i] = -s;
  }
}

// ----------------------------------------------------------------------------
// Extended-precision refinement of the generalised eigenpairs K S = M S Lambda.
//
// The FD solve divides by lx_i + ly_j + lz_l + alpha; an FP64 eigensolver leaves
// absolute eigenvalue errors ~ eps * lambda_max and eigenvector errors
// ~ eps * lambda_max / gap, which perturb the lowest (dominant) solution modes by
// ~eps * cond (~1e-11 at n ~ 1000).  One Newton step of Ogita & Aishima (2018),
// with the Gram matrices in x87 long double, brings them to FP64 rounding:
//   T = X^T K X,  R = I - X^T M X,  lam_i = T_ii / (1 - R_ii),
//   E_ii = R_ii / 2,  E_ij = (T_ij + lam_j R_ij) / (lam_j - lam_i),  X <- X (I + E).
// Pairs closer than 1e-15 * lambda_max keep only the symmetric part R_ij / 2.
// ----------------------------------------------------------------------------
template <class F>
static void parallel_rows(int n, int nthreads, F&& fn) {
  if (nthreads <= 1 || n < 64) {
    fn(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int chunks = std::min(n, nthreads * 4);
  std::atomic<int> next{0};
  for (int t = 0; t < nthreads; ++t)
    th.emplace_back([&] {
      for (;;) {
        const int c = next.fetch_add(1);
        if (c >= chunks) break;
        fn((int)((long)n * c / chunks), (int)((long)n * (c + 1) / chunks));
      }
    });
  for (auto& x : th) x.join();
}

// K X is formed element by element from the long-double element stiffness ke
// ((k+1)^2, already divided by h): FP64 rounding of K's entries alone would shift
// the lowest eigenvalues by ~ eps * lambda_max, since they come out of a
// cancellation of ratio lambda_max / lambda_min.
static void refine_eigenpairs(int n, int m, int k, int ne, const std::vector<long double>& ke, int off, bool per,
                              const std::vector<double>& mass, std::vector<double>& lam, std::vector<double>& S,
                              int nthreads) {
  // S: n x m (m eigenvectors of one invariant subspace, e.g. the symmetric ones),
  // lam: m.  Rows of X that are equal (or opposite) stay so: every row is updated
  // by the same arithmetic from its own entries.
  typedef long double ld;
  const int np = k + 1, nfull = ne * k + 1;
  const size_t nm = (size_t)n * m, mm = (size_t)m * m;
  std::vector<ld> X(nm), KX(nm), T(mm), R(mm), L(m);
  for (size_t t = 0; t < nm; ++t) X[t] = S[t];
  parallel_rows(n, nthreads, [&](int p0, int p1) {
    for (int p = p0; p < p1; ++p) {
      ld* row = &KX[(size_t)p * m];
      std::fill(row, row + m, 0.0L);
      // periodic: full nodes p and p + n are one unknown (only p = 0 has the alias)
      for (int alias = 0; alias <= (per ? 1 : 0); ++alias) {
        const int pf = p + off + alias * n;  // full-numbering index
        if (pf >= nfull) continue;
        // elements containing node pf: e = pf / k (as its left/inner node) and pf / k - 1 (as right end)
        for (int e = std::max(0, (pf - 1) / k); e <= std::min(ne - 1, pf / k); ++e) {
          const int li = pf - e * k;
          if (li < 0 || li > k) continue;
          for (int lj = 0; lj < np; ++lj) {
            const int qf = e * k + lj, q = per ? qf % n : qf - off;
            if (q < 0 || q >= n || qf >= nfull) continue;
            const ld kv = ke[(size_t)li * np + lj];
            const ld* xq = &X[(size_t)q * m];
            for (int j = 0; j < m; ++j) row[j] += kv * xq[j];
          }
        }
      }
    }
  });
  parallel_rows(m, nthreads, [&](int i0, int i1) {
    for (int i = i0; i < i1; ++i) {
      ld* ti = &T[(size_t)i * m];
      ld* ri = &R[(size_t)i * m];
      std::fill(ti, ti + m, 0.0L);
      std::fill(ri, ri + m, 0.0L);
      for (int p = 0; p < n; ++p) {
        const ld xpi = X[(size_t)p * m + i];
        const ld mx = (ld)mass[p] * xpi;
        const ld* kxp = &KX[(size_t)p * m];
        const ld* xp = &X[(size_t)p * m];
        for (int j = 0; j < m; ++j) {
          ti[j] += xpi * kxp[j];
          ri[j] += mx * xp[j];
        }
      }
      for (int j = 0; j < m; ++j) ri[j] = (i == j ? 1.0L : 0.0L) - ri[j];
    }
  });
  ld lmax = 0;
  for (int i = 0; i < m; ++i) {
    L[i] = T[(size_t)i * m + i] / (1.0L - R[(size_t)i * m + i]);
    lmax = std::max(lmax, std::fabs(L[i]));
  }
  // Pairs closer than tiny keep only the symmetric part of the update (no rotation
  // inside the pair).  Periodic spectra hold exactly double eigenvalues (Bloch
  // phases +theta and -theta) and, at phase pi, pairs split only by the
  // discretisation error (1.4e-10 lambda_max for Q^20 with 10 elements), across
  // which one Newton step would leave a second-order error (eps lambda_max / gap)^2
  // in S^T M S; inside such a pair any M-orthonormal basis is accurate to
  // eps lambda_max in K s - lambda M s.
  const ld tiny = (per ? 1e-8L : 1e-15L) * (lmax > 0 ? lmax : 1.0L);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const size_t ij = (size_t)i * m + j;
      if (i == j) {
        T[ij] = 0.5L * R[ij];
      } else {
        const ld dl = L[j] - L[i];
        T[ij] = std::fabs(dl) > tiny ? (T[ij] + L[j] * R[ij]) / dl : 0.5L * R[ij];
      }
    }
  parallel_rows(n, nthreads, [&](int p0, int p1) {
    std::vector<ld> acc(m);
    for (int p = p0; p < p1; ++p) {
      const ld* xp = &X[(size_t)p * m];
      for (int j = 0; j < m; ++j) acc[j] = xp[j];
      for (int i = 0; i < m; ++i) {
        const ld xpi = xp[i];
        const ld* ei = &T[(size_t)i * m];
        for (int j = 0; j < m; ++j) acc[j] += xpi * ei[j];
      }
      for (int j = 0; j < m; ++j) S[(size_t)p * m + j] = (double)acc[j];
    }
  });
  // keep ascending order
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return L[a] < L[b]; });
  bool sorted = true;
  for (int i = 0; i < m; ++i) sorted = sorted && idx[i] == i;
  std::vector<double> Sn = sorted ? std::vector<double>() : S;
  for (int c = 0; c < m; ++c) {
    lam[c] = (double)L[idx[c]];
    if (!sorted)
      for (int r = 0; r < n; ++r) S[(size_t)r * m + c] = Sn[(size_t)r * m + idx[c]];
  }
}

// Element stiffness (k+1)^2 in long double, divided by the half width h: the
// interior GLL nodes are polished in long double by Newton's method on P_k'
// (from the FP64 nodes; P_k'' from Legendre's equation), weights
// 2 / (k(k+1) P_k^2), closed-form derivative matrix with the diagonal set to
// minus the off-diagonal row sum, K_e = D^T W D / h.  At high k the FP64 node
// positions alone move the top of the spectrum by ~1e-13 relative.
static std::vector<long double> element_stiffness_ld(int k, const std::vector<double>& xr, double a, double b,
                                                     int ne) {
  typedef long double ld;
  const int np = k + 1;
  auto legendre = [k](ld x, ld* pkm1) {
    ld p0 = 1.0L, p1 = x;
    for (int j = 1; j < k; ++j) {
      const ld p2 = ((2.0L * j + 1.0L) * x * p1 - (ld)j * p0) / (ld)(j + 1);
      p0 = p1;
      p1 = p2;
    }
    if (pkm1) *pkm1 = k == 0 ? 0.0L : p0;
    return k == 0 ? 1.0L : p1;
  };
  std::vector<ld> x(np), w(np), p(np), D((size_t)np * np, 0.0L), ke((size_t)np * np, 0.0L);
  for (int i = 0; i < np; ++i) {
    x[i] = xr[i];
    if (i > 0 && i < k)
      for (int it = 0; it < 4; ++it) {
        ld pm1;
        const ld pk = legendre(x[i], &pm1);
        const ld dp = k * (x[i] * pk - pm1) / (x[i] * x[i] - 1.0L);
        const ld d2p = (2.0L * x[i] * dp - (ld)k * (k + 1) * pk) / (1.0L - x[i] * x[i]);
        x[i] -= dp / d2p;
      }
    p[i] = legendre(x[i], nullptr);
    w[i] = 2.0L / ((ld)k * (k + 1) * p[i] * p[i]);
  }
  for (int i = 0; i < np; ++i) {
    ld s = 0.0L;
    for (int j = 0; j < np; ++j) {
      if (i == j) continue;
      D[(size_t)i * np + j] = p[i] / (p[j] * (x[i] - x[j]));
      s += D[(size_t)i * np + j];
    }
    D[(size_t)i * np + i] = -s;
  }
  const ld h = ((ld)b - (ld)a) / (2.0L * ne);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      ld acc = 0.0L;
      for (int q = 0; q < np; ++q) acc += D[(size_t)q * np + i] * w[q] * D[(size_t)q * np + j];
      ke[(size_t)i * np + j] = acc / h;
    }
  return ke;
}

// ----------------------------------------------------------------------------
// 1D assembled operators and eigen-decomposition for one axis.
// ----------------------------------------------------------------------------
void build_axis(const AxisSpec& spec, AxisData& out, int nthreads) {
  const int k = spec.k, ne = spec.ne;
  if (k < 1 || ne < 1) throw std::invalid_argument("k >= 1 and ne >= 1 required");
  const bool dir = spec.dirichlet, per = spec.periodic && !spec.dirichlet;
  const int nfull = ne * k + 1;
  const int n = dir ? nfull - 2 : per ? nfull - 1 : nfull;
  if (n < 1) throw std::invalid_argument("Dirichlet needs ne*k >= 2");
  std::vector<double> xr, wr, D;
  gll_rule(k, xr, wr);
  gll_derivative(k, xr, D);
  // reference stiffness K_ref = D^T W D
  const int np = k + 1;
  std::vector<double> kref((size_t)np * np, 0.0);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      double s = 0.0;
      for (int q = 0; q < np; ++q) s += D[(size_t)q * np + i] * wr[q] * D[(size_t)q * np + j];
      kref[(size_t)i * np + j] = s;
    }
  const double h = (spec.b - spec.a) / (2.0 * ne);
  // banded assembly: kb[g][d] = K(g, g-k+d), d = 0..2k
  const int bw = 2 * k + 1;
  std::vector<double> kb((size_t)nfull * bw, 0.0), mf(nfull, 0.0), xf(nfull, 0.0);
  for (int el = 0; el < ne; ++el) {
    const int s = el * k;
    for (int i = 0; i < np; ++i) {
      mf[s + i] += h * wr[i];
      xf[s + i] = spec.a + h * (2.0 * el + 1.0 + xr[i]);
      for (int j = 0; j < np; ++j) kb[(size_t)(s + i) * bw + (j - i + k)] += kref[(size_t)i * np + j] / h;
    }
  }
  xf[0] = spec.a;
  xf[nfull - 1] = spec.b;
  // <grad 1, grad v> = 0: every row of the Neumann stiffness sums to zero up to one
  // rounding (diagonal = minus the off-diagonal row sum), before any restriction
  for (int g = 0; g < nfull; ++g) {
    double s = 0.0;
    for (int d = 0; d < bw; ++d)
      if (d != k) s += kb[(size_t)g * bw + d];
    kb[(size_t)g * bw + k] = -s;
  }
  if (dir) {
    // Dirichlet data at the removed end nodes: unknown d (full node d + 1) couples to
    // full node 0 through offset k - d - 1; unknown n-1-d (full n - d) to full node
    // n + 1 through offset k + d + 1
    const int depth = std::min(k, n);
    out.lift_lo.assign(depth, 0.0);
    out.lift_hi.assign(depth, 0.0);
    for (int d = 0; d < depth; ++d) {
      out.lift_lo[d] = -kb[(size_t)(d + 1) * bw + (k - d - 1)] / mf[d + 1];
      out.lift_hi[d] = -kb[(size_t)(n - d) * bw + (k + d + 1)] / mf[n - d];
    }
  } else if (!per) {
    out.lift_lo.assign(1, 1.0 / mf[0]);
    out.lift_hi.assign(1, 1.0 / mf[nfull - 1]);
  }
  if (per) {
    // fold the last node onto the first: its row (couplings through offsets
    // d <= k) adds onto row 0 (couplings through d >= k), its mass onto node 0
    for (int d = 0; d < bw; ++d) kb[d] += kb[(size_t)(nfull - 1) * bw + d];
    mf[0] += mf[nfull - 1];
  }
  const int off = dir ? 1 : 0;
  out.n = n;
  out.k = k;
  out.h = h;
  out.x.assign(xf.begin() + off, xf.begin() + off + n);
  out.mass.assign(mf.begin() + off, mf.begin() + off + n);
  out.hband.assign((size_t)n * bw, 0.0);
  auto column = [&](int g, int d) {  // unknown coupled to g through offset d - k, or -1
    int col = g - k + d;             // in restricted numbering
    if (per) return ((col % n) + n) % n;
    return col < 0 || col >= n ? -1 : col;
  };
  for (int g = 0; g < n; ++g)
    for (int d = 0; d < bw; ++d)
      if (column(g, d) >= 0) out.hband[(size_t)g * bw + d] = kb[(size_t)(g + off) * bw + d] / out.mass[g];
  // symmetric S1 = M^{-1/2} K M^{-1/2}, dense (periodic offsets that alias one
  // node add up)
  std::vector<double> mh(n);
  for (int g = 0; g < n; ++g) mh[g] = std::sqrt(out.mass[g]);
  std::vector<double> s1((size_t)n * n, 0.0);
  for (int g = 0; g < n; ++g)
    for (int d = 0; d < bw; ++d) {
      const int col = column(g, d);
      if (col < 0) continue;
      s1[(size_t)g * n + col] += kb[(size_t)(g + off) * bw + d] / (mh[g] * mh[col]);
    }
  // The uniform mesh is symmetric about the midpoint of [a, b]: the reflection
  // node i -> R(i) (n - 1 - i; periodic (n - i) mod n) commutes with K and M, so
  // every eigenvector can be taken symmetric (R s = s) or antisymmetric (R s = -s)
  // and the eigenproblem splits into one on the nrep orbit representatives
  // 0..nrep-1 and one on the nodd pairs {r, R(r)}, r != R(r).  Each block is
  // solved (Householder + implicit QR) and refined on its own; the eigenvectors
  // are built from the blocks, so mirrored entries are equal or opposite exactly.
  auto refl = [&](int i) { return per ? (n - i) % n : n - 1 - i; };
  const int nrep = per ? n / 2 + 1 : (n + 1) / 2;
  std::vector<int> pair_rep;  // representatives of the pairs, ascending
  for (int r = 0; r < nrep; ++r)
    if (refl(r) != r) pair_rep.push_back(r);
  const int nodd = (int)pair_rep.size();
  const double rs2 = 1.0 / std::sqrt(2.0);
  // symmetric block: basis e_r (fixed r) or (e_r + e_R(r)) / sqrt 2
  std::vector<double> ae((size_t)nrep * nrep), ao((size_t)nodd * nodd);
  auto wsym = [&](int r) { return refl(r) == r ? 1.0 : rs2; };
  auto orbit_sum = [&](int r, int c, double sign) {
    const int rr = refl(r), cc = refl(c);
    double v = s1[(size_t)r * n + c];
    if (cc != c) v += sign * s1[(size_t)r * n + cc];
    if (rr != r) {
      v += sign * s1[(size_t)rr * n + c];
      if (cc != c) v += s1[(size_t)rr * n + cc];
    }
    return v;
  };
  for (int i = 0; i < nrep; ++i)
    for (int j = 0; j < nrep; ++j) ae[(size_t)i * nrep + j] = wsym(i) * wsym(j) * orbit_sum(i, j, 1.0);
  for (int i = 0; i < nodd; ++i)
    for (int j = 0; j < nodd; ++j) ao[(size_t)i * nodd + j] = 0.5 * orbit_sum(pair_rep[i], pair_rep[j], -1.0);
  for (std::vector<double>* blk : {&ae, &ao}) {
    const int m = blk == &ae ? nrep : nodd;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) {
        const double v = 0.5 * ((*blk)[(size_t)i * m + j] + (*blk)[(size_t)j * m + i]);
        (*blk)[(size_t)i * m + j] = (*blk)[(size_t)j * m + i] = v;
      }
  }
  std::vector<double> lame(nrep), lamo(nodd);
  if (nrep) sym_eig(nrep, ae.data(), lame.data(), nthreads);
  if (nodd) sym_eig(nodd, ao.data(), lamo.data(), nthreads);
  // S_e = M^{-1/2} P_e Q_e,  S_o = M^{-1/2} P_o Q_o  (M is symmetric: the
  // representative's mass serves both nodes of a pair)
  std::vector<double> se((size_t)n * nrep, 0.0), so((size_t)n * std::max(nodd, 0), 0.0);
  for (int r = 0; r < nrep; ++r)
    for (int c = 0; c < nrep; ++c) {
      const double v = wsym(r) * ae[(size_t)r * nrep + c] / mh[r];
      se[(size_t)r * nrep + c] = v;
      se[(size_t)refl(r) * nrep + c] = v;
    }
  for (int j = 0; j < nodd; ++j) {
    const int r = pair_rep[j];
    for (int c = 0; c < nodd; ++c) {
      const double v = rs2 * ao[(size_t)j * nodd + c] / mh[r];
      so[(size_t)r * nodd + c] = v;
      so[(size_t)refl(r) * nodd + c] = -v;
    }
  }
  if (n > 1) {
    const std::vector<long double> ke = element_stiffness_ld(k, xr, spec.a, spec.b, ne);
    if (nrep) refine_eigenpairs(n, nrep, k, ne, ke, off, per, out.mass, lame, se, nthreads);
    if (nodd) refine_eigenpairs(n, nodd, k, ne, ke, off, per, out.mass, lamo, so, nthreads);
  }
  // natural order: all eigenpairs ascending (symmetric first among equal values)
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  auto lam_of = [&](int t) { return t < nrep ? lame[t] : lamo[t - nrep]; };
  std::stable_sort(order.begin(), order.end(), [&](int a2, int b2) { return lam_of(a2) < lam_of(b2); });
  out.lam.assign(n, 0.0);
  out.S.assign((size_t)n * n, 0.0);
  for (int c = 0; c < n; ++c) {
    const int t = order[c];
    out.lam[c] = lam_of(t);
    for (int r = 0; r < n; ++r)
      out.S[(size_t)r * n + c] = t < nrep ? se[(size_t)r * nrep + t] : so[(size_t)r * nodd + (t - nrep)];
  }
  // forward factor F = S^T M  (= Q^T M^{1/2})
  out.F.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) out.F[(size_t)c * n + r] = out.S[(size_t)r * n + c] * out.mass[r];
  // folded factors of the reflection-split transforms.  Folded vector of v:
  // v+_r = v_r + v_R(r), v-_r = v_r - v_R(r) for r < nrep (v+ = 2 v_r, v- = 0 at a
  // fixed node).  Forward: (F v)_sym = Ffold_sym v+, (F v)_anti = Ffold_anti v-,
  // with Ffold(mode, r) = F(mode, r), halved at fixed r for symmetric modes.
  // Backward: e = Bfold_sym c_sym, o = Bfold_anti c_anti on the representatives,
  // then u_r = e_r + o_r, u_R(r) = e_r - o_r.
  out.nrep = nrep;
  out.nodd = nodd;
  out.lam_fold.assign(n, 0.0);
  for (int t = 0; t < n; ++t) out.lam_fold[t] = lam_of(t);
  out.ffold.assign((size_t)n * nrep, 0.0);
  for (int t = 0; t < n; ++t)
    for (int r = 0; r < nrep; ++r) {
      const double s = t < nrep ? se[(size_t)r * nrep + t] : so[(size_t)r * nodd + (t - nrep)];
      out.ffold[(size_t)t * nrep + r] = s * out.mass[r] * (t < nrep && refl(r) == r ? 0.5 : 1.0);
    }
  out.bfold_sym.assign((size_t)nrep * nrep, 0.0);
  out.bfold_anti.assign((size_t)nrep * std::max(nodd, 0), 0.0);
  for (int r = 0; r < nrep; ++r) {
    for (int t = 0; t < nrep; ++t) out.bfold_sym[(size_t)r * nrep + t] = se[(size_t)r * nrep + t];
    for (int t = 0; t < nodd; ++t) out.bfold_anti[(size_t)r * nodd + t] = so[(size_t)r * nodd + t];
  }
}

}  // namespace semfd
