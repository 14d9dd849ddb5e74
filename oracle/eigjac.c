/* Test infrastructure only (part of the oracle; see oracle/__init__.py).
 *
 * Extended-precision generalised eigenpairs  K S = M S diag(lam),  S^T M S = I
 * of one assembled 1D axis (paper Sec. 2.3: the symmetric form
 * S1 = M^{-1/2} K M^{-1/2} = Q diag(lam) Q^T,  S = M^{-1/2} Q).
 *
 * Why extended precision: the fast-diagonalisation solve divides by
 * lx + ly + lz + alpha, so an eigenvalue error of eps * lambda_max (what any FP64
 * eigensolver of S1 leaves) is a relative error of eps * lambda_max / lambda_min
 * in the dominant low modes of the solution (~1e-11 at n ~ 1000).
 *
 * Route (cyclic Jacobi, Golub & Van Loan, Matrix Computations, Sec. 8.5):
 *  1. K and M are assembled in x87 long double from the reference-element
 *     stiffness and GLL weights, which the caller computes in high precision and
 *     passes as (hi, lo) pairs of doubles; element matrices are K_ref / h and
 *     h diag(w) (Appendix generator), shared end nodes are summed, Dirichlet
 *     drops the two end nodes, periodic adds the last node onto the first.
 *  2. The caller's FP64 eigenvectors Q0 of S1 (any dense solver) give a
 *     starting basis; one Newton-Schulz step Q = Q0 (3 I - Q0^T Q0) / 2 makes it
 *     orthonormal to long-double rounding.
 *  3. B = Q^T S1 Q in long double, S1 applied through the sparse rows of K.
 *  4. Cyclic Jacobi sweeps on B (parallel round-robin ordering of the pairs: in
 *     each round the n/2 pairs are disjoint, so their rotations commute), each
 *     rotation also applied to the columns of Q, until no off-diagonal entry
 *     exceeds LDBL_EPSILON * sqrt(|b_pp b_qq|).
 *  5. lam = diag(B) ascending, S = M^{-1/2} Q rounded to double.
 *
 * Arguments: n unknowns; k degree; ne elements; off = 1 Dirichlet (end nodes
 * removed), 0 otherwise; per = 1 periodic; kref_hi/lo (k+1)^2 row-major
 * reference stiffness; w_hi/lo (k+1) weights; h_hi/lo the half element width;
 * q0 (n x n row-major, column j an eigenvector of the FP64 S1); outputs lam (n)
 * and s (n x n row-major, column j the M-orthonormal eigenvector of lam[j]).
 * Returns 0, 1 on allocation failure, 2 if the sweeps do not converge.
 */
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

static ld two(const double *hi, const double *lo, int i) { return (ld)hi[i] + (ld)lo[i]; }

int oracle_eig_jacobi(int n, int k, int ne, int off, int per, const double *kref_hi, const double *kref_lo,
                      const double *w_hi, const double *w_lo, double h_hi, double h_lo, const double *q0,
                      double *lam, double *s) {
  if (n <= 0) return 0;
  const int np = k + 1;
  const size_t nn = (size_t)n * n;
  const ld h = (ld)h_hi + (ld)h_lo;
  int status = 0;
  ld *K = (ld *)calloc(nn, sizeof(ld));
  ld *Mh = (ld *)calloc((size_t)n, sizeof(ld)); /* M^{1/2} */
  ld *Q = (ld *)malloc(nn * sizeof(ld));
  ld *T = (ld *)malloc(nn * sizeof(ld));
  ld *B = (ld *)malloc(nn * sizeof(ld));
  int *nzc = (int *)malloc(nn * sizeof(int)), *nzn = (int *)calloc((size_t)n, sizeof(int));
  int *order = (int *)malloc((size_t)(n + 1) * sizeof(int)), *pp = (int *)malloc((size_t)(n + 1) * sizeof(int));
  ld *rc = (ld *)malloc((size_t)(n + 1) * sizeof(ld)), *rs = (ld *)malloc((size_t)(n + 1) * sizeof(ld));
  if (!K || !Mh || !Q || !T || !B || !nzc || !nzn || !order || !pp || !rc || !rs) {
    status = 1;
    goto done;
  }

  /* 1. assembly: full node g = e k + i -> unknown g - off (Dirichlet drops 0 and
   * nfull - 1), periodic maps full node ne k to unknown 0 */
  for (int e = 0; e < ne; ++e)
    for (int i = 0; i < np; ++i) {
      int gi = e * k + i;
      if (per) gi %= n; else gi -= off;
      if (gi < 0 || gi >= n) continue;
      Mh[gi] += h * two(w_hi, w_lo, i);
      for (int j = 0; j < np; ++j) {
        int gj = e * k + j;
        if (per) gj %= n; else gj -= off;
        if (gj < 0 || gj >= n) continue;
        K[(size_t)gi * n + gj] += two(kref_hi, kref_lo, i * np + j) / h;
      }
    }
  for (int i = 0; i < n; ++i) {
    Mh[i] = sqrtl(Mh[i]);
    for (int j = 0; j < n; ++j)
      if (K[(size_t)i * n + j] != 0.0L) nzc[(size_t)i * n + nzn[i]++] = j;
  }

  /* 2. Newton-Schulz orthonormalisation: T = Q0^T Q0, Q = Q0 (3 I - T) / 2 */
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      ld acc = 0.0L;
      for (int p = 0; p < n; ++p) acc += (ld)q0[(size_t)p * n + i] * (ld)q0[(size_t)p * n + j];
      T[(size_t)i * n + j] = (i == j ? 3.0L : 0.0L) - acc;
    }
#pragma omp parallel for schedule(dynamic, 4)
  for (int p = 0; p < n; ++p) {
    ld *row = Q + (size_t)p * n;
    for (int j = 0; j < n; ++j) row[j] = 0.0L;
    for (int i = 0; i < n; ++i) {
      const ld x = 0.5L * (ld)q0[(size_t)p * n + i];
      const ld *ti = T + (size_t)i * n;
      for (int j = 0; j < n; ++j) row[j] += x * ti[j];
    }
  }

  /* 3. T = S1 Q = M^{-1/2} K M^{-1/2} Q (sparse rows of K), B = Q^T T */
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i) {
    ld *row = T + (size_t)i * n;
    for (int j = 0; j < n; ++j) row[j] = 0.0L;
    for (int t = 0; t < nzn[i]; ++t) {
      const int c = nzc[(size_t)i * n + t];
      const ld kv = K[(size_t)i * n + c] / (Mh[i] * Mh[c]);
      const ld *qc = Q + (size_t)c * n;
      for (int j = 0; j < n; ++j) row[j] += kv * qc[j];
    }
  }
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      ld acc = 0.0L;
      for (int p = 0; p < n; ++p) acc += Q[(size_t)p * n + i] * T[(size_t)p * n + j];
      B[(size_t)i * n + j] = acc;
    }
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const ld v = 0.5L * (B[(size_t)i * n + j] + B[(size_t)j * n + i]);
      B[(size_t)i * n + j] = B[(size_t)j * n + i] = v;
    }

  /* 4. cyclic Jacobi, round-robin ordering: players 0..m-1 (m = n rounded up to
   * even; player n is a bye when n is odd); in round r player order[0] stays and
   * the others rotate; pairs (order[i], order[m-1-i]) */
  {
    const int m = n + (n & 1);
    int sweep;
    for (sweep = 0; sweep < 40; ++sweep) {
      long active_total = 0;
      for (int i = 0; i < m; ++i) order[i] = i;
      for (int round = 0; round < m - 1; ++round) {
        int npairs = 0;
        for (int i = 0; i < m / 2; ++i) {
          int p = order[i], q = order[m - 1 - i];
          if (p >= n || q >= n) continue;
          if (p > q) { const int t = p; p = q; q = t; }
          const ld bpq = B[(size_t)p * n + q], bpp = B[(size_t)p * n + p], bqq = B[(size_t)q * n + q];
          if (fabsl(bpq) <= LDBL_EPSILON * sqrtl(fabsl(bpp * bqq)) || bpq == 0.0L) continue;
          /* Rutishauser: theta = (b_qq - b_pp) / (2 b_pq), t the smaller root of
           * t^2 + 2 theta t - 1 = 0; J = [c s; -s c] zeroes b_pq */
          const ld theta = (bqq - bpp) / (2.0L * bpq);
          const ld t = (theta >= 0 ? 1.0L : -1.0L) / (fabsl(theta) + sqrtl(1.0L + theta * theta));
          const ld c = 1.0L / sqrtl(1.0L + t * t);
          pp[2 * npairs] = p;
          pp[2 * npairs + 1] = q;
          rc[npairs] = c;
          rs[npairs] = t * c;
          /* new diagonal from the accurate form; the off-diagonal pair becomes 0 */
          T[2 * npairs] = bpp - t * bpq;
          T[2 * npairs + 1] = bqq + t * bpq;
          ++npairs;
        }
        if (npairs) {
          active_total += npairs;
          /* B <- B J (columns p, q of every row) and Q <- Q J */
#pragma omp parallel for schedule(static)
          for (int r = 0; r < n; ++r) {
            ld *br = B + (size_t)r * n, *qr = Q + (size_t)r * n;
            for (int a = 0; a < npairs; ++a) {
              const int p = pp[2 * a], q = pp[2 * a + 1];
              const ld c = rc[a], sn = rs[a];
              const ld xp = br[p], xq = br[q];
              br[p] = c * xp - sn * xq;
              br[q] = sn * xp + c * xq;
              const ld yp = qr[p], yq = qr[q];
              qr[p] = c * yp - sn * yq;
              qr[q] = sn * yp + c * yq;
            }
          }
          /* B <- J^T B (rows p, q) */
#pragma omp parallel for schedule(static)
          for (int a = 0; a < npairs; ++a) {
            const int p = pp[2 * a], q = pp[2 * a + 1];
            const ld c = rc[a], sn = rs[a];
            ld *bp = B + (size_t)p * n, *bq = B + (size_t)q * n;
            for (int j = 0; j < n; ++j) {
              const ld xp = bp[j], xq = bq[j];
              bp[j] = c * xp - sn * xq;
              bq[j] = sn * xp + c * xq;
            }
          }
          for (int a = 0; a < npairs; ++a) {
            const int p = pp[2 * a], q = pp[2 * a + 1];
            B[(size_t)p * n + p] = T[2 * a];
            B[(size_t)q * n + q] = T[2 * a + 1];
            B[(size_t)p * n + q] = B[(size_t)q * n + p] = 0.0L;
          }
        }
        /* rotate every player but order[0] one place */
        const int last = order[m - 1];
        for (int i = m - 1; i > 1; --i) order[i] = order[i - 1];
        order[1] = last;
      }
      if (active_total == 0) break;
    }
    if (sweep == 40) status = 2;
  }

  /* 5. ascending eigenvalues, S = M^{-1/2} Q */
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 1; i < n; ++i) { /* insertion sort keeps equal eigenvalues in place */
    const int v = order[i];
    int j = i - 1;
    while (j >= 0 && B[(size_t)order[j] * n + order[j]] > B[(size_t)v * n + v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  for (int c = 0; c < n; ++c) {
    const int src = order[c];
    lam[c] = (double)B[(size_t)src * n + src];
    for (int r = 0; r < n; ++r) s[(size_t)r * n + c] = (double)(Q[(size_t)r * n + src] / Mh[r]);
  }

done:
  free(K); free(Mh); free(Q); free(T); free(B); free(nzc); free(nzn); free(order); free(pp); free(rc); free(rs);
  return status;
}
