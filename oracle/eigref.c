/* Test infrastructure only (part of the oracle; see oracle/__init__.py).
 *
 * One extended-precision refinement step of a generalised symmetric-definite
 * eigen-decomposition  K S = M S diag(lam),  S^T M S = I,  M diagonal.
 *
 * Why: the fast-diagonalisation solve (paper Sec. 2.3, eq. 3D-Poisson) inherits
 * the error of its eigenpairs amplified by the condition number; an FP64 dense
 * eigensolver leaves absolute eigenvalue errors of order eps*lambda_max, which
 * at n ~ 1000 perturb the lowest (dominant) modes of the solution by ~1e-11.
 * The Newton-type refinement of Ogita & Aishima (Japan J. Indust. Appl. Math.
 * 35, 2018) restores them to FP64 rounding.  With X the current eigenvectors,
 * computed in x87 long double:
 *     T = X^T K X,   R = I - X^T M X,
 *     lam_i  = T_ii / (1 - R_ii),
 *     E_ii   = R_ii / 2,
 *     E_ij   = (T_ij + lam_j R_ij) / (lam_j - lam_i)   (i != j),
 *     X_new  = X (I + E).
 * Pairs closer than a relative 1e-15 keep only the symmetric part R_ij / 2.
 * With periodic conditions the spectrum has exactly double eigenvalues (the
 * translation by one element is a symmetry of the discrete operator, and its
 * Bloch phases +theta and -theta give the same eigenvalues) and, at the Bloch
 * phase pi, pairs split only by the discretisation error (1.4e-10 lambda_max
 * for Q^20 with 10 elements).  One Newton step across such a gap g leaves a
 * second-order error (eps lambda_max / g)^2 in S^T M S; inside the pair any
 * M-orthonormal basis has K s - lambda M s ~ eps lambda_max.  So pairs closer
 * than a relative 1e-8 are treated as one eigenspace there (symmetric part
 * only: no rotation inside it).
 *
 * K is not taken from its FP64 entries: the lowest eigenvalues come out of a
 * cancellation of ratio lambda_max / lambda_min, so FP64 rounding of K's entries
 * alone shifts them by ~1e-11 relative.  Instead K X is formed element by element
 * in long double from the reference nodes xr (k+1, FP64) and weights wr:
 * D_ij = l_j'(xr_i) by the Lagrange product formula with the diagonal set to minus
 * the off-diagonal row sum (as the paper's LegendreD does), K_ref = D^T W D, element
 * matrix K_ref / h (Appendix SEGenerator1D).  M (diagonal, well conditioned) is
 * used as given.  `off` = 1 for homogeneous Dirichlet (the end nodes are removed),
 * 0 for Neumann and periodic; `per` = 1 for periodic (full node ne*k is node 0).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

int oracle_eig_refine(int n, int k, int ne, int off, int per, double a, double b, const double *xr,
                      const double *wr,
                      const double *M, double *lam, double *S) {
  if (n <= 0) return 0;
  const size_t nn = (size_t)n * n;
  const int np = k + 1, nfull = ne * k + 1;
  long double *X = (long double *)malloc(nn * sizeof(long double));
  long double *KX = (long double *)malloc(nn * sizeof(long double));
  long double *T = (long double *)malloc(nn * sizeof(long double));
  long double *R = (long double *)malloc(nn * sizeof(long double));
  long double *L = (long double *)malloc((size_t)n * sizeof(long double));
  long double *Ke = (long double *)malloc((size_t)np * np * sizeof(long double));
  long double *D = (long double *)malloc((size_t)np * np * sizeof(long double));
  if (!X || !KX || !T || !R || !L || !Ke || !D) {
    free(X); free(KX); free(T); free(R); free(L); free(Ke); free(D);
    return 1;
  }
  for (size_t t = 0; t < nn; ++t) X[t] = S[t];
  /* element stiffness in long double */
  for (int i = 0; i < np; ++i) {
    long double wi = 1.0L;
    for (int m = 0; m < np; ++m)
      if (m != i) wi *= (long double)xr[i] - (long double)xr[m];
    long double rs = 0.0L;
    for (int j = 0; j < np; ++j) {
      if (j == i) continue;
      long double wj = 1.0L;
      for (int m = 0; m < np; ++m)
        if (m != j) wj *= (long double)xr[j] - (long double)xr[m];
      D[i * np + j] = (wi / wj) / ((long double)xr[i] - (long double)xr[j]);
      rs += D[i * np + j];
    }
    D[i * np + i] = -rs;
  }
  const long double h = ((long double)b - (long double)a) / (2.0L * ne);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      long double acc = 0.0L;
      for (int q = 0; q < np; ++q) acc += D[q * np + i] * (long double)wr[q] * D[q * np + j];
      Ke[i * np + j] = acc / h;
    }
  /* K X: rows of the full (ne*k+1)-node numbering, element by element; for Dirichlet
   * the removed end nodes carry zero in every column of X; periodic: full nodes
   * gf and gf + n are the same unknown (only node 0 has the alias n = ne*k) */
#pragma omp parallel for schedule(static)
  for (int g = 0; g < n; ++g) {
    long double *row = KX + (size_t)g * n;
    for (int j = 0; j < n; ++j) row[j] = 0.0L;
    for (int alias = 0; alias <= per; ++alias) {
      const int gf = g + off + alias * n; /* full index */
      if (gf >= nfull) continue;
      for (int e = (gf - 1) / k < 0 ? 0 : (gf - 1) / k; e <= gf / k && e < ne; ++e) {
        const int li = gf - e * k; /* local index of gf in element e */
        if (li < 0 || li > k) continue;
        for (int lj = 0; lj < np; ++lj) {
          const int qf = e * k + lj;
          const int q = per ? qf % n : qf - off;
          if (q < 0 || q >= n || qf >= nfull) continue;
          const long double kv = Ke[li * np + lj];
          const long double *xq = X + (size_t)q * n;
          for (int j = 0; j < n; ++j) row[j] += kv * xq[j];
        }
      }
    }
  }
  /* T = X^T (K X),  R = I - X^T M X  (row i of T and R owned by one thread) */
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < n; ++i) {
    long double *ti = T + (size_t)i * n, *ri = R + (size_t)i * n;
    for (int j = 0; j < n; ++j) ti[j] = ri[j] = 0.0L;
    for (int p = 0; p < n; ++p) {
      const long double xpi = X[(size_t)p * n + i];
      const long double mx = (long double)M[p] * xpi;
      const long double *kxp = KX + (size_t)p * n, *xp = X + (size_t)p * n;
      for (int j = 0; j < n; ++j) {
        ti[j] += xpi * kxp[j];
        ri[j] += mx * xp[j];
      }
    }
    for (int j = 0; j < n; ++j) ri[j] = (i == j ? 1.0L : 0.0L) - ri[j];
  }
  long double lmax = 0.0L;
  for (int i = 0; i < n; ++i) {
    L[i] = T[(size_t)i * n + i] / (1.0L - R[(size_t)i * n + i]);
    if (fabsl(L[i]) > lmax) lmax = fabsl(L[i]);
  }
  /* E overwrites T */
  const long double tiny = (per ? 1e-8L : 1e-15L) * (lmax > 0 ? lmax : 1.0L);
#pragma omp parallel for schedule(static)
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const size_t ij = (size_t)i * n + j;
      if (i == j) {
        T[ij] = 0.5L * R[ij];
      } else {
        const long double d = L[j] - L[i];
        T[ij] = fabsl(d) > tiny ? (T[ij] + L[j] * R[ij]) / d : 0.5L * R[ij];
      }
    }
  /* X_new = X + X E  -> S */
#pragma omp parallel for schedule(dynamic, 8)
  for (int p = 0; p < n; ++p) {
    long double *acc = KX + (size_t)p * n; /* reuse as accumulator row */
    const long double *xp = X + (size_t)p * n;
    for (int j = 0; j < n; ++j) acc[j] = xp[j];
    for (int i = 0; i < n; ++i) {
      const long double xpi = xp[i];
      const long double *ei = T + (size_t)i * n;
      for (int j = 0; j < n; ++j) acc[j] += xpi * ei[j];
    }
    for (int j = 0; j < n; ++j) S[(size_t)p * n + j] = (double)acc[j];
  }
  for (int i = 0; i < n; ++i) lam[i] = (double)L[i];
  free(X); free(KX); free(T); free(R); free(L); free(Ke); free(D);
  return 0;
}
