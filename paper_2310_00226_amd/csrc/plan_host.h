// Host-side 1D operator construction and eigen-solver (FP64).
#pragma once
#include <vector>

namespace semfd {

struct AxisSpec {
  int k;           // polynomial degree
  int ne;          // number of elements
  double a, b;     // interval
  bool dirichlet;         // homogeneous Dirichlet (true) or Neumann / periodic (false)
  bool periodic = false;  // periodic: the node at b is the node at a (n = ne k)
  bool operator==(const AxisSpec& o) const {
    return k == o.k && ne == o.ne && a == o.a && b == o.b && dirichlet == o.dirichlet && periodic == o.periodic;
  }
};

struct AxisData {
  int n = 0, k = 0;
  double h = 0;
  std::vector<double> x;      // node coordinates (n)
  std::vector<double> mass;   // lumped mass diagonal (n)
  std::vector<double> hband;  // H = M^{-1} K banded rows: n x (2k+1), entry [g][d] = H(g, g-k+d)
                              // (periodic: the coupling of node g through offset d - k to node
                              // (g-k+d) mod n; offsets that alias one node keep separate entries)
  // non-homogeneous boundary data: the nodal right-hand side gains lift_lo[d] g_lo
  // at unknown d and lift_hi[d] g_hi at unknown n-1-d (Dirichlet: -H(d, end node)
  // of the full-grid assembly for the min(k, n) unknowns next to each end;
  // Neumann: 1 / M at the end node; periodic: none)
  std::vector<double> lift_lo, lift_hi;
  std::vector<double> lam;    // eigenvalues ascending (n)
  std::vector<double> S;      // backward factor S (n x n row-major), K S = M S Lambda, S^T M S = I
  std::vector<double> F;      // forward factor F = S^T M (n x n row-major)
  // Reflection split (node i -> R(i) = n - 1 - i, periodic (n - i) mod n): nrep
  // orbit representatives 0..nrep-1, nodd antisymmetric eigenvectors (n - nrep).
  // Mode order "folded": the nrep symmetric eigenvectors, then the nodd
  // antisymmetric ones, each ascending.
  int nrep = 0, nodd = 0;
  std::vector<double> lam_fold;    // eigenvalues in folded mode order (n)
  std::vector<double> ffold;       // n x nrep: forward factor on the folded vector (see build_axis)
  std::vector<double> bfold_sym;   // nrep x nrep: symmetric eigenvectors on the representatives
  std::vector<double> bfold_anti;  // nrep x nodd: antisymmetric eigenvectors on the representatives
};

void tridiag_qr(int n, double* d, double* e, double* z, int ldz, int nthreads);
void householder_tridiag(int n, double* a, double* d, double* e, int nthreads);
void sym_eig(int n, double* a, double* w, int nthreads);
void gll_rule(int k, std::vector<double>& x, std::vector<double>& w);
void build_axis(const AxisSpec& spec, AxisData& out, int nthreads);

}  // namespace semfd
