"""Pins of the oracle's 1D layer against closed forms, exact quadrature and
textbook special cases (no GPU)."""
import math

import numpy as np
import pytest

import oracle as O


# ---- GLL points and weights -------------------------------------------------

@pytest.mark.parametrize("k,nodes,weights", [
    (1, [-1, 1], [1, 1]),
    (2, [-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
    (3, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    (4, [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
])
def test_gll_closed_forms(k, nodes, weights):
    x, w = O.gll(k)
    np.testing.assert_allclose(x, nodes, rtol=0, atol=1e-15)
    np.testing.assert_allclose(w, weights, rtol=2e-15, atol=0)


@pytest.mark.parametrize("k", list(range(1, 13)) + [16, 20])
def test_gll_exact_to_degree_2k_minus_1(k):
    x, w = O.gll(k)
    assert abs(w.sum() - 2.0) < 1e-14
    for m in range(0, 2 * k):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 5e-14, (k, m)
    # and not exact at degree 2k (Lobatto rules lose two degrees); the defect shrinks
    # quickly with k, so only the low orders are checked
    if k <= 8:
        m = 2 * k
        assert abs(np.dot(w, x ** m) - 2.0 / (m + 1)) > 1e-10


def test_gll_nodes_are_roots_of_legendre_derivative():
    # interior nodes are the zeros of P_k'(x) = k (x P_k - P_{k-1}) / (x^2 - 1)
    for k in (5, 9, 20):
        x, _ = O.gll(k)
        xi = x[1:-1]
        p, pm1 = O.legendre(k, xi)
        dp = k * (xi * p - pm1) / (xi * xi - 1)
        assert np.max(np.abs(dp)) < 1e-11 * k * k


# ---- differentiation matrix and element matrices ---------------------------

@pytest.mark.parametrize("k", [1, 2, 4, 7, 12])
def test_diff_matrix_exact_on_polynomials(k):
    x, _ = O.gll(k)
    d = O.diff_matrix(x)
    for m in range(0, k + 1):
        deriv = m * x ** (m - 1) if m else np.zeros_like(x)
        np.testing.assert_allclose(d @ x ** m, deriv, atol=1e-12 * max(1, k) ** 2)


@pytest.mark.parametrize("k", [2, 4, 6, 10])
def test_diff_matrix_gll_closed_form(k):
    # closed form for Legendre-Gauss-Lobatto: D_ij = P_k(x_i) / (P_k(x_j)(x_i - x_j)),
    # D_00 = -k(k+1)/4, D_kk = k(k+1)/4, other diagonal entries 0.
    x, _ = O.gll(k)
    d = O.diff_matrix(x)
    p, _ = O.legendre(k, x)
    ref = np.zeros_like(d)
    for i in range(k + 1):
        for j in range(k + 1):
            if i != j:
                ref[i, j] = p[i] / (p[j] * (x[i] - x[j]))
    ref[0, 0] = -k * (k + 1) / 4
    ref[k, k] = k * (k + 1) / 4
    np.testing.assert_allclose(d, ref, atol=1e-12 * k * k)


def test_element_stiffness_textbook_k1_k2():
    _, _, k1 = O.element_matrices(1)
    np.testing.assert_allclose(k1, [[0.5, -0.5], [-0.5, 0.5]], atol=1e-15)
    _, _, k2 = O.element_matrices(2)
    np.testing.assert_allclose(k2, np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / 6.0, atol=1e-14)


@pytest.mark.parametrize("k", [2, 3, 5, 8, 20])
def test_element_stiffness_energy_of_legendre(k):
    # v = P_k at the nodes: v^T K_ref v = int_{-1}^{1} P_k'(x)^2 dx = k (k + 1), exact because the
    # integrand has degree 2k - 2 <= 2k - 1.
    x, _, kref = O.element_matrices(k)
    v, _ = O.legendre(k, x)
    assert abs(v @ kref @ v - k * (k + 1)) < 1e-11 * k * k
    # constants are in the kernel
    assert np.max(np.abs(kref @ np.ones(k + 1))) < 1e-11 * k * k


# ---- assembled 1D operators ----------------------------------------------------

@pytest.mark.parametrize("k,ne,a,b", [(1, 7, 0.0, 1.0), (4, 5, -1.0, 1.0), (6, 3, 0.0, 2 * math.pi), (20, 2, -16, 16)])
def test_assembly_neumann_invariants(k, ne, a, b):
    o = O.axis_operators(k, ne, a, b, "neumann")
    n = ne * k + 1
    assert o.K.shape == (n, n) and o.M.shape == (n,)
    assert abs(o.x[0] - a) < 1e-15 and abs(o.x[-1] - b) < 1e-13
    assert np.all(np.diff(o.x) > 0)
    # element boundaries sit at a + 2 h e
    np.testing.assert_allclose(o.x[::k], a + 2 * o.h * np.arange(ne + 1), atol=1e-13 * max(1, abs(b)))
    np.testing.assert_allclose(o.K, o.K.T, atol=0)
    assert np.max(np.abs(o.K @ np.ones(n))) < 1e-10 * np.max(np.abs(o.K))
    assert abs(o.M.sum() - (b - a)) < 1e-13 * (b - a)
    # exact integrals of polynomials of degree <= 2k-1 with the lumped mass
    if k >= 2:
        assert abs(o.M @ o.x ** 2 - (b ** 3 - a ** 3) / 3) < 1e-12 * max(1, abs(b)) ** 3
        # energy of u = x^2: int (2x)^2 = 4 (b^3 - a^3) / 3 (stiffness exact for degree <= k)
        u = o.x ** 2
        assert abs(u @ o.K @ u - 4 * (b ** 3 - a ** 3) / 3) < 1e-10 * max(1, abs(b)) ** 3


def test_assembly_dirichlet_sizes():
    for k, ne in [(1, 8), (4, 8), (4, 250), (5, 2)]:
        o = O.axis_operators(k, ne, -1, 1, "dirichlet")
        assert o.x.size == ne * k - 1
        assert np.all(np.abs(o.x) < 1)


# ---- 1D eigen-decomposition ----------------------------------------------------

@pytest.mark.parametrize("ne", [4, 9, 16])
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_k1_closed_form_spectra(ne, bc):
    # Q^1 with lumped mass is the second-order finite-difference Laplacian:
    # lambda_j = (4 / dx^2) sin^2(j pi / (2 ne)), j = 1..ne-1 (Dirichlet, DST-I) or
    # j = 0..ne (Neumann, DCT-I).
    a, b = -1.0, 1.0
    dx = (b - a) / ne
    o = O.axis_operators(1, ne, a, b, bc)
    lam, _, _ = O.axis_eigen(o)
    js = np.arange(1, ne) if bc == "dirichlet" else np.arange(0, ne + 1)
    ref = 4.0 / dx ** 2 * np.sin(js * np.pi / (2 * ne)) ** 2
    np.testing.assert_allclose(lam, ref, rtol=1e-13, atol=1e-12)


def _check_invariants(o, tol=1e-13):
    lam, s, f = O.axis_eigen(o)
    n = lam.size
    assert np.all(np.diff(lam) >= 0)
    # S^T M S = I
    g = s.T @ (o.M[:, None] * s)
    assert np.max(np.abs(g - np.eye(n))) <= tol, np.max(np.abs(g - np.eye(n)))
    # K S = M S Lambda, scale-free per column
    res = o.K @ s - (o.M[:, None] * s) * lam[None, :]
    kinf = np.max(np.sum(np.abs(o.K), axis=1))
    rel = np.max(np.max(np.abs(res), axis=0) / (kinf * np.max(np.abs(s), axis=0)))
    assert rel <= tol, rel
    # F = S^T M is the inverse of S
    assert np.max(np.abs(f @ s - np.eye(n))) <= tol
    return lam


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7, 8, 20])
@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_eigen_invariants(k, bc):
    _check_invariants(O.axis_operators(k, 6, -1.0, 1.0, bc))


def test_eigen_invariants_n999():
    lam = _check_invariants(O.axis_operators(4, 250, -1.0, 1.0, "dirichlet"))
    # smallest eigenvalue approaches the continuous (pi/2)^2 of -d2/dx2 on [-1,1]
    assert abs(lam[0] - (math.pi / 2) ** 2) < 1e-9


def test_eigen_against_generalized_solver():
    import scipy.linalg
    o = O.axis_operators(5, 7, 0.0, 3.0, "neumann")
    lam, _, _ = O.axis_eigen(o)
    ref = scipy.linalg.eigh(o.K, np.diag(o.M), eigvals_only=True)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-12 * lam[-1])


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_lowest_eigenvalues_match_continuous_spectrum_n999(bc):
    # -u'' on [-1, 1]: Dirichlet lambda_j = (j pi / 2)^2, j >= 1; Neumann j >= 0.  With Q^4 and
    # h = 1/250 the discretisation error of the low modes is ~ (j pi h / 2)^8, far below rounding,
    # so the computed pairs must sit on the continuous values to rounding of the low modes.
    o = O.axis_operators(4, 250, -1.0, 1.0, bc)
    lam, _, _ = O.axis_eigen(o)
    j = np.arange(1, 6) if bc == "dirichlet" else np.arange(0, 5)
    err = np.abs(lam[:5] - (j * np.pi / 2) ** 2)
    assert np.all(err <= 5e-14 * (1 + j ** 2)), err
