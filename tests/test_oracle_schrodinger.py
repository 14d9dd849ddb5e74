"""Pins of the oracle's variable-coefficient solver (alpha u - Lap u + V u = f by
PCG with the fast-diagonalisation solve of (shift I - Lap) as preconditioner,
the paper's Schrodinger-equation section), independent of the oracle itself:
dense direct solves, the spectrum bounds of the preconditioned operator, the
conjugate-gradient error bound, the order of accuracy on the paper's exact
solution, and the paper's iteration count for beta = 1."""
import math

import numpy as np
import pytest

import oracle as O
from workloads import SCHRODINGER_BOX, schrodinger_data



def _dense_a(prob, v):
    """alpha I + H_x (x) I (x) I + I (x) H_y (x) I + I (x) I (x) H_z + diag(V),
    assembled from the 1D matrices (row-major x, y, z; z fastest)."""
    nx, ny, nz = prob.shape
    hx, hy, hz = (prob.h_dense(a) for a in range(3))
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    a = (np.kron(np.kron(hx, iy), iz) + np.kron(np.kron(ix, hy), iz) + np.kron(np.kron(ix, iy), hz))
    return a + np.diag(prob.alpha + v.reshape(-1))


@pytest.mark.parametrize("case", [(2, (2, 3, 2), "neumann", 5.0), (3, (2, 2, 3), "dirichlet", 40.0)],
                         ids=["q2-neumann", "q3-dirichlet"])
def test_pcg_equals_dense_solve(case):
    """A general positive potential (not the paper's): PCG to 1e-14 equals the
    dense LU solution of the assembled nodal system."""
    k, ne, bc, beta = case
    box = (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5)
    prob = O.Problem(k, ne, box, 0.7, bc)
    rng = np.random.default_rng(11)
    v = rng.uniform(0.0, beta, size=prob.shape)
    f = rng.standard_normal(prob.shape)
    ref = np.linalg.solve(_dense_a(prob, v), f.reshape(-1)).reshape(prob.shape)
    u, it, hist = O.pcg_schrodinger(prob, v, f, prob.alpha + beta / 2, tol=1e-14, max_iter=200)
    assert it < 200 and hist[-1] <= 1e-14
    assert O.rel_max_err(u, ref) <= 1e-12
    # the operator itself against the assembled matrix
    w = rng.standard_normal(prob.shape)
    aw = (_dense_a(prob, v) @ w.reshape(-1)).reshape(prob.shape)
    assert O.rel_max_err(O.schrodinger_apply(prob, v, w), aw) <= 1e-13


@pytest.mark.parametrize("beta", [1.0, 10.0, 100.0])
def test_preconditioned_spectrum_bounds(beta):
    """With 0 <= V <= beta and P = shift I + H_3, shift = alpha + beta/2, every
    Rayleigh quotient <w, A w>_M / <w, P w>_M lies in [alpha/shift, (alpha+beta)/shift]
    (the Laplacian parts cancel); checked on random and on localised vectors."""
    alpha = 1.0
    prob = O.Problem(4, (3, 4, 3), SCHRODINGER_BOX, alpha, "neumann")
    v, _, _ = schrodinger_data(*(o.x for o in prob.axes), alpha, beta)
    assert v.min() >= 0.0 and v.max() <= beta
    shift = alpha + beta / 2
    m3 = prob.mass3()
    rng = np.random.default_rng(3)
    lo, hi = alpha / shift, (alpha + beta) / shift
    qs = []
    for t in range(40):
        w = rng.standard_normal(prob.shape)
        if t % 2:  # concentrate where V is large or small
            w *= (v / beta) ** 4 if t % 4 == 1 else (1.0 - v / beta) ** 4
        aw = O.schrodinger_apply(prob, v, w)
        pw = shift * w + O.apply_h3(prob, w)
        qs.append(np.sum(m3 * w * aw) / np.sum(m3 * w * pw))
    assert lo - 1e-12 <= min(qs) and max(qs) <= hi + 1e-12, (min(qs), max(qs), lo, hi)


@pytest.mark.parametrize("beta", [1.0, 10.0])
def test_pcg_error_within_cg_bound(beta):
    """Conjugate gradients: ||e_k||_A <= 2 rho^k ||e_0||_A with
    rho = (sqrt(kappa) - 1)/(sqrt(kappa) + 1), kappa = (alpha + beta)/alpha the
    bound on the preconditioned condition number; the error is measured against
    the dense solution."""
    alpha = 1.0
    prob = O.Problem(3, (3, 2, 3), SCHRODINGER_BOX, alpha, "neumann")
    v, _, _ = schrodinger_data(*(o.x for o in prob.axes), alpha, beta)
    f = np.random.default_rng(5).standard_normal(prob.shape)
    a = _dense_a(prob, v)
    m3 = prob.mass3().reshape(-1)
    ref = np.linalg.solve(a, f.reshape(-1))

    def anorm(e):
        e = e.reshape(-1)
        return math.sqrt(float(np.sum(m3 * e * (a @ e))))

    kappa = (alpha + beta) / alpha
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    e0 = anorm(ref)
    for k in range(1, 9):
        u, it, _ = O.pcg_schrodinger(prob, v, f, alpha + beta / 2, tol=0.0, max_iter=k)
        assert anorm(u.reshape(-1) - ref) <= 2 * rho ** k * e0 * (1 + 1e-9) + 1e-13 * e0, k


def test_manufactured_solution_converges_at_order_k_plus_2():
    """The paper's exact solution on [-16, 16]^3 (homogeneous Neumann), Q^5, beta = 1:
    the max-norm error falls by at least 2^(k+1) per halving of h (observed order
    ~ k + 2 = 7)."""
    errs = []
    for ne in (4, 8):
        prob = O.Problem(5, (ne, ne, ne), SCHRODINGER_BOX, 1.0, "neumann")
        v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, 1.0)
        u, it, _ = O.pcg_schrodinger(prob, v, f, 1.5, tol=1e-13)
        errs.append(np.max(np.abs(u - ue)))
    assert errs[0] / errs[1] >= 2.0 ** 6, errs
    assert errs[1] <= 1e-7, errs


@pytest.mark.parametrize("ne", [6, 12])
def test_beta1_converges_in_about_ten_iterations(ne):
    """Table tab7c: with beta = 1 PCG needs 10 iterations on every mesh (periodic
    conditions there; with the homogeneous Neumann conditions used here and the
    stop ||r||_M <= 1e-12 ||f||_M the count is 9-10)."""
    prob = O.Problem(5, (ne, ne, ne), SCHRODINGER_BOX, 1.0, "neumann")
    v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, 1.0)
    u, it, hist = O.pcg_schrodinger(prob, v, f, 1.5, tol=1e-12)
    assert 8 <= it <= 11, it
    assert all(b < a for a, b in zip(hist, hist[1:]))  # monotone residual decrease at kappa <= 2


def test_q20_robustness():
    """Sec. robustness: Q^20 on the Schrodinger problem stays accurate (the paper's
    Table tab8 reports max errors ~1e-13 on fine periodic meshes); here 5^3
    elements, beta = 1 and 10 (4.8e-14 and 3.2e-14 here)."""
    for beta in (1.0, 10.0):
        prob = O.Problem(20, (5, 5, 5), SCHRODINGER_BOX, 1.0, "neumann")
        v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, beta)
        u, it, _ = O.pcg_schrodinger(prob, v, f, 1.0 + beta / 2, tol=1e-14)
        err = np.max(np.abs(u - ue))
        assert err <= 2e-13, (beta, err)
