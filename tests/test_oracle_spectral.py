"""Pins of the oracle's spectral multipliers on the fast-diagonalisation
transforms (u = g(H_3 + a I) f with g(x) = exp(-t x) or x^(-s)): dense matrix
functions of the assembled operator, the solve of eq. 3D-Poisson as the power
s = 1, the semigroup property, and the decay of an exact eigenfunction."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O


def _dense_h(prob):
    nx, ny, nz = prob.shape
    hx, hy, hz = (prob.h_dense(a) for a in range(3))
    ix, iy, iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return np.kron(np.kron(hx, iy), iz) + np.kron(np.kron(ix, hy), iz) + np.kron(np.kron(ix, iy), hz)


def _dense_power(prob, a, s):
    """(H_3 + a I)^(-s) through the symmetric form M^(1/2) (H_3 + a I) M^(-1/2)."""
    m = np.sqrt(prob.mass3().reshape(-1))
    b = m[:, None] * (_dense_h(prob) + a * np.eye(m.size)) / m[None, :]
    w, q = np.linalg.eigh(0.5 * (b + b.T))
    return (q * w ** (-s)) @ q.T / m[:, None] * m[None, :]


CASES = [(2, (2, 3, 2), "neumann", 0.5), (3, (2, 2, 3), "dirichlet", 0.0)]


@pytest.mark.parametrize("case", CASES, ids=["q2-neumann", "q3-dirichlet"])
def test_exp_equals_dense_expm(case):
    k, ne, bc, a = case
    prob = O.Problem(k, ne, (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5), 1.0, bc)
    f = np.random.default_rng(7).standard_normal(prob.shape)
    for t in (1e-3, 0.05, 0.3):
        ref = (scipy.linalg.expm(-t * (_dense_h(prob) + a * np.eye(f.size))) @ f.reshape(-1)).reshape(prob.shape)
        assert O.rel_max_err(O.spectral_apply(prob, "exp", a, t, f), ref) <= 1e-11, t


@pytest.mark.parametrize("case", CASES, ids=["q2-neumann", "q3-dirichlet"])
def test_power_equals_dense_matrix_power(case):
    k, ne, bc, a = case
    if bc == "neumann":
        a = 0.5  # a > 0: the constant mode has lambda = 0
    prob = O.Problem(k, ne, (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5), 1.0, bc)
    f = np.random.default_rng(8).standard_normal(prob.shape)
    for s in (0.5, 1.7, -0.5):
        ref = (_dense_power(prob, a, s) @ f.reshape(-1)).reshape(prob.shape)
        assert O.rel_max_err(O.spectral_apply(prob, "power", a, s, f), ref) <= 1e-11, s


def test_power_one_is_the_solve_and_half_twice_too():
    prob = O.Problem(4, (3, 4, 2), (-1, 1, -1, 1, -1, 1), 2.0, "dirichlet")
    f = np.random.default_rng(9).standard_normal(prob.shape)
    sol = O.fd_solve(prob, f)
    assert O.rel_max_err(O.spectral_apply(prob, "power", 2.0, 1.0, f), sol) <= 1e-13
    half = O.spectral_apply(prob, "power", 2.0, 0.5, O.spectral_apply(prob, "power", 2.0, 0.5, f))
    assert O.rel_max_err(half, sol) <= 1e-12


def test_exp_semigroup_and_identity():
    prob = O.Problem(5, (2, 3, 3), (0, 1, 0, 2, 0, 1), 1.0, "neumann")
    f = np.random.default_rng(10).standard_normal(prob.shape)
    assert O.rel_max_err(O.spectral_apply(prob, "exp", 0.3, 0.0, f), f) <= 1e-13
    two = O.spectral_apply(prob, "exp", 0.3, 0.02, O.spectral_apply(prob, "exp", 0.3, 0.03, f))
    assert O.rel_max_err(two, O.spectral_apply(prob, "exp", 0.3, 0.05, f)) <= 1e-12


def test_exp_decays_an_eigenfunction_at_its_rate():
    """sin(pi x) sin(pi y) sin(pi z) on [-1, 1]^3 (Dirichlet) is an eigenfunction of
    -Lap with eigenvalue 3 pi^2, so exp(-t(-Lap + a)) multiplies it by
    exp(-t (3 pi^2 + a)), up to the Q^6 discretisation error."""
    prob = O.Problem(6, (6, 6, 6), (-1, 1, -1, 1, -1, 1), 1.0, "dirichlet")
    x, y, z = (o.x for o in prob.axes)
    f = np.sin(math.pi * x)[:, None, None] * np.sin(math.pi * y)[None, :, None] * np.sin(math.pi * z)[None, None, :]
    t, a = 0.02, 1.0
    u = O.spectral_apply(prob, "exp", a, t, f)
    assert O.rel_max_err(u, math.exp(-t * (3 * math.pi ** 2 + a)) * f) <= 1e-8
