"""Pins of the oracle's periodic boundary condition (Sec. 2.4 lists periodic
boundaries among those of the same tensor form; the Schroedinger tables of
Sec. 4 use them), independent of the fold-and-add assembly the oracle uses:
the finite-difference closed form of Q^1, a Bloch-wave assembly of the spectrum
for Q^k, the continuous spectrum, dense direct solves, the translation symmetry
of the discrete problem, and spectral convergence on a periodic exact solution."""
import math

import numpy as np
import pytest

import oracle as O
from workloads import SCHRODINGER_BOX, schrodinger_data


def test_periodic_sizes_and_nodes():
    """n = ne k unknowns (the DoF counts of Tables tab7c and tab8: 250^3 = (50 * 5)^3
    for Q^5, 500^3 = (25 * 20)^3 for Q^20); the node at b is the node at a."""
    for k, ne in ((5, 50), (20, 25), (1, 7), (3, 1)):
        o = O.axis_operators(k, ne, -16.0, 16.0, "periodic")
        assert o.x.size == o.M.size == o.K.shape[0] == ne * k
        assert o.x[0] == -16.0 and o.x[-1] < 16.0
        # the lumped mass integrates constants exactly: total = length
        assert abs(o.M.sum() - 32.0) <= 1e-12
        # constants are in the kernel of K; K is symmetric (to the rounding of D^T W D)
        assert np.max(np.abs(o.K.sum(axis=1))) <= 1e-12 * np.max(np.abs(o.K))
        assert np.max(np.abs(o.K - o.K.T)) <= 1e-14 * np.max(np.abs(o.K))


@pytest.mark.parametrize("ne", [5, 12, 16])
def test_k1_periodic_is_the_circulant_difference_laplacian(ne):
    """Q^1 with lumped mass is the periodic second-order difference Laplacian:
    H = (1/dx^2) circ(-1, 2, -1), eigenvalues (4/dx^2) sin^2(pi j / n), j = 0..n-1
    (the DFT diagonalises it: the FFT case of Sec. 4)."""
    a, b = 0.0, 3.0
    dx = (b - a) / ne
    o = O.axis_operators(1, ne, a, b, "periodic")
    h = o.K / o.M[:, None]
    ref = np.zeros((ne, ne))
    for i in range(ne):
        ref[i, i] += 2.0 / dx ** 2
        ref[i, (i + 1) % ne] -= 1.0 / dx ** 2
        ref[i, (i - 1) % ne] -= 1.0 / dx ** 2
    np.testing.assert_allclose(h, ref, rtol=0, atol=1e-12 / dx ** 2)
    lam, _, _ = O.axis_eigen(o)
    want = np.sort(4.0 / dx ** 2 * np.sin(np.pi * np.arange(ne) / ne) ** 2)
    np.testing.assert_allclose(lam, want, rtol=1e-13, atol=1e-12 * want[-1])


def _bloch_spectrum(k, ne, a, b):
    """Eigenvalues of the periodic problem from the element matrices alone: the
    translation by one element commutes with K and M, so the spectrum is the union
    over the Bloch phases theta_j = 2 pi j / ne of the k x k Hermitian problems on
    one cell (cell nodes 0..k-1; the element's local node k is cell node 0 of the
    next cell, carrying the phase e^{i theta})."""
    _, w, k_ref = O.element_matrices(k)
    h = (b - a) / (2.0 * ne)
    ke = k_ref / h
    m = h * w[:k].copy()
    m[0] += h * w[k]
    out = []
    for j in range(ne):
        th = 2.0 * np.pi * j / ne
        kt = np.zeros((k, k), dtype=complex)
        for li in range(k + 1):
            for lj in range(k + 1):
                kt[li % k, lj % k] += ke[li, lj] * np.exp(1j * th * (lj // k - li // k))
        kt = 0.5 * (kt + kt.conj().T)
        s = 1.0 / np.sqrt(m)
        out.extend(np.linalg.eigvalsh(s[:, None] * kt * s[None, :]))
    return np.sort(np.array(out))


@pytest.mark.parametrize("k,ne", [(2, 9), (3, 6), (5, 7), (8, 4), (4, 1), (6, 2)])
def test_spectrum_equals_bloch_assembly(k, ne):
    o = O.axis_operators(k, ne, -1.0, 2.0, "periodic")
    lam, _, _ = O.axis_eigen(o)
    ref = _bloch_spectrum(k, ne, -1.0, 2.0)
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-12 * ref[-1])


def _check_invariants(o, tol=1e-13):
    lam, s, f = O.axis_eigen(o)
    n = lam.size
    assert np.all(np.diff(lam) >= 0)
    g = s.T @ (o.M[:, None] * s)
    assert np.max(np.abs(g - np.eye(n))) <= tol, np.max(np.abs(g - np.eye(n)))
    res = o.K @ s - (o.M[:, None] * s) * lam[None, :]
    kinf = np.max(np.sum(np.abs(o.K), axis=1))
    rel = np.max(np.max(np.abs(res), axis=0) / (kinf * np.max(np.abs(s), axis=0)))
    assert rel <= tol, rel
    assert np.max(np.abs(f @ s - np.eye(n))) <= tol
    return lam


@pytest.mark.parametrize("k,ne", [(1, 9), (4, 6), (5, 50), (20, 10), (3, 1), (7, 2)])
def test_eigen_invariants_periodic(k, ne):
    """S^T M S = I and K S = M S Lambda (scale-free) to 1e-13, with the exactly
    double eigenvalues of the periodic spectrum."""
    _check_invariants(O.axis_operators(k, ne, -16.0, 16.0, "periodic"))


def test_lowest_eigenvalues_match_continuous_periodic_spectrum():
    """-u'' on a period of length L: 0 once, then (2 pi j / L)^2 twice for j >= 1;
    Q^4 with 250 elements on [-1, 1] resolves the low modes far below rounding."""
    o = O.axis_operators(4, 250, -1.0, 1.0, "periodic")
    lam = _check_invariants(o)
    want = np.array([0.0] + [(2 * np.pi * j / 2.0) ** 2 for j in (1, 1, 2, 2, 3, 3)])
    err = np.abs(lam[:7] - want)
    assert np.all(err <= 5e-14 * (1 + want)), err


CASES = [
    (2, (3, 2, 4), (0.0, 1.0, -1.0, 1.0, 0.0, 2.0), 0.5),
    (3, (2, 3, 2), (-1.0, 1.0, 0.0, 0.5, 0.0, 3.0), 2.0),
    (4, (1, 2, 1), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}")
def test_periodic_fd_equals_dense_lu(case):
    k, ne, box, alpha = case
    prob = O.Problem(k, ne, box, alpha, "periodic")
    f = np.random.default_rng(5).standard_normal(prob.shape)
    ref = O.dense_solve(prob, f)
    assert O.rel_max_err(O.fd_solve(prob, f), ref) <= 1e-12
    # the nodal residual of the dense solution vanishes
    r = O.residual(prob, ref, f)
    assert np.max(np.abs(r)) <= 1e-11 * np.max(np.abs(f))


def test_periodic_translation_by_one_element():
    """Shifting f by k nodes (one element) along a periodic axis shifts u by the
    same amount (a symmetry of the discrete problem); a shift by one node is not a
    symmetry for k > 1 and changes the result."""
    k, ne = 3, (4, 5, 3)
    prob = O.Problem(k, ne, (0.0, 2.0, -1.0, 1.0, 0.0, 1.5), 0.8, "periodic")
    f = np.random.default_rng(9).standard_normal(prob.shape)
    u = O.fd_solve(prob, f)
    for ax in range(3):
        us = O.fd_solve(prob, np.roll(f, k, axis=ax))
        assert O.rel_max_err(us, np.roll(u, k, axis=ax)) <= 1e-13, ax
    u1 = O.fd_solve(prob, np.roll(f, 1, axis=2))
    assert O.rel_max_err(u1, np.roll(u, 1, axis=2)) > 1e-3


def test_periodic_constant_mode():
    prob = O.Problem(5, (3, 4, 2), (0.0, 1.0, 0.0, 2.0, 0.0, 3.0), 2.5, "periodic")
    u = O.fd_solve(prob, np.full(prob.shape, 5.0))
    assert np.max(np.abs(u - 2.0)) <= 1e-13


def test_periodic_spectral_convergence():
    """-Lap u + u = f on [0, 2pi]^3 with u = sin(x + 0.3) cos(2y) sin(z - 1)
    (periodic), f = 7u: the nodal error falls by more than (h_0 / h_1)^k when
    the elements shrink (measured: 23.5x for Q^4, 4 -> 8 elements; 20.4x for Q^6,
    8 -> 12), and is below 5e-9 for Q^6 with 12 elements per axis."""
    def err(k, ne):
        prob = O.Problem(k, (ne,) * 3, (0.0, 2 * np.pi) * 3, 1.0, "periodic")
        x, y, z = np.meshgrid(*(o.x for o in prob.axes), indexing="ij")
        ue = np.sin(x + 0.3) * np.cos(2 * y) * np.sin(z - 1.0)
        return np.max(np.abs(O.fd_solve(prob, 7.0 * ue) - ue))
    e4, e8 = err(4, 4), err(4, 8)
    assert e8 < e4 / 2 ** 4, (e4, e8)
    e8, e12 = err(6, 8), err(6, 12)
    assert e12 < e8 / 1.5 ** 6 and e12 < 5e-9, (e8, e12)


def test_periodic_pcg_paper_problem():
    """The paper's Schroedinger problem with periodic conditions (its exact
    solution is periodic on [-16, 16]^3), Q^5 with 20 elements per axis (n = 100),
    beta = 1: PCG to 1e-12 takes the paper's ~10 iterations (Table tab7c) and
    the error against the exact solution is the discretisation error (~1.3e-11);
    the PCG result equals a dense-free reference: one more FD-preconditioned
    Richardson sweep does not move it."""
    prob = O.Problem(5, (20, 20, 20), SCHRODINGER_BOX, 1.0, "periodic")
    v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, 1.0)
    u, it, hist = O.pcg_schrodinger(prob, v, f, 1.5, tol=1e-12)
    assert 9 <= it <= 11 and hist[-1] <= 1e-12
    assert np.max(np.abs(u - ue)) <= 3e-11
    r = f - O.schrodinger_apply(prob, v, u)
    du = O.fd_solve(prob, r, alpha=1.5)
    assert np.max(np.abs(du)) <= 1e-11 * np.max(np.abs(u))


def test_periodic_pcg_equals_dense_solve():
    prob = O.Problem(2, (3, 2, 3), (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5), 0.7, "periodic")
    rng = np.random.default_rng(12)
    v = rng.uniform(0.0, 8.0, size=prob.shape)
    f = rng.standard_normal(prob.shape)
    nx, ny, nz = prob.shape
    hx, hy, hz = (prob.h_dense(a) for a in range(3))
    a = (np.kron(np.kron(hx, np.eye(ny)), np.eye(nz)) + np.kron(np.kron(np.eye(nx), hy), np.eye(nz))
         + np.kron(np.kron(np.eye(nx), np.eye(ny)), hz)) + np.diag(prob.alpha + v.reshape(-1))
    ref = np.linalg.solve(a, f.reshape(-1)).reshape(prob.shape)
    u, it, hist = O.pcg_schrodinger(prob, v, f, prob.alpha + 4.0, tol=1e-14, max_iter=200)
    assert O.rel_max_err(u, ref) <= 1e-12
    assert math.isfinite(hist[-1])
