"""Pins of the oracle's non-homogeneous boundary data (Sec. 2.1 remark: Dirichlet
and Neumann data move into the right-hand side, the matrix to invert stays the
same), independent of the lift formula itself: a dense solve of the full-grid
system with the Dirichlet rows replaced by the data, exact reproduction of linear
solutions (which lie in Q^k and which GLL quadrature integrates exactly), the
total flux through the faces, and convergence on a smooth exact solution."""
import numpy as np
import pytest

import oracle as O

BOX = (0.0, 1.0, -1.0, 1.0, 0.0, 2.0)


def _faces_from(prob, fn, kind):
    """Face data from a function fn(x, y, z) -> (u, ux, uy, uz): the values u
    (Dirichlet) or the outward normal derivative (Neumann) at the face nodes."""
    xs = [o.x for o in prob.axes]
    ends = [(prob.box[2 * a], prob.box[2 * a + 1]) for a in range(3)]
    faces = []
    for a in range(3):
        for side in (0, 1):
            coords = list(xs)
            coords[a] = np.array([ends[a][side]])
            g = np.meshgrid(*coords, indexing="ij")
            vals = fn(*g)
            if kind == "dirichlet":
                v = vals[0]
            else:
                v = (1.0 if side else -1.0) * vals[1 + a]
            faces.append(np.squeeze(v, axis=a))
    return faces


def _linear(x, y, z):
    u = 1.0 + x + 2.0 * y - 0.5 * z
    one = np.ones_like(u)
    return u, one, 2.0 * one, -0.5 * one


def _smooth(x, y, z):
    e = np.exp(0.5 * x)
    u = e * np.sin(y + 0.3) * np.cos(0.7 * z)
    return (u, 0.5 * u, e * np.cos(y + 0.3) * np.cos(0.7 * z), -0.7 * e * np.sin(y + 0.3) * np.sin(0.7 * z))


def _grid(prob):
    return np.meshgrid(*(o.x for o in prob.axes), indexing="ij")


@pytest.mark.parametrize("bc,alpha", [("dirichlet", 0.0), ("dirichlet", 1.3), ("neumann", 0.8)])
@pytest.mark.parametrize("k,ne", [(1, (3, 2, 4)), (2, (2, 3, 2)), (5, (2, 1, 3))])
def test_linear_solutions_are_reproduced(bc, alpha, k, ne):
    """-Lap u = 0 for a linear u, which lies in Q^k; GLL quadrature integrates
    every term of the weak form exactly (the alpha terms use the same quadrature on
    both sides), so the discrete solution is u itself."""
    prob = O.Problem(k, ne, BOX, alpha, bc)
    u = _linear(*_grid(prob))[0]
    f = alpha * u
    c = O.lift_boundary(prob, _faces_from(prob, _linear, bc))
    uh = O.fd_solve(prob, f + c)
    assert np.max(np.abs(uh - u)) <= 1e-12 * np.max(np.abs(u))


def test_dirichlet_lift_equals_dense_constrained_solve():
    """The full-grid system (Neumann-size assembly) with every boundary row
    replaced by u = g, solved densely, equals the interior solve of f + lift."""
    k, ne, alpha = 2, (2, 3, 2), 0.7
    prob = O.Problem(k, ne, BOX, alpha, "dirichlet")
    full = O.Problem(k, ne, BOX, alpha, "neumann", eigen=False)
    rng = np.random.default_rng(4)
    g_full = rng.standard_normal(full.shape)
    f = rng.standard_normal(prob.shape)
    a, m3 = O.dense_system(full)
    rhs = np.zeros(full.shape)
    rhs[1:-1, 1:-1, 1:-1] = f
    rhs = m3 * rhs.reshape(-1)
    bnd = np.ones(full.shape, dtype=bool)
    bnd[1:-1, 1:-1, 1:-1] = False
    bi = np.flatnonzero(bnd.reshape(-1))
    a[bi, :] = 0.0
    a[bi, bi] = 1.0
    rhs[bi] = g_full.reshape(-1)[bi]
    ref = np.linalg.solve(a, rhs).reshape(full.shape)[1:-1, 1:-1, 1:-1]
    faces = [g_full[0, 1:-1, 1:-1], g_full[-1, 1:-1, 1:-1], g_full[1:-1, 0, 1:-1], g_full[1:-1, -1, 1:-1],
             g_full[1:-1, 1:-1, 0], g_full[1:-1, 1:-1, -1]]
    u = O.fd_solve(prob, f + O.lift_boundary(prob, faces))
    assert O.rel_max_err(u, ref) <= 1e-12


def test_neumann_lift_carries_the_face_flux():
    """Tested against v = 1: the lifted right-hand side adds, in the M_3-weighted
    sum, the integral of the data over the boundary; for data constant on each
    face that is data x face area."""
    prob = O.Problem(4, (3, 2, 5), BOX, 1.0, "neumann")
    vals = [0.3, -1.1, 2.0, 0.7, -0.4, 1.5]
    faces = [np.full(tuple(n for b, n in enumerate(prob.shape) if b != a), vals[2 * a + s])
             for a in range(3) for s in (0, 1)]
    c = O.lift_boundary(prob, faces)
    lens = [BOX[1] - BOX[0], BOX[3] - BOX[2], BOX[5] - BOX[4]]
    area = [lens[1] * lens[2], lens[0] * lens[2], lens[0] * lens[1]]
    want = sum(vals[2 * a + s] * area[a] for a in range(3) for s in (0, 1))
    assert abs(np.sum(prob.mass3() * c) - want) <= 1e-13 * sum(abs(v) * max(area) for v in vals)


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_smooth_solution_converges(bc):
    """u = e^{x/2} sin(y + 0.3) cos(0.7 z), -Lap u = 1.24 u, alpha = 1: the nodal
    error falls by more than 2^k when the elements halve (Q^4) and is below 1e-8
    for Q^6 with 4 elements per axis."""
    def err(k, ne):
        prob = O.Problem(k, (ne,) * 3, BOX, 1.0, bc)
        u = _smooth(*_grid(prob))[0]
        c = O.lift_boundary(prob, _faces_from(prob, _smooth, bc))
        return np.max(np.abs(O.fd_solve(prob, 2.24 * u + c) - u))
    e2, e4 = err(4, 2), err(4, 4)
    assert e4 < e2 / 2 ** 4, (e2, e4)
    assert err(6, 4) < 1e-8


def test_homogeneous_and_periodic():
    prob = O.Problem(3, (2, 2, 2), BOX, 1.0, "dirichlet")
    assert not np.any(O.lift_boundary(prob, [None] * 6))
    per = O.Problem(3, (2, 2, 2), BOX, 1.0, "periodic")
    assert not np.any(O.lift_boundary(per, [None] * 6))
    with pytest.raises(ValueError):
        O.lift_boundary(per, [np.zeros((6, 6))] + [None] * 5)
