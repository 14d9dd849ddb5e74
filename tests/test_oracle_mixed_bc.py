"""Pins of the oracle with a different boundary condition on each axis (the
operators are Kronecker sums of per-axis 1D operators, so each axis carries its
own condition; Sec. 2.4 remark), independent of the fast diagonalisation: dense
LU of the assembled system, exact linear solutions with boundary data, and
convergence on a smooth exact solution."""
import numpy as np
import pytest

import oracle as O

BOX = (0.0, 1.0, -1.0, 1.0, 0.0, 2.0)
COMBOS = [("dirichlet", "neumann", "periodic"), ("periodic", "dirichlet", "periodic"),
          ("neumann", "periodic", "dirichlet"), ("periodic", "periodic", "neumann")]


@pytest.mark.parametrize("bcs", COMBOS, ids=lambda b: "-".join(x[0] for x in b))
def test_mixed_fd_equals_dense_lu(bcs):
    prob = O.Problem(2, (3, 2, 3), BOX, 0.6, bcs)
    sizes = {"dirichlet": lambda ne: 2 * ne - 1, "neumann": lambda ne: 2 * ne + 1, "periodic": lambda ne: 2 * ne}
    assert prob.shape == tuple(sizes[b](n) for b, n in zip(bcs, (3, 2, 3)))
    f = np.random.default_rng(6).standard_normal(prob.shape)
    assert O.rel_max_err(O.fd_solve(prob, f), O.dense_solve(prob, f)) <= 1e-12


def _faces(prob, fn):
    """Dirichlet axes: u on the faces; Neumann axes: the outward normal derivative;
    periodic axes: none."""
    xs = [o.x for o in prob.axes]
    out = []
    for a in range(3):
        for side in (0, 1):
            if prob.bcs[a] == "periodic":
                out.append(None)
                continue
            coords = list(xs)
            coords[a] = np.array([prob.box[2 * a + side]])
            vals = fn(*np.meshgrid(*coords, indexing="ij"))
            v = vals[0] if prob.bcs[a] == "dirichlet" else (1.0 if side else -1.0) * vals[1 + a]
            out.append(np.squeeze(v, axis=a))
    return out


def test_mixed_linear_solution_exact():
    """u = 1 + x + 2y (constant along the periodic z axis) with Dirichlet data on
    the x faces and Neumann data on the y faces is reproduced exactly."""
    def lin(x, y, z):
        u = 1.0 + x + 2.0 * y + 0.0 * z
        return u, np.ones_like(u), 2.0 * np.ones_like(u), np.zeros_like(u)
    for k in (1, 3, 5):
        prob = O.Problem(k, (3, 2, 2), BOX, 0.7, ("dirichlet", "neumann", "periodic"))
        u = lin(*np.meshgrid(*(o.x for o in prob.axes), indexing="ij"))[0]
        uh = O.fd_solve(prob, 0.7 * u + O.lift_boundary(prob, _faces(prob, lin)))
        assert np.max(np.abs(uh - u)) <= 1e-12 * np.max(np.abs(u)), k


def test_mixed_smooth_solution_converges():
    """u = e^{x/2} sin(y + 0.3) cos(pi z): Dirichlet in x, Neumann in y, periodic in
    z on [0, 2]; -Lap u = (pi^2 + 0.75) u.  Error falls by more than 2^k per
    halving (Q^4) and is below 1e-8 at Q^6 with 6 elements per axis (3.5e-8 with 4)."""
    def smooth(x, y, z):
        e = np.exp(0.5 * x)
        u = e * np.sin(y + 0.3) * np.cos(np.pi * z)
        return (u, 0.5 * u, e * np.cos(y + 0.3) * np.cos(np.pi * z),
                -np.pi * e * np.sin(y + 0.3) * np.sin(np.pi * z))

    def err(k, ne):
        prob = O.Problem(k, (ne,) * 3, BOX, 1.0, ("dirichlet", "neumann", "periodic"))
        u = smooth(*np.meshgrid(*(o.x for o in prob.axes), indexing="ij"))[0]
        f = (np.pi ** 2 + 1.75) * u
        return np.max(np.abs(O.fd_solve(prob, f + O.lift_boundary(prob, _faces(prob, smooth))) - u))
    e2, e4 = err(4, 2), err(4, 4)
    assert e4 < e2 / 2 ** 4, (e2, e4)
    assert err(6, 6) < 1e-8


def test_mixed_lift_rejects_periodic_faces():
    prob = O.Problem(2, (2, 2, 2), BOX, 1.0, ("dirichlet", "periodic", "neumann"))
    with pytest.raises(ValueError):
        O.lift_boundary(prob, [None, None, np.zeros((3, 5)), None, None, None])
