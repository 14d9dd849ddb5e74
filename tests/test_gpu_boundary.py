"""GPU parity of non-homogeneous boundary data (sem_lift_boundary) against the
oracle's lift_boundary: the lifted right-hand side element by element, the
solves that follow it (FP64 and refined split BF16), the exact reproduction of a
linear solution and the error on a smooth exact solution.

Bars: lifted right-hand side within 1e-14 (||f|| + ||H|| ||g||) (a few FP64
roundings per node); solves as for homogeneous data (FP64 1e-12, refined 1e-10,
plus 10 x the oracle's rounding floor).
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import normal_noise

pytestmark = pytest.mark.gpu

BOX = (0.0, 1.0, -1.0, 1.0, 0.0, 2.0)
CASES = [
    (4, (9, 7, 8), "dirichlet", 1.0),     # 35 x 27 x 31
    (3, (30, 25, 44), "dirichlet", 0.0),  # 89 x 74 x 131: several tiles, Laplace
    (4, (1, 2, 1), "dirichlet", 2.0),     # 3 x 7 x 3: the two ends' bands overlap
    (5, (6, 4, 7), "neumann", 0.8),       # 31 x 21 x 36
    (2, (40, 3, 1), "neumann", 1.5),      # 81 x 7 x 3
    (9, (2, 3, 2), "dirichlet", 1.0),     # 17 x 26 x 17, k > 8
]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def P():
    import paper_2310_00226_amd as P
    return P


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _random_faces(shape, seed, skip=()):
    rng = np.random.default_rng(seed)
    out = []
    for a in range(3):
        fs = tuple(n for b, n in enumerate(shape) if b != a)
        for s in (0, 1):
            out.append(None if 2 * a + s in skip else rng.standard_normal(fs))
    return out


def _smooth(x, y, z):
    e = np.exp(0.5 * x)
    u = e * np.sin(y + 0.3) * np.cos(0.7 * z)
    return (u, 0.5 * u, e * np.cos(y + 0.3) * np.cos(0.7 * z), -0.7 * e * np.sin(y + 0.3) * np.sin(0.7 * z))


def _linear(x, y, z):
    u = 1.0 + x + 2.0 * y - 0.5 * z
    one = np.ones_like(u)
    return u, one, 2.0 * one, -0.5 * one


def _faces_from(prob, fn, bc):
    xs = [o.x for o in prob.axes]
    out = []
    for a in range(3):
        for side in (0, 1):
            coords = list(xs)
            coords[a] = np.array([prob.box[2 * a + side]])
            vals = fn(*np.meshgrid(*coords, indexing="ij"))
            v = vals[0] if bc == "dirichlet" else (1.0 if side else -1.0) * vals[1 + a]
            out.append(np.squeeze(v, axis=a))
    return out


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}-{c[2]}")
def test_lifted_rhs_and_solve(torch, P, case):
    k, ne, bc, alpha = case
    _log(f"[boundary] k={k} ne={ne} {bc}")
    prob = O.Problem(k, ne, BOX, alpha, bc)
    plan = P.Plan(k, ne, BOX, alpha, bc)
    f = normal_noise(prob.shape, seed=80 + k)
    faces = _random_faces(prob.shape, 90 + k, skip=(3,))  # one face homogeneous
    ref = f + O.lift_boundary(prob, faces)
    fd = _dev(torch, f)
    plan.lift_boundary([None if g is None else _dev(torch, g) for g in faces], fd)
    got = fd.cpu().numpy()
    hnorm = sum(np.max(np.sum(np.abs(prob.h_dense(a)), axis=1)) for a in range(3))
    gmax = max(np.max(np.abs(g)) for g in faces if g is not None)
    scale = np.max(np.abs(f)) + (hnorm if bc == "dirichlet" else 1.0 / min(o.M.min() for o in prob.axes)) * gmax
    assert np.max(np.abs(got - ref)) <= 1e-14 * scale
    uref = O.fd_solve(prob, ref)
    u = plan.solve(fd).cpu().numpy()
    floor = np.max(np.abs(uref - O.fd_solve(prob, ref, order=(0, 1, 2))))
    assert np.max(np.abs(u - uref)) <= 1e-12 * np.max(np.abs(uref)) + 10 * floor


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_linear_solution_exact(torch, P, bc):
    k, ne, alpha = 5, (4, 3, 5), 0.9
    prob = O.Problem(k, ne, BOX, alpha, bc)
    plan = P.Plan(k, ne, BOX, alpha, bc)
    u = _linear(*np.meshgrid(*(o.x for o in prob.axes), indexing="ij"))[0]
    fd = _dev(torch, alpha * u)
    plan.lift_boundary([_dev(torch, g) for g in _faces_from(prob, _linear, bc)], fd)
    uh = plan.solve(fd).cpu().numpy()
    assert np.max(np.abs(uh - u)) <= 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_smooth_solution_refined(torch, P, bc):
    """u = e^{x/2} sin(y + 0.3) cos(0.7 z) with its boundary data, Q^6, 8^3 elements:
    split-BF16 refined solve within 1e-10 of the oracle, and within the
    discretisation error of the exact solution (oracle: 2.2e-14; bound 1e-11)."""
    k, ne, alpha = 6, (8, 8, 8), 1.0
    prob = O.Problem(k, ne, BOX, alpha, bc)
    plan = P.Plan(k, ne, BOX, alpha, bc)
    u = _smooth(*np.meshgrid(*(o.x for o in prob.axes), indexing="ij"))[0]
    f = 2.24 * u
    faces = _faces_from(prob, _smooth, bc)
    ref = O.fd_solve(prob, f + O.lift_boundary(prob, faces))
    fd = _dev(torch, f)
    plan.lift_boundary([_dev(torch, g) for g in faces], fd)
    uh, it, rel, st = plan.solve_refined(fd, prec="bf16x3", tol=1e-12)
    uh = uh.cpu().numpy()
    err_o, err_x = np.max(np.abs(uh - ref)), np.max(np.abs(uh - u))
    _log(f"[boundary] smooth {bc}: {it} iterations, vs oracle {err_o:.2e}, vs exact {err_x:.2e}")
    assert st == 0 and err_o <= 1e-10 * np.max(np.abs(ref)) and err_x < 1e-11


def test_lift_rejects_invalid(torch, P):
    per = P.Plan(3, (2, 2, 2), BOX, 1.0, "periodic")
    f = torch.zeros(per.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):
        per.lift_boundary([torch.zeros(per.shape[1:], dtype=torch.float64, device="cuda")] + [None] * 5, f)
    per.lift_boundary([None] * 6, f)  # homogeneous: nothing to do
    plan = P.Plan(3, (2, 2, 2), BOX, 1.0, "dirichlet")
    f = torch.ones(plan.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):
        plan.lift_boundary([f.view(-1)[: plan.shape[1] * plan.shape[2]]] + [None] * 5, f)  # aliases f
    g = f.clone()
    plan.lift_boundary([None] * 6, g)
    assert torch.equal(g, f)
