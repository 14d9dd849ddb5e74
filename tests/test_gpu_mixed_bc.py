"""GPU parity of plans with one boundary condition per axis
(sem_plan_create_mixed) against the oracle: FP64 solves and residuals (the
residual kernels wrap only the periodic axes), refined solves, boundary data on
the Dirichlet and Neumann axes, batches and PCG.

Bars as for the uniform conditions: FP64 solve 1e-12 (+ 10 x the oracle's
rounding floor), residual 1e-14 ||H||, refined / batched / PCG 1e-10.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import batch_rhs, normal_noise

pytestmark = pytest.mark.gpu

BOX = (0.0, 1.0, -1.0, 1.0, 0.0, 2.0)
CASES = [
    (4, (12, 9, 10), ("dirichlet", "neumann", "periodic"), 1.0),    # 47 x 37 x 40
    (3, (50, 45, 43), ("periodic", "dirichlet", "periodic"), 0.0),  # 150 x 134 x 129: a channel
    (5, (6, 30, 7), ("neumann", "periodic", "dirichlet"), 0.5),     # 31 x 150 x 34
    (2, (1, 3, 40), ("periodic", "periodic", "neumann"), 2.0),      # 2 x 6 x 81: aliasing offsets
    (9, (3, 2, 4), ("dirichlet", "periodic", "neumann"), 1.0),      # 26 x 18 x 37: generic residual
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


def _bound(prob, f, ref, tol):
    floor = np.max(np.abs(ref - O.fd_solve(prob, f, order=(0, 1, 2))))
    return tol * np.max(np.abs(ref)) + 10 * floor


def _ids(c):
    return f"k{c[0]}-{'-'.join(b[0] for b in c[2])}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
def test_mixed_solve_and_residual(torch, P, case):
    k, ne, bcs, alpha = case
    _log(f"[mixed] k={k} ne={ne} {bcs}")
    prob = O.Problem(k, ne, BOX, alpha, bcs)
    plan = P.Plan(k, ne, BOX, alpha, bcs)
    assert plan.shape == prob.shape
    f = normal_noise(prob.shape, seed=110 + k)
    ref = O.fd_solve(prob, f)
    u = plan.solve(_dev(torch, f)).cpu().numpy()
    assert np.max(np.abs(u - ref)) <= _bound(prob, f, ref, 1e-12)
    uu = normal_noise(prob.shape, seed=120 + k)
    r = plan.residual(_dev(torch, uu), _dev(torch, f)).cpu().numpy()
    hnorm = sum(np.max(np.sum(np.abs(prob.h_dense(a)), axis=1)) for a in range(3)) + alpha
    assert np.max(np.abs(r - O.residual(prob, uu, f))) <= 1e-14 * hnorm


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("case", CASES[:3], ids=_ids)
def test_mixed_refined(torch, P, case, prec):
    k, ne, bcs, alpha = case
    prob = O.Problem(k, ne, BOX, alpha, bcs)
    plan = P.Plan(k, ne, BOX, alpha, bcs)
    f = normal_noise(prob.shape, seed=130 + k)
    ref = O.fd_solve(prob, f)
    u, it, rel, st = plan.solve_refined(_dev(torch, f), prec=prec, tol=1e-12)
    assert st == 0 and np.max(np.abs(u.cpu().numpy() - ref)) <= _bound(prob, f, ref, 1e-10)


def test_mixed_boundary_data(torch, P):
    """u = e^{x/2} sin(y + 0.3) cos(pi z): Dirichlet data on the x faces, Neumann
    data on the y faces, periodic z; lifted right-hand side and solve vs the
    oracle, and the error against u."""
    k, ne, bcs = 6, (6, 6, 6), ("dirichlet", "neumann", "periodic")
    prob = O.Problem(k, ne, BOX, 1.0, bcs)
    plan = P.Plan(k, ne, BOX, 1.0, bcs)

    def fn(x, y, z):
        e = np.exp(0.5 * x)
        u = e * np.sin(y + 0.3) * np.cos(np.pi * z)
        return (u, 0.5 * u, e * np.cos(y + 0.3) * np.cos(np.pi * z),
                -np.pi * e * np.sin(y + 0.3) * np.sin(np.pi * z))
    xs = [o.x for o in prob.axes]
    faces = []
    for a in range(3):
        for side in (0, 1):
            if bcs[a] == "periodic":
                faces.append(None)
                continue
            coords = list(xs)
            coords[a] = np.array([BOX[2 * a + side]])
            vals = fn(*np.meshgrid(*coords, indexing="ij"))
            v = vals[0] if bcs[a] == "dirichlet" else (1.0 if side else -1.0) * vals[1 + a]
            faces.append(np.squeeze(v, axis=a))
    u = fn(*np.meshgrid(*xs, indexing="ij"))[0]
    f = (np.pi ** 2 + 1.75) * u
    rhs = f + O.lift_boundary(prob, faces)
    fd = _dev(torch, f)
    plan.lift_boundary([None if g is None else _dev(torch, g) for g in faces], fd)
    assert np.max(np.abs(fd.cpu().numpy() - rhs)) <= 1e-13 * np.max(np.abs(rhs))
    uh = plan.solve(fd).cpu().numpy()
    ref = O.fd_solve(prob, rhs)
    err = np.max(np.abs(uh - u))
    _log(f"[mixed] boundary data: vs oracle {np.max(np.abs(uh - ref)):.2e}, vs exact {err:.2e}")
    assert np.max(np.abs(uh - ref)) <= _bound(prob, rhs, ref, 1e-12) and err < 1e-8
    with pytest.raises(P.SemError):  # the periodic axis has no faces
        plan.lift_boundary([None] * 4 + [_dev(torch, np.zeros(plan.shape[:2]))] + [None], fd)


def test_mixed_batch(torch, P):
    specs = [
        {"k": 4, "ne": (25, 26, 24), "alpha": 1.0, "bc": ("periodic", "dirichlet", "periodic")},  # 100 x 103 x 96
        {"k": 3, "ne": (5, 7, 2), "alpha": 0.5, "bc": ("neumann", "periodic", "dirichlet")},
        {"k": 8, "ne": (2, 1, 3), "alpha": 3.0, "bc": "dirichlet"},
    ]
    plans = [P.Plan(s["k"], s["ne"], BOX, s["alpha"], s["bc"]) for s in specs]
    batch = P.Batch(plans)
    fs = [batch_rhs(p.shape, 131, i) for i, p in enumerate(plans)]
    fd = [_dev(torch, f) for f in fs]
    probs = [O.Problem(s["k"], s["ne"], BOX, s["alpha"], s["bc"]) for s in specs]
    refs = [O.fd_solve(pr, f) for pr, f in zip(probs, fs)]
    for prec in ("f32", "bf16x3"):
        ud = [torch.empty_like(f) for f in fd]
        its, st = batch.solve(fd, ud, prec=prec, tol=1e-12)
        assert st == 0
        for i in range(len(specs)):
            err = np.max(np.abs(ud[i].cpu().numpy() - refs[i]))
            assert err <= _bound(probs[i], fs[i], refs[i], 1e-10), (prec, i, err)


def test_mixed_pcg(torch, P):
    """PCG with a random positive potential on a plan periodic in x and y and
    Neumann in z, against the oracle's PCG."""
    k, ne, bcs, alpha, beta = 4, (9, 8, 10), ("periodic", "periodic", "neumann"), 0.5, 20.0
    prob = O.Problem(k, ne, BOX, alpha, bcs)
    plan = P.Plan(k, ne, BOX, alpha, bcs)
    rng = np.random.default_rng(77)
    v = rng.uniform(0.0, beta, size=prob.shape)
    f = rng.standard_normal(prob.shape)
    ref, it_ref, _ = O.pcg_schrodinger(prob, v, f, alpha + beta / 2, tol=1e-13, max_iter=300)
    for prec in ("f64", "bf16x3"):
        u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=alpha + beta / 2, prec=prec,
                                        tol=1e-13, max_iter=300)
        err = O.rel_max_err(u.cpu().numpy(), ref)
        _log(f"[mixed] pcg {prec}: {it} iterations (oracle {it_ref}), err {err:.2e}")
        assert st == 0 and err <= 1e-10
