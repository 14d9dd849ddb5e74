"""GPU parity of the variable-coefficient solver (alpha u - Lap u + V u = f by PCG
with the FD preconditioner, sem_pcg_solve) against the oracle's PCG and against
the paper's exact solution.

Bar: ||u - u_oracle||_inf <= 1e-10 ||u_oracle||_inf for every preconditioner
precision (the operator, the update and the inner products are FP64, so every
precision converges to the same discrete solution); errors against the exact
solution within the oracle's own (pinned) discretisation error.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from workloads import SCHRODINGER_BOX, schrodinger_data

pytestmark = pytest.mark.gpu

PRECS = ["f64", "f32", "bf16x3", "bf16"]


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


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("case", ["neumann-q5", "dirichlet-q3", "dirichlet-q4-long-z"])
def test_pcg_matches_oracle(torch, P, prec, case):
    if case == "neumann-q5":  # the paper's problem: its V (beta = 10) and exact solution
        k, ne, bc, box, alpha, beta = 5, (6, 7, 5), "neumann", SCHRODINGER_BOX, 1.0, 10.0
        prob = O.Problem(k, ne, box, alpha, bc)
        v, _, f = schrodinger_data(*(o.x for o in prob.axes), alpha, beta)
    else:  # a general positive potential and right-hand side, several tiles and ragged tails
        if case == "dirichlet-q3":
            k, ne, bc, box, alpha, beta = 3, (30, 22, 27), "dirichlet", (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5), 0.5, 40.0
        else:  # n = (15, 19, 359): 180 representatives per z row (the 256-thread unfold with its inner products)
            k, ne, bc, box, alpha, beta = 4, (4, 5, 90), "dirichlet", (0.0, 1.0, 0.0, 1.2, 0.0, 20.0), 1.0, 5.0
        prob = O.Problem(k, ne, box, alpha, bc)
        rng = np.random.default_rng(41)
        v = rng.uniform(0.0, beta, size=prob.shape)
        f = rng.standard_normal(prob.shape)
    shift = alpha + beta / 2
    ref, it_ref, _ = O.pcg_schrodinger(prob, v, f, shift, tol=1e-14, max_iter=500)
    plan = P.Plan(k, ne, box, alpha, bc)
    u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=shift, prec=prec, tol=1e-13,
                                    max_iter=500)
    err = O.rel_max_err(u.cpu().numpy(), ref)
    _log(f"[pcg] {case} {prec}: {it} iterations (oracle {it_ref} to 1e-14), rel residual {rel:.1e}, err {err:.2e}")
    assert st == 0 and rel <= 1e-13
    assert err <= 1e-10, err
    if prec == "f64":
        assert it <= it_ref  # the oracle iterates to 1e-14, this solve to 1e-13


def test_pcg_exact_solution_q5(torch, P):
    """The paper's exact solution, Q^5, 24^3 elements (n = 121), beta = 1: the
    error equals the oracle's discretisation error (3.7e-12) and PCG takes ~10
    iterations (Table tab7c)."""
    prob = O.Problem(5, (24, 24, 24), SCHRODINGER_BOX, 1.0, "neumann")
    v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, 1.0)
    plan = P.Plan(5, (24, 24, 24), SCHRODINGER_BOX, 1.0, "neumann")
    for prec in ("f64", "bf16x3"):
        u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=1.5, prec=prec, tol=1e-12)
        err = float(np.max(np.abs(u.cpu().numpy() - ue)))
        _log(f"[pcg] exact solution Q^5 n=121 {prec}: {it} iterations, max error {err:.2e}")
        assert st == 0 and 8 <= it <= 11
        assert err <= 1e-11, err


def test_pcg_q20(torch, P):
    """Sec. robustness: Q^20, 5^3 elements, beta = 1: max error vs the exact
    solution ~5e-14 as in the oracle (Table tab8 reports ~1e-13)."""
    prob = O.Problem(20, (5, 5, 5), SCHRODINGER_BOX, 1.0, "neumann")
    v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, 1.0)
    plan = P.Plan(20, (5, 5, 5), SCHRODINGER_BOX, 1.0, "neumann")
    u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=1.5, prec="f64", tol=1e-14)
    err = float(np.max(np.abs(u.cpu().numpy() - ue)))
    _log(f"[pcg] Q^20: {it} iterations, max error {err:.2e}")
    assert st == 0 and err <= 2e-13, err


def test_pcg_rejects_invalid(torch, P):
    plan = P.Plan(3, (3, 3, 3), SCHRODINGER_BOX, 1.0, "neumann")
    v = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    f = torch.ones_like(v)
    for kw in ({"shift": float("nan")}, {"shift": float("inf")}, {"tol": -1.0}, {"max_iter": 0}):
        args = {"shift": 1.0, **kw}
        with pytest.raises(P.SemError):
            plan.pcg_solve(v, f, **args)
    with pytest.raises(P.SemError):
        plan.pcg_solve(v, f, u=f, shift=1.0)  # u aliases f
    # default shift alpha + max(V)/2 not positive (V = -3, alpha = 1), or V not finite
    with pytest.raises(P.SemError, match="SEM_EINVAL"):
        plan.pcg_solve(torch.full_like(v, -3.0), f)
    vbad = v.clone()
    vbad[1, 2, 0] = float("nan")
    with pytest.raises(P.SemError, match="SEM_ENONFINITE"):
        plan.pcg_solve(vbad, f)
    # zero right-hand side: u = 0 in no iterations
    u, it, rel, st = plan.pcg_solve(v, torch.zeros_like(v), shift=1.0)
    assert st == 0 and it == 0 and float(u.abs().max()) == 0.0


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_pcg_default_shift_is_alpha_plus_half_max_v(torch, P, prec):
    """Without a shift the library takes the paper's alpha + beta/2 with beta = max(V),
    reduced on the device: the same iterates as the explicit shift (bit-equal)."""
    k, ne, box, alpha, beta = 4, (9, 8, 10), SCHRODINGER_BOX, 1.0, 10.0
    plan = P.Plan(k, ne, box, alpha, "neumann")
    v, _, f = schrodinger_data(*(plan.nodes(a) for a in range(3)), alpha, beta)
    vmax = float(np.max(v))
    vd, fd = _dev(torch, v), _dev(torch, f)
    u0, it0, rel0, st0 = plan.pcg_solve(vd, fd, prec=prec, tol=1e-12)
    assert plan.last_pcg_shift == alpha + 0.5 * vmax
    u1, it1, rel1, st1 = plan.pcg_solve(vd, fd, shift=alpha + 0.5 * vmax, prec=prec, tol=1e-12)
    assert plan.last_pcg_shift == alpha + 0.5 * vmax
    assert st0 == st1 == 0 and it0 == it1
    assert torch.equal(u0, u1)
    for sh in (0.0, -2.0):  # any shift <= 0 selects the default
        u2, it2, _, _ = plan.pcg_solve(vd, fd, shift=sh, prec=prec, tol=1e-12)
        assert it2 == it0 and torch.equal(u2, u0)


class _Lines:
    def __init__(self, t):
        self.t = t

    def __getitem__(self, key):
        return self.t[key].cpu().numpy()


def test_pcg_full_size_sampled(torch, P):
    """The benchmarked configuration, Table tab5's largest: Q^5, 200^3 elements on
    [-16, 16]^3, periodic (n = 1000, 1e9 unknowns), beta = 1, split-BF16
    preconditioner.  The nodal residual
    f - (alpha + V) u - H_3 u at 64 seeded nodes, recomputed by the oracle, is within
    a 1e-12 normwise backward error, and the error vs the exact solution at those
    nodes is below the discretisation error of the finer oracle meshes."""
    ne = 200
    plan = P.Plan(5, (ne, ne, ne), SCHRODINGER_BOX, 1.0, "periodic")
    assert plan.shape == (1000, 1000, 1000)
    xs = [plan.nodes(a) for a in range(3)]
    v, ue, f = schrodinger_data(*xs, 1.0, 1.0)
    vd, fd = _dev(torch, v), _dev(torch, f)
    del f
    u, it, rel, st = plan.pcg_solve(vd, fd, shift=1.5, prec="bf16x3", tol=1e-12)
    _log(f"[pcg] full size n=1000 periodic: {it} iterations, rel residual {rel:.1e}")
    assert st == 0 and 8 <= it <= 12
    prob = O.Problem(5, (ne, ne, ne), SCHRODINGER_BOX, 1.0, "periodic", eigen=False)
    rng = np.random.default_rng(13)
    idx = np.stack([rng.integers(0, n, size=64) for n in plan.shape], axis=1)
    fl = _Lines(fd)
    r = O.residual_at(prob, _Lines(u), fl, idx)
    uv = np.array([float(u[i, j, l]) for i, j, l in idx])
    r -= v[idx[:, 0], idx[:, 1], idx[:, 2]] * uv
    hnorm = 1.0 + 1.0 + sum(np.max(np.sum(np.abs(prob.h_dense(a)), axis=1)) for a in range(3))
    scale = float(fd.abs().max()) + hnorm * float(u.abs().max())
    back = float(np.max(np.abs(r))) / scale
    err = float(np.max(np.abs(uv - ue[idx[:, 0], idx[:, 1], idx[:, 2]])))
    _log(f"[pcg]   sampled backward error {back:.2e}, sampled error vs exact {err:.2e}")
    assert back <= 1e-12
    assert err <= 1e-11


def test_pcg_q20_n501(torch, P):
    """Sec. robustness at the size of Table tab8's first row: Q^20, 25^3 elements
    (n = 501), beta = 1, 10, 100; the paper reports max errors 1.89e-13,
    1.62e-13, 1.29e-13 there (periodic); here (Neumann) the error must stay
    within 5e-13 (the largest entry of that table is 6.3e-13)."""
    plan = P.Plan(20, (25, 25, 25), SCHRODINGER_BOX, 1.0, "neumann")
    xs = [plan.nodes(a) for a in range(3)]
    for beta in (1.0, 10.0, 100.0):
        v, ue, f = schrodinger_data(*xs, 1.0, beta)
        u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=1.0 + beta / 2, prec="f64",
                                        tol=1e-14, max_iter=300)
        err = float((u - _dev(torch, ue)).abs().max())
        _log(f"[pcg] Q^20 n=501 beta={beta:g}: {it} iterations, max error {err:.2e}")
        assert st == 0 and err <= 5e-13, (beta, err)
