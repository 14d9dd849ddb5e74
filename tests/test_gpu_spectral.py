"""GPU parity of the spectral multipliers on the FD transforms (sem_apply_spectral:
exp(-t (H_3 + a)) and (H_3 + a)^(-s)) against the oracle.

Bar: ||u - u_oracle||_inf <= 1e-12 ||u_oracle||_inf + 10 x the oracle's own
rounding floor (two contraction orders), as for the FP64 solve.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

CASES = [
    (4, (12, 9, 10), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), "dirichlet"),
    (3, (7, 8, 5), (0.0, 2.0, -1.0, 0.5, 0.0, 1.0), "neumann"),
    (6, (40, 3, 33), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), "dirichlet"),
]
MULTS = [("exp", 0.0), ("exp", 1e-3), ("exp", 0.05), ("power", 0.5), ("power", 1.0), ("power", 1.5),
         ("power", -0.5)]


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


def _floor(prob, kind, a, param, f):
    """Rounding floor of the oracle: the same multiplier with the axes contracted
    in another order."""
    lam = prob.lam3() + a
    t = f
    for ax in (0, 1, 2):
        t = O.mode_product(t, prob.eig[ax][2], ax)
    t = t * (np.exp(-param * lam) if kind == "exp" else lam ** (-param))
    for ax in (0, 1, 2):
        t = O.mode_product(t, prob.eig[ax][1], ax)
    return np.max(np.abs(t - O.spectral_apply(prob, kind, a, param, f)))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[3]}-{c[1]}")
def test_multipliers_match_oracle(torch, P, case):
    k, ne, box, bc = case
    a = 0.7
    prob = O.Problem(k, ne, box, 1.0, bc)
    plan = P.Plan(k, ne, box, 1.0, bc)
    f = np.random.default_rng(17).standard_normal(prob.shape)
    fd = torch.from_numpy(f).to("cuda")
    for kind, param in MULTS:
        ref = O.spectral_apply(prob, kind, a, param, f)
        u = plan.apply_spectral(kind, a, param, fd).cpu().numpy()
        err = np.max(np.abs(u - ref))
        bound = 1e-12 * np.max(np.abs(ref)) + 10 * _floor(prob, kind, a, param, f)
        _log(f"[spectral] {case[3]} k={k} {kind}({param}): rel err {err / np.max(np.abs(ref)):.2e}")
        assert err <= bound, (kind, param, err, bound)


def test_power_one_is_the_solve_and_in_place(torch, P):
    plan = P.Plan(4, (9, 11, 8), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), 2.5, "dirichlet")
    f = torch.randn(plan.shape, dtype=torch.float64, device="cuda")
    sol = plan.solve(f)
    u = plan.apply_spectral("power", 2.5, 1.0, f)
    assert float((u - sol).abs().max() / sol.abs().max()) <= 1e-13
    g = f.clone()
    plan.apply_spectral("exp", 2.5, 0.01, g, g)  # u may alias f
    assert torch.equal(g, plan.apply_spectral("exp", 2.5, 0.01, f))


def test_spectral_rejects_invalid(torch, P):
    plan = P.Plan(3, (3, 3, 3), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0, "neumann")
    f = torch.ones(plan.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError):
        plan.apply_spectral("exp", 0.0, -1.0, f)  # negative time
    with pytest.raises(P.SemError):
        plan.apply_spectral("power", 0.0, 0.5, f)  # Neumann: L has a zero eigenvalue
    with pytest.raises(P.SemError):
        plan.apply_spectral("exp", float("nan"), 0.1, f)


def test_power_minus_one_is_the_operator(torch, P):
    """s = -1 applies H_3 + a itself: equal to minus the banded residual of u = f
    with a zero right-hand side (a different kernel, no transforms), on a
    Dirichlet and a Neumann grid."""
    for bc in ("dirichlet", "neumann"):
        plan = P.Plan(4, (6, 5, 7), (0.0, 1.0, 0.0, 1.5, 0.0, 2.0), 1.0, bc)
        f = torch.randn(plan.shape, dtype=torch.float64, device="cuda")
        op = -plan.residual(f, torch.zeros_like(f))
        u = plan.apply_spectral("power", 1.0, -1.0, f)
        assert float((u - op).abs().max() / op.abs().max()) <= 1e-12, bc
