"""sem_solve_noalloc (the FP64 solve with the library's fixed scratch array)
against sem_solve: same kernels, so the results must be equal bit for bit (and
so within the FP64 parity bar), on two calls in a row, the second with a smaller
problem; in place as well; sizes beyond the fixed array are rejected; and no
device allocation happens during the calls."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MAX_UNKNOWNS = 8 * 1024 * 1024  # SEM_NOALLOC_MAX_UNKNOWNS
TOL = 1e-12  # relative max error, the FP64 parity bar


def _close(u, ref):
    return float((u - ref).abs().max()) <= TOL * float(ref.abs().max())


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_2310_00226_amd as P
    return P


@pytest.fixture(scope="module")
def torch():
    import torch
    return torch


def _case(P, torch, k, ne, bc, alpha, seed):
    plan = P.Plan(k, ne, (-1.0, 1.0, -0.5, 1.5, 0.0, 2.0), alpha, bc)
    rng = np.random.default_rng(seed)
    f = torch.from_numpy(rng.standard_normal(plan.shape)).to("cuda")
    return plan, f


def test_noalloc_equals_solve_two_calls(P, torch):
    # first call large (many tiles, ragged tails), second smaller: the scratch
    # array holds the first call's intermediate when the second starts
    cases = [(4, (40, 33, 37), "dirichlet", 1.0, 7), (3, (5, 9, 4), "neumann", 0.5, 8)]
    for k, ne, bc, alpha, seed in cases:
        plan, f = _case(P, torch, k, ne, bc, alpha, seed)
        _log(f"[noalloc] k={k} ne={ne} {bc}: {plan.numel} unknowns")
        ref = plan.solve(f)
        torch.cuda.synchronize()
        before = torch.cuda.memory_stats().get("num_alloc_retries", 0), torch.cuda.memory_allocated()
        u = torch.empty_like(f)
        torch.cuda.synchronize()
        alloc0 = torch.cuda.memory_allocated()
        plan.solve_noalloc(f, u)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == alloc0  # nothing through torch
        assert _close(u, ref) and torch.equal(u, ref), float((u - ref).abs().max())
        # in place (u aliases f), as sem_solve allows
        g = f.clone()
        plan.solve_noalloc(g, g)
        torch.cuda.synchronize()
        assert torch.equal(g, ref)
        del before


def test_noalloc_rejects_too_large(P, torch):
    plan = P.Plan(1, (205, 205, 205), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0, "dirichlet")  # 204^3 > 8 Mi
    assert plan.numel > MAX_UNKNOWNS
    f = torch.zeros(plan.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SemError, match="SEM_EINVAL"):
        plan.solve_noalloc(f)
    # the largest size that fits: 2^23 unknowns
    plan2 = P.Plan(1, (129, 257, 257), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0, "dirichlet")  # 128*256*256 = 8 Mi
    assert plan2.numel == MAX_UNKNOWNS
    rng = np.random.default_rng(3)
    f2 = torch.from_numpy(rng.standard_normal(plan2.shape)).to("cuda")
    ref = plan2.solve(f2)
    u = plan2.solve_noalloc(f2)
    torch.cuda.synchronize()
    assert torch.equal(u, ref)
