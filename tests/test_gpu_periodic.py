"""GPU parity of periodic plans (SEM_BC_PERIODIC) against the oracle: the FP64
solve, the matrix-free residual (wrap-around neighbours in the march kernel for
k <= 8 and in the generic kernel above), refined low-precision solves, batched
solves, and the variable-coefficient PCG on the paper's periodic Schroedinger
problem (Tables tab7c and tab8).

Bars: as for the other boundary conditions -- FP64 solve within 1e-12 of the
oracle's max plus 10 x its rounding floor; residual within 1e-14 ||H||_inf
(absolute, unit-size inputs); refined and batched solves within 1e-10; PCG
within 1e-10 of the oracle's PCG.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import SCHRODINGER_BOX, batch_rhs, normal_noise, schrodinger_data

pytestmark = pytest.mark.gpu

CASES = [
    # k, ne, box, alpha
    (4, (12, 9, 10), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), 1.0),      # 48 x 36 x 40
    (3, (50, 45, 43), (0.0, 2.0, -1.0, 1.0, 0.0, 3.0), 0.5),       # 150 x 135 x 129: tiles + tails
    (5, (51, 50, 52), (-16.0, 16.0, -16.0, 16.0, -16.0, 16.0), 1.0),  # 255 x 250 x 260
    (2, (1, 3, 1), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0),           # 2 x 6 x 2: offsets alias nodes
    (1, (200, 3, 1), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0),         # 200 x 3 x 1
    (6, (1, 30, 1), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), 0.3),       # 6 x 180 x 6, n < 2k + 1
    (8, (3, 20, 17), (0.0, 1.0, 0.0, 5.0, -1.0, 1.0), 3.0),        # 24 x 160 x 136
    (9, (3, 2, 4), (0.0, 1.0, 0.0, 1.0, 0.0, 2.0), 1.0),           # 27 x 18 x 36: generic residual
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


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{c[1]}")
def test_periodic_solve_and_residual(torch, P, case):
    k, ne, box, alpha = case
    _log(f"[periodic] solve + residual k={k} ne={ne}")
    prob = O.Problem(k, ne, box, alpha, "periodic")
    plan = P.Plan(k, ne, box, alpha, "periodic")
    assert plan.shape == tuple(k * n for n in ne)
    np.testing.assert_allclose(plan.nodes(0), prob.axes[0].x, rtol=0, atol=1e-13)
    f = normal_noise(prob.shape, seed=40 + k)
    ref = O.fd_solve(prob, f)
    u = plan.solve(_dev(torch, f)).cpu().numpy()
    err = np.max(np.abs(u - ref))
    assert err <= _bound(prob, f, ref, 1e-12), err
    # residual of arbitrary (u, f)
    uu = normal_noise(prob.shape, seed=50 + k)
    r = plan.residual(_dev(torch, uu), _dev(torch, f)).cpu().numpy()
    hnorm = sum(np.max(np.sum(np.abs(prob.h_dense(a)), axis=1)) for a in range(3)) + alpha
    rerr = np.max(np.abs(r - O.residual(prob, uu, f)))
    _log(f"    solve rel err {err / np.max(np.abs(ref)):.2e}, residual err / ||H|| {rerr / hnorm:.2e}")
    assert rerr <= 1e-14 * hnorm


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[3], CASES[5], CASES[6]],
                         ids=lambda c: f"k{c[0]}-{c[1]}")
def test_periodic_refined(torch, P, case, prec):
    k, ne, box, alpha = case
    prob = O.Problem(k, ne, box, alpha, "periodic")
    plan = P.Plan(k, ne, box, alpha, "periodic")
    f = normal_noise(prob.shape, seed=60 + k)
    ref = O.fd_solve(prob, f)
    u, iters, rel, st = plan.solve_refined(_dev(torch, f), prec=prec, tol=1e-12, max_iter=40)
    err = np.max(np.abs(u.cpu().numpy() - ref))
    _log(f"[periodic] refined {prec} k={k} ne={ne}: {iters} iterations, rel err {err / np.max(np.abs(ref)):.2e}")
    assert st == 0 and err <= _bound(prob, f, ref, 1e-10)


def test_periodic_batch(torch, P):
    """Periodic plans in a batch with Dirichlet and Neumann ones, in FP32 and in
    SEM_BF16X3 (the 100 x 104 x 96 periodic problem takes the split-BF16 passes)."""
    specs = [
        {"k": 4, "ne": (25, 26, 24), "alpha": 1.0, "bc": "periodic"},
        {"k": 3, "ne": (5, 7, 2), "alpha": 0.5, "bc": "periodic"},
        {"k": 2, "ne": (1, 3, 1), "alpha": 2.0, "bc": "periodic"},
        {"k": 8, "ne": (2, 1, 3), "alpha": 3.0, "bc": "dirichlet"},
        {"k": 5, "ne": (9, 4, 6), "alpha": 0.7, "bc": "neumann"},
    ]
    box = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)
    plans = [P.Plan(s["k"], s["ne"], box, s["alpha"], s["bc"]) for s in specs]
    batch = P.Batch(plans)
    fs = [batch_rhs(p.shape, 71, i) for i, p in enumerate(plans)]
    fd = [_dev(torch, f) for f in fs]
    refs = [O.fd_solve(O.Problem(s["k"], s["ne"], box, s["alpha"], s["bc"]), f) for s, f in zip(specs, fs)]
    for prec in ("f32", "bf16x3"):
        ud = [torch.empty_like(f) for f in fd]
        its, st = batch.solve(fd, ud, prec=prec, tol=1e-12, max_iter=40)
        assert st == 0
        for i, (s, ref) in enumerate(zip(specs, refs)):
            prob = O.Problem(s["k"], s["ne"], box, s["alpha"], s["bc"])
            err = np.max(np.abs(ud[i].cpu().numpy() - ref))
            assert err <= _bound(prob, fs[i], ref, 1e-10), (prec, i, err)
        _log(f"[periodic] batch {prec}: iterations {its}")


@pytest.mark.parametrize("beta", [1.0, 10.0])
def test_periodic_pcg_matches_oracle(torch, P, beta):
    """The paper's Schroedinger problem with periodic conditions, Q^5 with 20
    elements per axis (n = 100): the GPU PCG (FP64 and split-BF16
    preconditioner) equals the oracle's PCG and takes the same number of
    iterations (+-1)."""
    prob = O.Problem(5, (20, 20, 20), SCHRODINGER_BOX, 1.0, "periodic")
    v, ue, f = schrodinger_data(*(o.x for o in prob.axes), 1.0, beta)
    shift = 1.0 + beta / 2
    ref, it_ref, _ = O.pcg_schrodinger(prob, v, f, shift, tol=1e-12, max_iter=300)
    plan = P.Plan(5, (20, 20, 20), SCHRODINGER_BOX, 1.0, "periodic")
    for prec in ("f64", "bf16x3"):
        u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=shift, prec=prec, tol=1e-12,
                                        max_iter=300)
        err = O.rel_max_err(u.cpu().numpy(), ref)
        _log(f"[periodic] pcg beta={beta:g} {prec}: {it} iterations (oracle {it_ref}), err {err:.2e}")
        assert st == 0 and abs(it - it_ref) <= 1 and err <= 1e-10


@pytest.mark.timeout(900)
def test_periodic_pcg_table_tab7c_mesh(torch, P):
    """Table tab7c's first mesh, 250^3 DoFs (Q^5, 50 elements per axis, periodic).
    beta = 1 takes the paper's 10 iterations (+-1).  For beta = 10 and 100 no
    reading of the paper's stop reproduces its 35 and 85 (parity unpinned: this
    PCG takes 19-24 and 48-64 iterations for every stop from 1e-12 to round-off,
    the paper's finest meshes print 25 and 72), so there the GPU iteration is
    held to the oracle's PCG on the same mesh: the same iteration count (+-1,
    FP64 preconditioner) and the same solution (1e-10); the split-BF16
    preconditioner within +-2 iterations or 10% (52 against 48 at beta = 100).  Errors against the exact solution are
    the discretisation error at beta = 1 (~1.3e-13) and grow with the condition
    number at the 1e-12 stop (2.3e-12 at beta = 100)."""
    plan = P.Plan(5, (50, 50, 50), SCHRODINGER_BOX, 1.0, "periodic")
    assert plan.shape == (250, 250, 250)
    prob = O.Problem(5, (50, 50, 50), SCHRODINGER_BOX, 1.0, "periodic")
    xs = [plan.nodes(a) for a in range(3)]
    for beta, ebound in ((1.0, 1e-12), (10.0, 1e-11), (100.0, 1e-11)):
        v, ue, f = schrodinger_data(*xs, 1.0, beta)
        shift = 1.0 + beta / 2
        ref, it_ref, _ = O.pcg_schrodinger(prob, v, f, shift, tol=1e-12, max_iter=300)
        vd, fd = _dev(torch, v), _dev(torch, f)
        u, it, rel, st = plan.pcg_solve(vd, fd, shift=shift, prec="f64", tol=1e-12, max_iter=300)
        err_ref = O.rel_max_err(u.cpu().numpy(), ref)
        u2, it2, _, st2 = plan.pcg_solve(vd, fd, shift=shift, prec="bf16x3", tol=1e-12, max_iter=300)
        err = float((u2 - _dev(torch, ue)).abs().max())
        _log(f"[periodic] 250^3 beta={beta:g}: {it} iterations FP64 preconditioner, {it2} split BF16, oracle "
             f"{it_ref} (paper: 10 / 35 / 85); rel err vs oracle {err_ref:.2e}, max error vs exact {err:.2e}")
        assert st == 0 and st2 == 0 and abs(it - it_ref) <= 1, (beta, it, it_ref)
        assert abs(it2 - it_ref) <= max(2, it_ref // 10), (beta, it2, it_ref)
        assert err_ref <= 1e-10 and err <= ebound, (beta, err_ref, err)
        if beta == 1.0:
            assert 9 <= it <= 11 and 9 <= it2 <= 11  # Table tab7c: 10 on every mesh


def test_periodic_q20_table_tab8(torch, P):
    """Table tab8's first row exactly: Q^20, 25^3 elements, periodic (500^3 DoFs),
    beta = 1, 10, 100; the paper reports max errors 1.89e-13, 1.62e-13, 1.29e-13.
    Here they must stay within 5e-13."""
    plan = P.Plan(20, (25, 25, 25), SCHRODINGER_BOX, 1.0, "periodic")
    assert plan.shape == (500, 500, 500)
    xs = [plan.nodes(a) for a in range(3)]
    for beta in (1.0, 10.0, 100.0):
        v, ue, f = schrodinger_data(*xs, 1.0, beta)
        u, it, rel, st = plan.pcg_solve(_dev(torch, v), _dev(torch, f), shift=1.0 + beta / 2, prec="f64",
                                        tol=1e-14, max_iter=300)
        err = float((u - _dev(torch, ue)).abs().max())
        _log(f"[periodic] Q^20 500^3 beta={beta:g}: {it} iterations, max error {err:.2e}")
        assert st == 0 and err <= 5e-13, (beta, err)


def test_periodic_rejects_singular(torch, P):
    with pytest.raises(P.SemError) as ei:
        P.Plan(3, (2, 2, 2), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 0.0, "periodic")
    assert ei.value.status == 4  # SEM_ESINGULAR: constants are in the kernel
