"""Pins of the oracle's Cahn-Hilliard BDF2/IMEX step (paper Sec. 3.5) (no GPU)."""
import numpy as np

import oracle as O
from workloads import ch_initial

EPS, MOB, DT = 0.05, 0.02, 1e-4


def _problem(ne=(4, 3, 5)):
    return O.Problem(3, ne, (0, 2 * np.pi, 0, 2 * np.pi, 0, 2 * np.pi), 0.0, "neumann")


def test_ch_step_solves_the_bdf2_system():
    # (a I + m dt eps H3^2) phi_{n+1} = phi_hat - (m dt / eps) H3 F'(phi_bar), with H3 applied from
    # the assembled 1D matrices (not the eigenbasis)
    p = _problem()
    phi0 = ch_initial(p.shape, seed=5, amplitude=0.5)
    phi1 = phi0 + 0.01 * np.random.default_rng(6).standard_normal(p.shape)
    phi2 = O.ch_step(p, phi1, phi0, EPS, MOB, DT)
    res = O.ch_operator_residual(p, phi2, phi1, phi0, EPS, MOB, DT)
    scale = np.max(np.abs(2 * phi1 - 0.5 * phi0))
    lam_max = sum(e[0][-1] for e in p.eig)
    assert np.max(np.abs(res)) < 1e-12 * scale * (1 + MOB * DT * EPS * lam_max ** 2)


def test_ch_mass_conservation():
    # 1^T M3 H3 = 0 for homogeneous Neumann, so with phi_{-1} = phi_0 the mass stays at its
    # initial value step after step
    p = _problem()
    m3 = p.mass3()
    phi_nm1 = phi_n = ch_initial(p.shape, seed=9, amplitude=0.05)
    m0 = np.sum(m3 * phi_n)
    for _ in range(20):
        phi_nm1, phi_n = phi_n, O.ch_step(p, phi_n, phi_nm1, EPS, MOB, DT)
    assert abs(np.sum(m3 * phi_n) - m0) < 1e-13 * np.sum(m3)


def test_ch_linear_regime_matches_scalar_recurrence():
    # For a tiny eigenmode v (H3 v = lam v) F'(phi) ~ -phi and each step is linear:
    # (a + m dt eps lam^2) x_{n+1} = (2 x_n - x_{n-1}/2) + (m dt / eps) lam (2 x_n - x_{n-1}).
    # Its closed form through the characteristic roots must match the oracle's time stepping.
    p = _problem((3, 3, 3))
    (lx, sx, _), (ly, sy, _), (lz, sz, _) = p.eig
    i, j, l = 2, 1, 3
    v = sx[:, i][:, None, None] * sy[:, j][None, :, None] * sz[:, l][None, None, :]
    lam = lx[i] + ly[j] + lz[l]
    np.testing.assert_allclose(O.apply_h3(p, v), lam * v, atol=1e-10 * lam * np.max(np.abs(v)))
    a, beta = 1.5, MOB * DT / EPS * lam
    c2, c1, c0 = a + MOB * DT * EPS * lam ** 2, -(2 + 2 * beta), 0.5 + beta
    r1, r2 = np.roots([c2, c1, c0])
    x0 = 1e-9
    # x_{-1} = x_0 = x0 fixes A r1^{-1} + B r2^{-1} = x0 and A + B = x0
    mat = np.array([[1.0, 1.0], [1 / r1, 1 / r2]])
    coef = np.linalg.solve(mat, np.array([x0, x0], dtype=complex))
    nsteps = 30
    phi_nm1 = phi_n = x0 * v
    for _ in range(nsteps):
        phi_nm1, phi_n = phi_n, O.ch_step(p, phi_n, phi_nm1, EPS, MOB, DT)
    x_closed = (coef[0] * r1 ** nsteps + coef[1] * r2 ** nsteps).real
    np.testing.assert_allclose(phi_n, x_closed * v, atol=1e-10 * abs(x_closed) * np.max(np.abs(v)))


def test_ch_bdf2_second_order_in_time():
    """Accuracy test of the BDF2 scheme (Cahn-Hilliard section): the manufactured
    solution cos(pi x) cos(pi y) cos(pi z) e^t on [-1, 1]^3 with eps = 0.2, m = 0.01
    and its source, Q^5 with 8^3 elements (the spatial error is below the time
    error), started from the exact phi(0) and phi(-dt): the relative l2 error at
    T = 0.1 falls by ~4 per halving of dt (second order; the paper's figure)."""
    from workloads import ch_manufactured
    eps, mob, T = 0.2, 0.01, 0.1
    prob = O.Problem(5, (8, 8, 8), (-1, 1, -1, 1, -1, 1), 0.0, "neumann")
    xs = [o.x for o in prob.axes]
    errs = []
    for dt in (0.02, 0.01, 0.005):
        cur, _ = ch_manufactured(*xs, 0.0, eps, mob)
        prev, _ = ch_manufactured(*xs, -dt, eps, mob)
        for n in range(int(round(T / dt))):
            _, s = ch_manufactured(*xs, (n + 1) * dt, eps, mob)
            cur, prev = O.ch_step(prob, cur, prev, eps, mob, dt, forcing=s), cur
        ex, _ = ch_manufactured(*xs, T, eps, mob)
        errs.append(np.linalg.norm(cur - ex) / np.linalg.norm(ex))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 <= r <= 4.4 for r in ratios), (errs, ratios)
    assert errs[-1] <= 1e-5, errs
