"""Pin of the oracle's eigenpairs (Sec. 2.3) against a 30-digit reference (no GPU).

The reference is built here with mpmath along a different route from the
oracle's: GLL nodes as the roots of P_k' from its monomial coefficients
(mpmath.polyroots), the closed-form GLL derivative matrix
(D_ij = P_k(x_i) / (P_k(x_j) (x_i - x_j)), D_00 = -k(k+1)/4, D_kk = k(k+1)/4,
zero elsewhere on the diagonal), assembly in mpmath, and mpmath's symmetric
eigensolver on M^{-1/2} K M^{-1/2}.  The oracle's FP64 eigenpairs must agree to
FP64 rounding: eigenvalues to a few ulps of themselves, also at the bottom of
the spectrum (a zero eigenvalue to long-double rounding of lambda_max), the
solve operator S diag(1 / (lambda + alpha)) S^T M, which does not depend on the
choice of basis inside repeated eigenvalues (periodic spectra), to 1e-15 of its
largest entry; S^T M S = I as closely as the exact eigenvectors rounded to FP64
satisfy it, and each eigenvector of a simple eigenvalue to a few ulps.
"""
import mpmath
import numpy as np
import pytest

import oracle as O

DPS = 30


def _legendre_coeffs(k):
    """Monomial coefficients (highest degree first) of P_k, from the three-term
    recurrence in exact rational mpf arithmetic."""
    p0, p1 = [mpmath.mpf(1)], [mpmath.mpf(1), mpmath.mpf(0)]
    if k == 0:
        return p0
    for m in range(1, k):
        # (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}
        xp = p1 + [mpmath.mpf(0)]
        pm = [mpmath.mpf(0)] * (len(xp) - len(p0)) + p0
        p0, p1 = p1, [((2 * m + 1) * a - m * b) / (m + 1) for a, b in zip(xp, pm)]
    return p1


def _reference_axis(k, ne, a, b, bc):
    with mpmath.workdps(DPS + 20):
        c = _legendre_coeffs(k)
        deg = len(c) - 1
        dc = [ci * (deg - i) for i, ci in enumerate(c[:-1])]  # P_k'
        inner = sorted(mpmath.re(r) for r in mpmath.polyroots(dc, maxsteps=400, extraprec=400)) if k >= 2 else []
        x = [mpmath.mpf(-1)] + inner + [mpmath.mpf(1)]
        pk = [mpmath.polyval(c, xi) for xi in x]
        w = [2 / (k * (k + 1) * p * p) for p in pk]
        npt = k + 1
        d = mpmath.matrix(npt, npt)
        for i in range(npt):
            for j in range(npt):
                if i != j:
                    d[i, j] = pk[i] / (pk[j] * (x[i] - x[j]))
        d[0, 0] = -mpmath.mpf(k * (k + 1)) / 4
        d[k, k] = mpmath.mpf(k * (k + 1)) / 4
        kref = d.T * mpmath.diag(w) * d
        h = (mpmath.mpf(b) - mpmath.mpf(a)) / (2 * ne)
        nfull = ne * k + 1
        n = {"dirichlet": nfull - 2, "neumann": nfull, "periodic": nfull - 1}[bc]

        def unknown(g):
            if bc == "dirichlet":
                return g - 1 if 1 <= g <= nfull - 2 else None
            if bc == "periodic":
                return g % n
            return g

        K = mpmath.matrix(n, n)
        M = [mpmath.mpf(0)] * n
        for e in range(ne):
            for i in range(npt):
                gi = unknown(e * k + i)
                if gi is None:
                    continue
                M[gi] += h * w[i]
                for j in range(npt):
                    gj = unknown(e * k + j)
                    if gj is not None:
                        K[gi, gj] += kref[i, j] / h
        mh = [mpmath.sqrt(v) for v in M]
        s1 = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                s1[i, j] = K[i, j] / (mh[i] * mh[j])
        ev, q = mpmath.eigsy(s1)
        lam = [ev[i] for i in range(n)]
        order = sorted(range(n), key=lambda i: lam[i])
        lam = [lam[i] for i in order]
        s = mpmath.matrix(n, n)
        for r in range(n):
            for cc, src in enumerate(order):
                s[r, cc] = q[r, src] / mh[r]
        return lam, s, M


CASES = [(k, ne, bc) for (k, ne) in ((4, 3), (6, 2), (20, 2)) for bc in ("dirichlet", "neumann", "periodic")]


@pytest.mark.parametrize("k,ne,bc", CASES)
def test_eigenpairs_match_30_digit_reference(k, ne, bc):
    a, b, alpha = -1.0, 1.0, 0.7
    lam_r, s_r, m_r = _reference_axis(k, ne, a, b, bc)
    o = O.axis_operators(k, ne, a, b, bc)
    lam, s, f = O.axis_eigen(o)
    n = lam.size
    assert n == len(lam_r)
    lam_ref = np.array([float(v) for v in lam_r])
    eps = np.finfo(float).eps
    # eigenvalues: a few ulps of themselves (the bottom of the spectrum too); a zero
    # eigenvalue (Neumann) to a few long-double units of lambda_max
    err = np.abs(lam - lam_ref)
    floor = 4 * float(np.finfo(np.longdouble).eps) * lam_ref[-1]
    assert np.all(err <= 8 * eps * np.abs(lam_ref) + floor), np.max(err / (np.abs(lam_ref) + floor))
    # S^T M S = I, as closely as the exact eigenvectors rounded to FP64 satisfy it (the
    # storage floor: 4e-16 at n = 13, 3e-15 at Q^20 with n ~ 40)
    s_ref = np.array([[float(s_r[i, j]) for j in range(n)] for i in range(n)])
    floor_g = np.max(np.abs(s_ref.T @ (o.M[:, None] * s_ref) - np.eye(n)))
    g = s.T @ (o.M[:, None] * s)
    assert np.max(np.abs(g - np.eye(n))) <= max(1e-15, 1.5 * floor_g), (np.max(np.abs(g - np.eye(n))), floor_g)
    # eigenvectors column by column, up to sign, where the eigenvalue is separated by
    # more than 1e-6 lambda_max (the periodic pairs split only by the discretisation,
    # 1.4e-8 lambda_max at Q^20, are covered by the basis-free solve operator below)
    gap = np.minimum(np.r_[np.inf, np.diff(lam_ref)], np.r_[np.diff(lam_ref), np.inf])
    for j in np.nonzero(gap > 1e-6 * lam_ref[-1])[0]:
        sg = 1.0 if s[:, j] @ s_ref[:, j] >= 0 else -1.0
        dev = np.max(np.abs(s[:, j] - sg * s_ref[:, j])) / np.max(np.abs(s_ref[:, j]))
        assert dev <= 64 * eps, (j, dev)
    # the solve operator, independent of the basis inside repeated eigenvalues
    with mpmath.workdps(DPS):
        mr = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                acc = mpmath.mpf(0)
                for c in range(n):
                    acc += s_r[i, c] * s_r[j, c] / (lam_r[c] + alpha)
                mr[i, j] = acc * m_r[j]
        g_ref = np.array([[float(mr[i, j]) for j in range(n)] for i in range(n)])
    g_or = (s / (lam + alpha)[None, :]) @ f
    assert np.max(np.abs(g_or - g_ref)) <= 1e-15 * np.max(np.abs(g_ref)) * max(1, n / 16), \
        np.max(np.abs(g_or - g_ref)) / np.max(np.abs(g_ref))
