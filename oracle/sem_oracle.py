"""Plain FP64 oracle: test infrastructure only (see oracle/__init__.py).

Paper: Liu, Shen & Zhang, arXiv 2310.00226.  Section numbers below refer to it.

Conventions.  A 3D nodal array is a C-ordered numpy array of shape
(nx, ny, nz); entry [i, j, l] is the value at node (x_i, y_j, z_l).  The paper
stores the same array column-major (x fastest); only the storage order differs,
the mathematics is unchanged.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# 1D reference element: Gauss-Lobatto-Legendre points, weights, derivative
# ---------------------------------------------------------------------------


def legendre(k: int, x):
    """(P_k(x), P_{k-1}(x)) by the three-term Legendre recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if k == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for n in range(1, k):
        p_prev, p = p, ((2 * n + 1) * x * p - n * p_prev) / (n + 1)
    return p, p_prev


def gll(k: int):
    """(k+1)-point Gauss-Lobatto-Legendre nodes (ascending) and weights on [-1, 1].

    Sec. 2.1: the Q^k basis is the Lagrange basis at these points and all
    integrals use this quadrature.  Interior nodes are the roots of P_k'; they
    are found by Newton's method from the Chebyshev-Lobatto points, using
    P_k'' from Legendre's differential equation.  Weights: 2 / (k(k+1) P_k(x)^2).
    """
    if k < 1:
        raise ValueError("k >= 1")
    x = -np.cos(np.pi * np.arange(k + 1) / k)
    x[0], x[-1] = -1.0, 1.0
    xi = x[1:-1].copy()
    for _ in range(100):
        p, pm1 = legendre(k, xi)
        dp = k * (xi * p - pm1) / (xi * xi - 1.0)
        d2p = (2.0 * xi * dp - k * (k + 1) * p) / (1.0 - xi * xi)
        step = dp / d2p
        xi -= step
        if np.all(np.abs(step) <= 1e-16 * np.maximum(1.0, np.abs(xi))):
            break
    x[1:-1] = xi
    # symmetry of the rule: average the two halves to remove rounding asymmetry
    x = 0.5 * (x - x[::-1])
    p, _ = legendre(k, x)
    w = 2.0 / (k * (k + 1) * p * p)
    return x, w


def diff_matrix(x):
    """D[i, j] = l_j'(x_i) for the Lagrange basis at nodes x (Appendix LegendreD).

    Off-diagonal: (w_i / w_j) / (x_i - x_j) with w_i = prod_{m != i}(x_i - x_m);
    diagonal: sum_{m != i} 1 / (x_i - x_m)  (the derivative of l_i at x_i).
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    diff = x[:, None] - x[None, :]
    np.fill_diagonal(diff, 1.0)
    omega = np.prod(diff, axis=1)
    d = (omega[:, None] / omega[None, :]) / diff
    inv = 1.0 / diff
    np.fill_diagonal(inv, 0.0)
    d[np.arange(n), np.arange(n)] = inv.sum(axis=1)
    return d


def element_matrices(k: int):
    """Reference-element stiffness K_ref = D^T W D and lumped mass diag(w).

    Sec. 2.1: stiffness entries are <phi_i', phi_j'> and mass entries
    <phi_i, phi_j> under GLL quadrature; the mass is diagonal because the basis
    interpolates at the quadrature points (Appendix SEGenerator1D).
    """
    x, w = gll(k)
    d = diff_matrix(x)
    k_ref = d.T @ (w[:, None] * d)
    return x, w, k_ref


# ---------------------------------------------------------------------------
# 1D global operators on one axis
# ---------------------------------------------------------------------------


@dataclass
class AxisOps:
    k: int
    ne: int
    a: float
    b: float
    bc: str          # "dirichlet" | "neumann" (homogeneous) | "periodic"
    x: np.ndarray    # node coordinates of the unknowns
    K: np.ndarray    # dense stiffness, n x n
    M: np.ndarray    # lumped mass (diagonal), length n
    h: float         # half element width


def axis_operators(k: int, ne: int, a: float, b: float, bc: str) -> AxisOps:
    """Assemble the 1D stiffness K and lumped mass M on [a, b] with ne elements.

    Appendix SEGenerator1D: ne uniform elements of width 2h, h = (b - a)/(2 ne);
    neighbouring elements share their end node, giving ne*k + 1 nodes; element
    matrices are K_ref / h and h * diag(w).  Homogeneous Neumann keeps every
    node (natural condition).  Homogeneous Dirichlet removes the two boundary
    nodes, leaving ne*k - 1 unknowns (the DoF counts of Table 1).  Periodic
    (Sec. 2.4 lists it among the boundary conditions of the same tensor form;
    Sec. 4 uses it for the Schroedinger tables) identifies the node at b with the
    node at a: the last row and column of the Neumann matrices are added onto the
    first, leaving ne*k unknowns (the DoF counts of Tables tab7c and tab8, e.g.
    250^3 = (50 * 5)^3 for Q^5).
    """
    if bc not in ("dirichlet", "neumann", "periodic"):
        raise ValueError(bc)
    xr, w, k_ref = element_matrices(k)
    h = (b - a) / (2.0 * ne)
    nfull = ne * k + 1
    kfull = np.zeros((nfull, nfull))
    mfull = np.zeros(nfull)
    xfull = np.zeros(nfull)
    for e in range(ne):
        s = e * k
        kfull[s:s + k + 1, s:s + k + 1] += k_ref / h
        mfull[s:s + k + 1] += h * w
        xfull[s:s + k + 1] = a + h * (2 * e + 1 + xr)
    xfull[0], xfull[-1] = a, b
    # <grad 1, grad v> = 0: make every row of the (Neumann) stiffness sum to zero up to one
    # rounding, as LegendreD does for D, before the Dirichlet restriction
    offd = kfull - np.diag(np.diag(kfull))
    np.fill_diagonal(kfull, -offd.sum(axis=1))
    if bc == "dirichlet":
        sl = slice(1, nfull - 1)
        return AxisOps(k, ne, a, b, bc, xfull[sl].copy(), kfull[sl, sl].copy(), mfull[sl].copy(), h)
    if bc == "periodic":
        # P^T K P, P^T m with P the (n+1) x n map of node g to node g mod n
        n = nfull - 1
        fold = np.zeros((nfull, n))
        fold[np.arange(nfull), np.arange(nfull) % n] = 1.0
        return AxisOps(k, ne, a, b, bc, xfull[:n].copy(), fold.T @ kfull @ fold, fold.T @ mfull, h)
    return AxisOps(k, ne, a, b, bc, xfull, kfull, mfull, h)


def element_matrices_hp(k: int, digits: int = 40):
    """Reference-element stiffness and GLL weights to `digits` significant digits
    (mpmath), returned as (hi, lo) pairs of float64 arrays (value = hi + lo).

    Same definitions as element_matrices (Sec. 2.1, Appendix generator): interior
    nodes are the roots of P_k', polished by Newton's method in high precision from
    the float64 nodes; weights 2 / (k(k+1) P_k(x)^2); D[i, j] = l_j'(x_i) by the
    product formula, D[i, i] = sum_{m != i} 1 / (x_i - x_m); K_ref = D^T W D.
    Used where float64 rounding of the operator itself matters: the eigenvalues at
    the bottom of the spectrum come out of a cancellation of ratio
    lambda_max / lambda_min.
    """
    import mpmath
    key = (k, digits)
    if key in _HP_CACHE:
        return _HP_CACHE[key]
    with mpmath.workdps(digits + 10):
        x0, _ = gll(k)
        xs = [mpmath.mpf(-1)] + [mpmath.mpf(float(v)) for v in x0[1:-1]] + [mpmath.mpf(1)]

        def leg(xv):
            p_prev, p = mpmath.mpf(1), xv
            for m in range(1, k):
                p_prev, p = p, ((2 * m + 1) * xv * p - m * p_prev) / (m + 1)
            return p, p_prev

        for j in range(1, k):
            xv = xs[j]
            for _ in range(8):
                p, pm1 = leg(xv)
                dp = k * (xv * p - pm1) / (xv * xv - 1)
                d2p = (2 * xv * dp - k * (k + 1) * p) / (1 - xv * xv)
                xv = xv - dp / d2p
            xs[j] = xv
        ws = [2 / (k * (k + 1) * leg(xv)[0] ** 2) for xv in xs]
        npt = k + 1
        om = [mpmath.fprod(xs[i] - xs[m] for m in range(npt) if m != i) for i in range(npt)]
        d = [[(om[i] / om[j]) / (xs[i] - xs[j]) if i != j else
              mpmath.fsum(1 / (xs[i] - xs[m]) for m in range(npt) if m != i) for j in range(npt)]
             for i in range(npt)]
        kref = [[mpmath.fsum(d[q][i] * ws[q] * d[q][j] for q in range(npt)) for j in range(npt)]
                for i in range(npt)]

        def split(vals):
            hi = np.array([float(v) for v in vals])
            lo = np.array([float(v - mpmath.mpf(float(v))) for v in vals])
            return hi, lo

        out = (split([kref[i][j] for i in range(npt) for j in range(npt)]), split(ws))
    _HP_CACHE[key] = out
    return out


_HP_CACHE: dict = {}


def axis_eigen(ops: AxisOps, refine: bool = True):
    """Generalised eigenpairs K s = lambda M s, ascending, M-orthonormal.

    Sec. 2.3: with M diagonal, form the symmetric S1 = M^{-1/2} K M^{-1/2},
    symmetrise it, take S1 = Q Lambda Q^T, and set T = M^{-1/2} Q (here S);
    its inverse is Q^T M^{1/2} = S^T M (here the forward factor F).
    Returns (lam, S, F).

    The paper leaves the accuracy of the eigenpairs to the library routine.  An
    FP64 dense eigensolver leaves absolute eigenvalue errors ~ eps * lambda_max,
    which the divide of eq. 3D-Poisson turns into relative errors of the lowest
    (dominant) solution modes of ~ eps * cond (~1e-11 at n ~ 1000).  With
    `refine`, numpy's eigenvectors only start a cyclic Jacobi iteration in x87 long
    double on the operator assembled from high-precision element matrices
    (oracle/eigjac.c), which brings the pairs to FP64 rounding.
    """
    mh = np.sqrt(ops.M)
    s1 = ops.K / (mh[:, None] * mh[None, :])
    s1 = 0.5 * (s1 + s1.T)
    lam, q = np.linalg.eigh(s1)
    order = np.argsort(lam, kind="stable")
    lam, q = lam[order], q[:, order]
    s = q / mh[:, None]
    if refine and lam.size > 1:
        from ._native import eig_jacobi
        lam, s = eig_jacobi(ops, q)
    f = (s * ops.M[:, None]).T
    return lam, s, f


_EIG_CACHE: dict = {}


def _axis_eigen_cached(k, ne, a, b, bc):
    key = (k, ne, a, b, bc)
    if key not in _EIG_CACHE:
        if len(_EIG_CACHE) > 16:
            _EIG_CACHE.clear()
        ops = axis_operators(k, ne, a, b, bc)
        _EIG_CACHE[key] = (ops, axis_eigen(ops))
    return _EIG_CACHE[key]


# ---------------------------------------------------------------------------
# 3D problem
# ---------------------------------------------------------------------------


class Problem:
    """-Lap u + alpha u = f on a box, Q^k SEM with ne[a] elements on axis a
    (Sec. 2, eq. pde / matvec3D), with homogeneous Dirichlet, homogeneous Neumann
    or periodic conditions: one kind for every axis (bc a string), or one per
    axis (bc a sequence of three; the operators are Kronecker sums of per-axis
    1D operators, so each axis carries its own condition, Sec. 2.4 remark)."""

    def __init__(self, k: int, ne, box, alpha: float, bc, eigen: bool = True):
        """eigen=False builds only the 1D operators (enough for residuals)."""
        self.k = int(k)
        self.ne = tuple(int(v) for v in ne)
        self.box = tuple(float(v) for v in box)
        self.alpha = float(alpha)
        self.bc = bc
        self.bcs = (bc,) * 3 if isinstance(bc, str) else tuple(bc)
        if len(self.bcs) != 3:
            raise ValueError(bc)
        if eigen:
            pairs = [_axis_eigen_cached(self.k, self.ne[a], self.box[2 * a], self.box[2 * a + 1], self.bcs[a])
                     for a in range(3)]
            self.axes = [p[0] for p in pairs]
            self.eig = [p[1] for p in pairs]
        else:
            self.axes = [axis_operators(self.k, self.ne[a], self.box[2 * a], self.box[2 * a + 1], self.bcs[a])
                         for a in range(3)]
            self.eig = None

    @property
    def shape(self):
        return tuple(o.x.size for o in self.axes)

    def lam3(self):
        lx, ly, lz = (e[0] for e in self.eig)
        return lx[:, None, None] + ly[None, :, None] + lz[None, None, :]

    def mass3(self):
        mx, my, mz = (o.M for o in self.axes)
        return mx[:, None, None] * my[None, :, None] * mz[None, None, :]

    def h_dense(self, a: int):
        o = self.axes[a]
        return o.K / o.M[:, None]


def mode_product(x, mat, axis: int, out=None):
    """Y = x contracted with mat along `axis`: Y[.., l, ..] = sum_m mat[l, m] x[.., m, ..].

    Sec. 2.4 (eq. tensorprod and its three-statement listing): one mode product
    per axis, each a plain matrix product.
    """
    nx, ny, nz = x.shape
    if axis == 2:
        return np.matmul(x, mat.T, out=out)
    if axis == 1:
        return np.matmul(mat, x, out=out)
    if axis == 0:
        res = np.matmul(mat, x.reshape(nx, ny * nz),
                        out=None if out is None else out.reshape(nx, ny * nz))
        return res.reshape(nx, ny, nz)
    raise ValueError(axis)


def fd_solve(prob: Problem, f: np.ndarray, order=(2, 1, 0), alpha=None) -> np.ndarray:
    """Fast-diagonalisation solve of eq. (3D-Poisson) with the alpha shift.

    u = (S_x (x) S_y (x) S_z) [ (F_x (x) F_y (x) F_z) f ] ./ (Lambda3D + alpha),
    F = S^T M.  By default the mode products run in the paper's order: z, y, x
    forward, then the entrywise divide (Appendix Poisson3D adds alpha), then z, y,
    x backward.  The Kronecker factors act on different axes and commute, so any
    `order` gives the same result in exact arithmetic; a second order measures the
    FP64 rounding floor of the solve itself.  `alpha` (default prob.alpha)
    replaces the shift, as the preconditioner of the variable-coefficient
    problem needs.
    """
    f = np.ascontiguousarray(f, dtype=np.float64)
    lams = [e[0] for e in prob.eig]
    buf1 = np.empty_like(f)
    buf2 = np.empty_like(f)
    src, dst = f, buf1
    for a in order:
        mode_product(src, prob.eig[a][2], a, out=dst)
        src, dst = dst, (buf2 if dst is buf1 else buf1)
    shift = prob.alpha if alpha is None else float(alpha)
    src /= (lams[0][:, None, None] + lams[1][None, :, None] + lams[2][None, None, :] + shift)
    for a in order:
        mode_product(src, prob.eig[a][1], a, out=dst)
        src, dst = dst, (buf2 if dst is buf1 else buf1)
    return src


def apply_h3(prob: Problem, u: np.ndarray) -> np.ndarray:
    """(H_x (+) H_y (+) H_z) u with H = M^{-1} K per axis (eq. matvec3D, H-form)."""
    out = mode_product(u, prob.h_dense(2), 2)
    out += mode_product(u, prob.h_dense(1), 1)
    out += mode_product(u, prob.h_dense(0), 0)
    return out


def residual(prob: Problem, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Nodal residual r = f - (alpha I + H_3) u, i.e. M_3^{-1}(M_3 f - A u)."""
    return f - prob.alpha * u - apply_h3(prob, u)


def residual_at(prob: Problem, u: np.ndarray, f: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """The nodal residual at the points idx (an (m, 3) integer array), each
    evaluated from the rows of H_x, H_y, H_z through that point."""
    idx = np.asarray(idx, dtype=np.int64)
    hx, hy, hz = (prob.h_dense(a) for a in range(3))
    out = np.empty(idx.shape[0])
    for t, (i, j, l) in enumerate(idx):
        s = prob.alpha * u[i, j, l]
        s += hx[i, :] @ u[:, j, l]
        s += hy[j, :] @ u[i, :, l]
        s += hz[l, :] @ u[i, j, :]
        out[t] = f[i, j, l] - s
    return out



def _face_shape(shape, axis):
    return tuple(n for a, n in enumerate(shape) if a != axis)


def lift_boundary(prob: Problem, faces) -> np.ndarray:
    """Correction c with which the homogeneous solve of f + c gives the solution
    with non-homogeneous boundary data (Sec. 2.1 remark: the data move into the
    right-hand side, the matrix to invert is unchanged).

    faces[2a], faces[2a + 1] (None: homogeneous) hold the data on the face
    x_a = box[2a] and x_a = box[2a + 1], as arrays of the plan's shape with axis a
    removed (the face nodes whose other coordinates are unknowns).

    Dirichlet axis a (data = u on the face): write u = u_0 + u_b with u_b the data
    at the face nodes of the full grid (ne k + 1 nodes on axis a, zero elsewhere);
    the equations at the unknowns become A u_0 = M_3 f - A u_b, i.e. in nodal
    form c = -(H_x (+) H_y (+) H_z) u_b at the unknowns, H = M^{-1} K of the
    full-grid (Neumann) assembly; alpha u_b vanishes there and so do the other
    axes' terms (they keep the coordinate x_a, and x_a = an end is no unknown),
    leaving c = -H_a(unknowns, end node) g along axis a.
    Neumann axis a (data = outward normal derivative): the weak form gains the
    boundary integral of the data times v, by GLL quadrature on the face the face
    masses times the data; divided by the lumped mass M_3 it is the data over
    the end node's 1D mass, added on the face's nodes (edges and corners take the
    contributions of every face they lie on).
    Periodic axes have no faces.
    """
    c = np.zeros(prob.shape)
    for a in range(3):
        bc = prob.bcs[a]
        if all(faces[2 * a + s] is None for s in (0, 1)):
            continue
        if bc == "periodic":
            raise ValueError("a periodic axis has no boundary data")
        if bc == "neumann":
            col = np.zeros((prob.shape[a], 2))
            col[0, 0] = 1.0 / prob.axes[a].M[0]
            col[-1, 1] = 1.0 / prob.axes[a].M[-1]
        else:
            full = axis_operators(prob.k, prob.ne[a], prob.box[2 * a], prob.box[2 * a + 1], "neumann")
            hfull = full.K / full.M[:, None]
            col = -hfull[1:-1][:, [0, -1]]
        for side in (0, 1):
            g = faces[2 * a + side]
            if g is None:
                continue
            g = np.asarray(g, dtype=np.float64).reshape(_face_shape(prob.shape, a))
            c += np.moveaxis(np.multiply.outer(col[:, side], g), 0, a)
    return c

def dense_system(prob: Problem):
    """Assembled dense A = K(x)M(x)M + M(x)K(x)M + M(x)M(x)K + alpha M(x)M(x)M and
    the diagonal of M(x)M(x)M, in the C (x-slowest) ordering (eq. matvec3D)."""
    kx, ky, kz = (o.K for o in prob.axes)
    mx, my, mz = (np.diag(o.M) for o in prob.axes)
    a = (np.kron(np.kron(kx, my), mz) + np.kron(np.kron(mx, ky), mz)
         + np.kron(np.kron(mx, my), kz) + prob.alpha * np.kron(np.kron(mx, my), mz))
    m3 = np.kron(np.kron(prob.axes[0].M, prob.axes[1].M), prob.axes[2].M)
    return a, m3


def dense_solve(prob: Problem, f: np.ndarray) -> np.ndarray:
    """Brute force: solve A u = M_3 f by LU with partial pivoting."""
    a, m3 = dense_system(prob)
    u = np.linalg.solve(a, m3 * f.reshape(-1))
    return u.reshape(prob.shape)


# ---------------------------------------------------------------------------
# Cahn-Hilliard BDF2 / IMEX step (Sec. 3.5)
# ---------------------------------------------------------------------------


def ch_step(prob: Problem, phi_n, phi_nm1, eps: float, mob: float, dt: float, forcing=None):
    """One step of eq. (chscheme-2): phi_{n+1} = D phi_hat + (m dt/eps) D Lap F'(phi_bar).

    a = 3/2, phi_hat = 2 phi_n - phi_{n-1}/2, phi_bar = 2 phi_n - phi_{n-1},
    F'(phi) = phi^3 - phi (F = (phi^2 - 1)^2 / 4), D = (a I + m dt eps Lap^2)^{-1}.
    The discrete Laplacian is -H_3, so in the eigenbasis Lap -> -Lambda3D:
    phi_{n+1} = S_3 [ (F_3 phi_hat - (m dt/eps) Lambda3D F_3 g) / (a + m dt eps Lambda3D^2) ].
    (prob.alpha is not used.)  `forcing` (nodal values of a source s at t_{n+1},
    as in the accuracy test of the BDF2 scheme, where a manufactured solution
    defines s) adds dt * s to phi_hat: BDF2 applied to phi_t = m Lap mu + s.
    """
    a = 1.5
    phi_hat = 2.0 * phi_n - 0.5 * phi_nm1
    phi_bar = 2.0 * phi_n - phi_nm1
    g = phi_bar ** 3 - phi_bar
    (lx, sx, fx), (ly, sy, fy), (lz, sz, fz) = prob.eig
    lam = prob.lam3()

    def fwd(v):
        return mode_product(mode_product(mode_product(v, fz, 2), fy, 1), fx, 0)

    def bwd(v):
        return mode_product(mode_product(mode_product(v, sz, 2), sy, 1), sx, 0)

    if forcing is not None:
        phi_hat = phi_hat + dt * forcing
    c = (fwd(phi_hat) - (mob * dt / eps) * lam * fwd(g)) / (a + mob * dt * eps * lam * lam)
    return bwd(c)


def ch_operator_residual(prob: Problem, phi_np1, phi_n, phi_nm1, eps, mob, dt):
    """Residual of (a I + m dt eps H_3^2) phi_{n+1} = phi_hat - (m dt/eps) H_3 g,
    evaluated with the assembled H (independent of the eigen path)."""
    a = 1.5
    phi_hat = 2.0 * phi_n - 0.5 * phi_nm1
    phi_bar = 2.0 * phi_n - phi_nm1
    g = phi_bar ** 3 - phi_bar
    lhs = a * phi_np1 + mob * dt * eps * apply_h3(prob, apply_h3(prob, phi_np1))
    rhs = phi_hat - (mob * dt / eps) * apply_h3(prob, g)
    return lhs - rhs


# ---------------------------------------------------------------------------
# Other spectral multipliers on the same transforms (Sec. 1's list of
# applications: exponential time differencing and fractional powers)
# ---------------------------------------------------------------------------


def spectral_apply(prob: Problem, kind: str, a: float, param: float, f: np.ndarray) -> np.ndarray:
    """u = S_3 g(Lambda3D + a) S_3^{-1} f = g(H_3 + a I) f with S_3^{-1} = S_3^T M_3 (the
    transforms of eq. 3D-Poisson) and g(x) = exp(-param x) ("exp": the solution
    operator of u_t = Lap u - a u over a time param) or x^(-param) ("power": the
    fractional Helmholtz operator; param = 1 is the solve of eq. 3D-Poisson)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam = prob.lam3() + a
    t = f
    for ax in (2, 1, 0):
        t = mode_product(t, prob.eig[ax][2], ax)
    if kind == "exp":
        t = t * np.exp(-param * lam)
    elif kind == "power":
        t = t * lam ** (-param)
    else:
        raise ValueError(kind)
    for ax in (2, 1, 0):
        t = mode_product(t, prob.eig[ax][1], ax)
    return t


# ---------------------------------------------------------------------------
# Variable coefficients: alpha u - Lap u + V(x) u = f by PCG (the paper's
# Schrodinger-equation section, eq. shrodinger)
# ---------------------------------------------------------------------------


def schrodinger_apply(prob: Problem, v: np.ndarray, u: np.ndarray) -> np.ndarray:
    """A u = alpha u + H_3 u + V u: the GLL-quadrature weak form
    alpha M_3 u + K_3 u + M_3 V u = M_3 f divided by the diagonal M_3 (nodal form,
    as eq. matvec3D in H-form), with the potential V given at the nodes."""
    return prob.alpha * u + apply_h3(prob, u) + v * u


def pcg_schrodinger(prob: Problem, v: np.ndarray, f: np.ndarray, shift: float, tol: float = 1e-12,
                    max_iter: int = 500):
    """Preconditioned conjugate gradients for A u = f (schrodinger_apply) with
    the fast-diagonalisation solve of (shift I + H_3) as preconditioner; the
    paper takes shift = alpha + beta/2 for 0 <= V <= beta.  A and the
    preconditioner are self-adjoint and positive in the M_3-weighted inner
    product <a, b> = sum M_3 a b, which the iteration uses throughout (the same
    iterates as plain PCG on the symmetric weak form).  Starts from u = 0 and
    stops when ||r||_M <= tol ||f||_M.  Returns (u, iterations, [||r_k||_M / ||f||_M])."""
    m3 = prob.mass3()

    def dot(a, b):
        return float(np.sum(m3 * a * b))

    u = np.zeros_like(f)
    r = np.array(f, dtype=np.float64, copy=True)
    fn = math.sqrt(dot(f, f))
    hist = []
    if fn == 0.0:
        return u, 0, hist
    z = fd_solve(prob, r, alpha=shift)
    p = z.copy()
    rz = dot(r, z)
    for it in range(1, max_iter + 1):
        q = schrodinger_apply(prob, v, p)
        a = rz / dot(p, q)
        u += a * p
        r -= a * q
        hist.append(math.sqrt(dot(r, r)) / fn)
        if hist[-1] <= tol:
            return u, it, hist
        z = fd_solve(prob, r, alpha=shift)
        rz_new = dot(r, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return u, max_iter, hist


def rel_max_err(a, b) -> float:
    """||a - b||_inf / ||b||_inf."""
    b = np.asarray(b)
    return float(np.max(np.abs(np.asarray(a) - b)) / max(np.max(np.abs(b)), 1e-300))


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "np", "dataclass", "annotations")]
