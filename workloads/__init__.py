"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the solver: it only evaluates the
manufactured functions of the paper's accuracy tests at given node
coordinates and draws seeded random numbers.  Node coordinates are always
passed in by the caller (from whichever side is being exercised), so nothing
here depends on the oracle or on the GPU library.

Workloads (paper: Liu, Shen & Zhang, arXiv 2310.00226):
  * "sin111"  u = sin(pi x) sin(pi y) sin(pi z)             (high-order check)
  * "uD"      Dirichlet test solution of Sec. 3.1 (Table 1)
  * "uN"      Neumann test solution of Sec. 3.1 (Table 1) / Appendix script
The right-hand side is f = alpha*u - Laplacian(u), evaluated exactly.
  * Schrodinger-type problem of the paper's variable-coefficient section
    (eq. beta): alpha u - Laplacian(u) + V u = f on [-16, 16]^3 with
    V = beta sin^2(pi x/4) sin^2(pi y/4) sin^2(pi z/4) and exact solution
    cos(pi x/16) cos(pi y/16) cos(pi z/16) (which satisfies homogeneous Neumann
    conditions on that box).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np

NOISE_SEED = 2310       # Helmholtz n=999 workload, N(0,1) * 1e-3
BATCH_SEED = 2311       # 256-solve batch
CH_SEED = 2312          # Cahn-Hilliard initial state


def _outer3(a, b, c):
    return a[:, None, None] * b[None, :, None] * c[None, None, :]


def manufactured(kind: str, x, y, z, alpha: float):
    """Return (u_exact, f) on the tensor grid x (nx) * y (ny) * z (nz), float64.

    f = alpha*u - (u_xx + u_yy + u_zz), written out per separable term.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    pi = math.pi
    if kind == "sin111":
        sx, sy, sz = np.sin(pi * x), np.sin(pi * y), np.sin(pi * z)
        u = _outer3(sx, sy, sz)
        f = (alpha + 3.0 * pi * pi) * u
        return u, f
    if kind == "uD":
        # sin(pi x) sin(2 pi y) sin(3 pi z) + (x - x^3)(y^2 - y^4)(1 - z^2)
        t1 = _outer3(np.sin(pi * x), np.sin(2 * pi * y), np.sin(3 * pi * z))
        gx, gy, gz = x - x**3, y**2 - y**4, 1.0 - z**2
        gxx, gyy, gzz = -6.0 * x, 2.0 - 12.0 * y**2, -2.0 * np.ones_like(z)
        t2 = _outer3(gx, gy, gz)
        lap2 = _outer3(gxx, gy, gz) + _outer3(gx, gyy, gz) + _outer3(gx, gy, gzz)
        u = t1 + t2
        f = alpha * u + 14.0 * pi * pi * t1 - lap2
        return u, f
    if kind == "uN":
        # cos(pi x) cos(2 pi y) cos(3 pi z) + (1-x^2)^3 (1-y^2)^2 (1-z^2)^4
        t1 = _outer3(np.cos(pi * x), np.cos(2 * pi * y), np.cos(3 * pi * z))
        gx, gy, gz = (1 - x**2) ** 3, (1 - y**2) ** 2, (1 - z**2) ** 4
        gxx = -30.0 * x**4 + 36.0 * x**2 - 6.0
        gyy = -4.0 + 12.0 * y**2
        gzz = (56.0 * z**2 - 8.0) * (1 - z**2) ** 2
        t2 = _outer3(gx, gy, gz)
        lap2 = _outer3(gxx, gy, gz) + _outer3(gx, gyy, gz) + _outer3(gx, gy, gzz)
        u = t1 + t2
        f = alpha * u + 14.0 * pi * pi * t1 - lap2
        return u, f
    raise ValueError(f"unknown manufactured solution {kind!r}")


SCHRODINGER_BOX = (-16.0, 16.0, -16.0, 16.0, -16.0, 16.0)


def schrodinger_data(x, y, z, alpha: float, beta: float):
    """(V, u_exact, f) of the Schrodinger-type test problem on the tensor grid
    x * y * z: V from eq. (beta), u = cos(pi x/16) cos(pi y/16) cos(pi z/16) and
    f = (alpha + 3 (pi/16)^2 + V) u, since -Laplacian(u) = 3 (pi/16)^2 u."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    s2 = [np.sin(math.pi * t / 4.0) ** 2 for t in (x, y, z)]
    c = [np.cos(math.pi * t / 16.0) for t in (x, y, z)]
    v = beta * _outer3(*s2)
    u = _outer3(*c)
    f = (alpha + 3.0 * (math.pi / 16.0) ** 2 + v) * u
    return v, u, f


def ch_manufactured(x, y, z, t: float, eps: float, mob: float):
    """(phi*, s) of the Cahn-Hilliard accuracy test at time t: the exact solution
    phi* = cos(pi x) cos(pi y) cos(pi z) e^t on [-1, 1]^3 (homogeneous Neumann) and
    the source s = phi*_t - m Lap mu*, mu* = -eps Lap phi* + (phi*^3 - phi*)/eps,
    which makes phi* solve phi_t = m Lap mu + s (eq. CH-sys plus a source).
    With C = cos cos cos: Lap C = -3 pi^2 C, and cos^3(pi x) = (3 cos(pi x) +
    cos(3 pi x))/4 gives Lap(C^3) term by term."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    pi = math.pi
    c = [np.cos(pi * v) for v in (x, y, z)]
    c3 = [np.cos(pi * v) ** 3 for v in (x, y, z)]
    d2c3 = [(-3.0 * pi * pi * np.cos(pi * v) - 9.0 * pi * pi * np.cos(3.0 * pi * v)) / 4.0 for v in (x, y, z)]
    C = _outer3(*c)
    lap_c3 = _outer3(d2c3[0], c3[1], c3[2]) + _outer3(c3[0], d2c3[1], c3[2]) + _outer3(c3[0], c3[1], d2c3[2])
    et, e3t = math.exp(t), math.exp(3.0 * t)
    phi = C * et
    # Lap mu* = -eps Lap^2 phi* + (Lap(phi*^3) - Lap phi*)/eps, Lap^2 C = 9 pi^4 C
    lap_mu = -eps * (9.0 * pi ** 4) * C * et + (lap_c3 * e3t + 3.0 * pi * pi * C * et) / eps
    s = phi - mob * lap_mu
    return phi, s


def normal_noise(shape, seed: int, scale: float = 1.0, chunks: int = 16) -> np.ndarray:
    """Seeded N(0, scale^2) array of `shape` (float64).

    The leading axis is split into `chunks` fixed slabs, each drawn from its own
    PCG64 stream spawned from SeedSequence(seed); the result depends only on
    (shape, seed, scale, chunks), not on the number of threads used.
    """
    shape = tuple(int(s) for s in shape)
    out = np.empty(shape, dtype=np.float64)
    n0 = shape[0]
    nchunk = max(1, min(chunks, n0))
    bounds = [n0 * c // nchunk for c in range(nchunk + 1)]
    seqs = np.random.SeedSequence(seed).spawn(nchunk)

    def fill(c):
        g = np.random.Generator(np.random.PCG64(seqs[c]))
        sl = out[bounds[c]:bounds[c + 1]]
        g.standard_normal(out=sl.reshape(-1), dtype=np.float64)  # a leading-axis slab is contiguous
        if scale != 1.0:
            sl *= scale

    with ThreadPoolExecutor(max_workers=min(16, nchunk)) as ex:
        list(ex.map(fill, range(nchunk)))
    return out


def helmholtz_rhs(x, y, z, alpha: float, noise_scale: float = 1e-3, seed: int = NOISE_SEED):
    """f = alpha*u - Lap u for u = sin(pi x)sin(pi y)sin(pi z), plus seeded noise."""
    _, f = manufactured("sin111", x, y, z, alpha)
    if noise_scale:
        f += normal_noise(f.shape, seed, noise_scale)
    return f


def batch_draws(count: int = 256, seed: int = BATCH_SEED, k_range=(2, 8), ne_range=(8, 64)):
    """Per-solve parameters of the batched workload: k uniform in {2..8}, Ne per
    axis uniform in {8..64} (both inclusive ranges), alpha ~ U[0, 10]; Dirichlet
    on [-1, 1]^3."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        k = int(g.integers(k_range[0], k_range[1] + 1))
        ne = tuple(int(v) for v in g.integers(ne_range[0], ne_range[1] + 1, size=3))
        alpha = float(g.uniform(0.0, 10.0))
        out.append({"k": k, "ne": ne, "alpha": alpha})
    return out


def batch_rhs(shape, seed: int, index: int) -> np.ndarray:
    """N(0,1) right-hand side of solve `index` in the batch."""
    return normal_noise(shape, seed * 1000003 + index, 1.0, chunks=1)


def ch_initial(shape, seed: int = CH_SEED, amplitude: float = 0.05) -> np.ndarray:
    """phi_0 ~ U[-amplitude, amplitude] on the node grid."""
    g = np.random.Generator(np.random.PCG64(seed))
    return g.uniform(-amplitude, amplitude, size=tuple(shape)).astype(np.float64)
