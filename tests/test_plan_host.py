"""Host side of the library (no GPU): the plan's 1D operators and eigenpairs
against the oracle, eigen invariants, argument validation, and the exported
C ABI."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2310_00226_amd as P
    return P


def test_library_exports_every_declared_symbol(P):
    with open(os.path.join(ROOT, "include", "sem.h")) as fh:
        text = fh.read()
    names = sorted(set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text)))
    assert len(names) >= 10
    lib = ctypes.CDLL(P.binding.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("k,ne,a,b,bc", [
    (1, 9, -1.0, 1.0, "dirichlet"), (2, 3, -1.0, 1.0, "neumann"), (4, 8, -1.0, 1.0, "dirichlet"),
    (5, 7, 0.0, 3.0, "neumann"), (8, 5, -2.0, 1.0, "dirichlet"), (20, 3, -16.0, 16.0, "neumann"),
    (1, 9, 0.0, 2.0, "periodic"), (3, 1, -1.0, 1.0, "periodic"), (4, 2, -1.0, 1.0, "periodic"),
    (5, 50, -16.0, 16.0, "periodic"), (20, 10, -16.0, 16.0, "periodic"), (7, 3, 0.0, 1.0, "periodic"),
])
def test_plan_axis_matches_oracle(P, k, ne, a, b, bc):
    d = P.axis_host(k, ne, a, b, bc)
    o = O.axis_operators(k, ne, a, b, bc)
    lam_o, _, _ = O.axis_eigen(o)
    np.testing.assert_allclose(d["x"], o.x, rtol=0, atol=1e-14 * max(1, abs(a), abs(b)))
    np.testing.assert_allclose(d["mass"], o.M, rtol=1e-14)
    # backward-stable eigenvalues: |dlam| <~ eps * ||S1||
    assert np.max(np.abs(d["lam"] - lam_o)) <= 1e-13 * lam_o[-1]
    n = lam_o.size
    S, F, M = d["S"], d["F"], d["mass"]
    assert np.max(np.abs(S.T @ (M[:, None] * S) - np.eye(n))) <= 1e-13
    res = o.K @ S - (M[:, None] * S) * d["lam"][None, :]
    kinf = np.max(np.sum(np.abs(o.K), axis=1))
    assert np.max(np.max(np.abs(res), axis=0) / (kinf * np.max(np.abs(S), axis=0))) <= 1e-13
    np.testing.assert_allclose(F, S.T * M[None, :], atol=1e-14 * np.max(np.abs(F)))


def test_plan_axis_n999_invariants(P):
    d = P.axis_host(4, 250, -1.0, 1.0, "dirichlet")
    o = O.axis_operators(4, 250, -1.0, 1.0, "dirichlet")
    S, M, lam = d["S"], d["mass"], d["lam"]
    assert np.max(np.abs(S.T @ (M[:, None] * S) - np.eye(999))) <= 1e-13
    res = o.K @ S - (M[:, None] * S) * lam[None, :]
    kinf = np.max(np.sum(np.abs(o.K), axis=1))
    assert np.max(np.max(np.abs(res), axis=0) / (kinf * np.max(np.abs(S), axis=0))) <= 1e-13
    assert abs(lam[0] - (math.pi / 2) ** 2) < 1e-9


@pytest.mark.parametrize("args", [
    (0, 4, -1.0, 1.0, "dirichlet"),     # k < 1
    (4, 0, -1.0, 1.0, "dirichlet"),     # ne < 1
    (4, 4, 1.0, 1.0, "dirichlet"),      # empty interval
    (4, 4, 1.0, -1.0, "neumann"),       # reversed interval
    (1, 1, -1.0, 1.0, "dirichlet"),     # no interior node
])
def test_axis_host_rejects_invalid(P, args):
    with pytest.raises(P.SemError) as ei:
        P.axis_host(*args)
    assert ei.value.status == 1  # SEM_EINVAL


@pytest.mark.parametrize("bc", ["dirichlet", "neumann"])
def test_plan_lowest_eigenvalues_match_continuous_spectrum_n999(P, bc):
    # see the oracle's test of the same name: the low modes are refined to rounding
    d = P.axis_host(4, 250, -1.0, 1.0, bc)
    j = np.arange(1, 6) if bc == "dirichlet" else np.arange(0, 5)
    err = np.abs(d["lam"][:5] - (j * np.pi / 2) ** 2)
    assert np.all(err <= 5e-14 * (1 + j ** 2)), err


@pytest.mark.parametrize("eps,mob,dt,prec,sweeps", [
    (0.0, 0.02, 1e-4, 1, 2),            # eps must be > 0
    (0.05, -1.0, 1e-4, 1, 2),           # mobility must be > 0
    (0.05, 0.02, float("nan"), 1, 2),   # dt must be finite
    (0.05, 0.02, 1e-4, 7, 2),           # unknown precision
    (0.05, 0.02, 1e-4, 1, -1),          # negative sweep count
])
def test_ch_create_rejects_invalid(P, eps, mob, dt, prec, sweeps):
    # argument checks come before any device work, so this runs without a GPU
    import ctypes
    ne = (ctypes.c_int * 3)(4, 4, 4)
    box = (ctypes.c_double * 6)(0, 1, 0, 1, 0, 1)
    out = ctypes.c_void_p(None)
    st = P.lib.sem_ch_create(4, ne, box, eps, mob, dt, prec, sweeps, ctypes.byref(out))
    assert st == 1 and not out.value  # SEM_EINVAL, nothing created


def test_plan_periodic_band_rows(P):
    """Periodic: H = M^{-1} K has the wrap-around couplings in its band rows; the
    library's banded rows, applied with wrapped indices, equal the oracle's dense
    H (checked through sem_axis_host's S and lambda: S diag(lam) S^{-1} = H)."""
    for k, ne in ((3, 4), (2, 1), (5, 3)):
        d = P.axis_host(k, ne, 0.0, 1.0, "periodic")
        o = O.axis_operators(k, ne, 0.0, 1.0, "periodic")
        h = d["S"] @ np.diag(d["lam"]) @ d["F"]
        np.testing.assert_allclose(h, o.K / o.M[:, None], rtol=0, atol=1e-11 * np.max(np.abs(o.K / o.M[:, None])))


def _create(P, k, ne, box, alpha, bc):
    """sem_plan_create through the raw C ABI: argument checks and the singularity
    test run on the host before any device call."""
    lib = ctypes.CDLL(P.binding.LIB_PATH)
    lib.sem_plan_create.restype = ctypes.c_int
    p = ctypes.c_void_p(None)
    st = lib.sem_plan_create(ctypes.c_int(k), (ctypes.c_int * 3)(*ne), (ctypes.c_double * 6)(*box),
                             ctypes.c_double(alpha), ctypes.c_int(bc), ctypes.byref(p))
    return st, p


@pytest.mark.parametrize("k,ne,bc,why", [
    (6, (683, 1, 1), 0, "Dirichlet axis of 6 * 683 - 1 = 4097 unknowns"),
    (4, (1024, 1, 1), 1, "Neumann axis of 4097 unknowns"),
    (8, (513, 2, 2), 2, "periodic axis of 4104 unknowns"),
    (65, (1, 1, 1), 1, "k > 64"),
    (4, (2, 2, 2), 3, "unknown boundary condition"),
    (4, (0, 2, 2), 1, "no element"),
    (1, (1, 2, 2), 0, "Dirichlet axis without an interior node"),
])
def test_plan_create_rejects_before_device_use(P, k, ne, bc, why):
    st, p = _create(P, k, ne, (0.0, 1.0) * 3, 1.0, bc)
    assert st == 1 and not p.value, why  # SEM_EINVAL, no plan


@pytest.mark.parametrize("bc", [1, 2])
def test_plan_create_singular_without_shift(P, bc):
    """Neumann and periodic with alpha = 0: the constants are in the kernel."""
    st, p = _create(P, 3, (2, 2, 2), (0.0, 1.0) * 3, 0.0, bc)
    assert st == 4 and not p.value  # SEM_ESINGULAR


def _create_mixed(P, k, ne, box, alpha, bcs):
    lib = ctypes.CDLL(P.binding.LIB_PATH)
    lib.sem_plan_create_mixed.restype = ctypes.c_int
    p = ctypes.c_void_p(None)
    st = lib.sem_plan_create_mixed(ctypes.c_int(k), (ctypes.c_int * 3)(*ne), (ctypes.c_double * 6)(*box),
                                   ctypes.c_double(alpha), (ctypes.c_int * 3)(*bcs), ctypes.byref(p))
    return st, p


@pytest.mark.parametrize("bcs,alpha,status", [
    ((0, 1, 3), 1.0, 1),   # unknown condition on z
    ((2, 2, -1), 1.0, 1),  # unknown condition on z
    ((1, 2, 2), 0.0, 4),   # no Dirichlet axis and alpha = 0: singular
    ((2, 1, 1), 0.0, 4),
    ((0, 2, 1), -1.0, 1),  # negative alpha
])
def test_plan_create_mixed_rejects_before_device_use(P, bcs, alpha, status):
    st, p = _create_mixed(P, 3, (2, 2, 2), (0.0, 1.0) * 3, alpha, bcs)
    assert st == status and not p.value


def test_mixed_axis_sizes_follow_each_condition(P):
    """Through the host-only axis builder: n = ne k - 1, ne k + 1, ne k."""
    for bc, n in (("dirichlet", 11), ("neumann", 13), ("periodic", 12)):
        assert P.axis_host(3, 4, 0.0, 1.0, bc)["lam"].size == n
