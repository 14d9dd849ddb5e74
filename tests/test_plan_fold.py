"""The reflection-split ("folded") factors of the BF16 passes, on the host (no GPU).

The uniform mesh of an axis is symmetric about its midpoint, so the 1D
eigenvectors are symmetric or antisymmetric and each transform splits into two
half-size blocks on the folded vector (v+_r = v_r + v_R(r), v-_r = v_r - v_R(r)).
Here the whole folded pipeline of the BF16 passes is emulated in float64 numpy
from the plan's folded factors (sem_axis_fold_host), in the order and index
conventions the kernels use (fold z; z forward + fold y; y forward + fold x;
x forward + divide; z, y, x backward to the folded node form; unfold), and
compared with the oracle's solve."""
import numpy as np
import pytest

import oracle as O
from workloads import normal_noise


@pytest.fixture(scope="module")
def P():
    import paper_2310_00226_amd as P
    return P


def refl(n, per):
    i = np.arange(n)
    return (n - i) % n if per else n - 1 - i


def fold_last(v, nrep, per):
    """v+ (nrep) then v- (nrep) along the last axis."""
    n = v.shape[-1]
    r = np.arange(nrep)
    m = refl(n, per)[:nrep]
    return np.concatenate([v[..., r] + v[..., m], v[..., r] - v[..., m]], axis=-1)


def emulate(P, k, ne, box, alpha, bcs, f):
    ax = [P.axis_fold_host(k, ne[a], box[2 * a], box[2 * a + 1], bcs[a]) for a in range(3)]
    per = [bc == "periodic" for bc in bcs]
    nr = [d["nrep"] for d in ax]
    no = [d["nodd"] for d in ax]

    def fwd(x, a):
        """x[..., folded node axis a (2 nrep)] -> modes of axis a in folded order as a
        new leading axis: out[l, ...] = ffold[l, :] . (v+ or v-)."""
        d = ax[a]
        xp, xm = x[..., :nr[a]], x[..., nr[a]:]
        ys = np.tensordot(d["ffold"][:nr[a]], xp, axes=([1], [x.ndim - 1]))
        ya = np.tensordot(d["ffold"][nr[a]:], xm, axes=([1], [x.ndim - 1]))
        return np.concatenate([ys, ya], axis=0)

    def bwd(c, a):
        """c[..., folded modes of axis a] -> folded node form (e then o) as a new leading axis."""
        d = ax[a]
        cs, ca = c[..., :nr[a]], c[..., nr[a]:]
        e = np.tensordot(d["bfold_sym"], cs, axes=([1], [c.ndim - 1]))
        o = np.tensordot(d["bfold_anti"], ca, axes=([1], [c.ndim - 1])) if no[a] else np.zeros_like(e)
        return np.concatenate([e, o], axis=0)

    x0 = fold_last(f, nr[2], per[2])                  # (x, y, z+-)
    y1 = fold_last(fwd(x0, 2), nr[1], per[1])         # (lz, x, y+-)
    y2 = fold_last(fwd(y1, 1), nr[0], per[0])         # (ly, lz, x+-)
    y3 = fwd(y2, 0)                                   # (lx, ly, lz)
    lx, ly, lz = (d["lam_fold"] for d in ax)
    y3 = y3 / (lx[:, None, None] + ly[None, :, None] + lz[None, None, :] + alpha)
    z4 = bwd(y3, 2)                                   # (z'', lx, ly)
    z5 = bwd(z4, 1)                                   # (y'', z'', lx)
    z6 = bwd(z5, 0)                                   # (x'', y'', z'')
    # unfold every axis: node r -> e_r + o_r, node R(r) -> e_r - o_r
    u = z6
    for a in range(3):
        n = f.shape[a]
        m = refl(n, per[a])
        e, o = np.split(u, 2, axis=a)
        out = np.zeros(u.shape[:a] + (n,) + u.shape[a + 1:])
        idx = [slice(None)] * 3
        for r in range(nr[a]):
            idx[a] = r
            er, orr = e[tuple(idx)], o[tuple(idx)]
            idx2 = list(idx)
            idx2[a] = r
            out[tuple(idx2)] = er + orr
            if m[r] != r:
                idx2[a] = m[r]
                out[tuple(idx2)] = er - orr
        u = out
    return u


CASES = [
    (4, (5, 4, 6), (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0), 1.0, ("dirichlet",) * 3),
    (3, (4, 3, 5), (-1.0, 2.0, 0.0, 1.5, -0.5, 0.5), 0.5, ("neumann",) * 3),
    (2, (3, 4, 5), (0.0, 1.0, 0.0, 2.0, 0.0, 1.0), 1.0, ("periodic",) * 3),
    (5, (3, 2, 3), (0.0, 1.0, -1.0, 1.0, 0.0, 2.0), 2.0, ("periodic", "dirichlet", "neumann")),
    (1, (7, 6, 3), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 1.0, ("dirichlet", "periodic", "neumann")),
    (3, (1, 2, 1), (0.0, 1.0, 0.0, 1.0, 0.0, 1.0), 3.0, ("periodic", "periodic", "dirichlet")),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"k{c[0]}-{'-'.join(b[0] for b in c[4])}-{c[1]}")
def test_folded_pipeline_equals_oracle_solve(P, case):
    k, ne, box, alpha, bcs = case
    prob = O.Problem(k, ne, box, alpha, bcs)
    f = normal_noise(prob.shape, seed=77)
    u = emulate(P, k, ne, box, alpha, bcs, f)
    ref = O.fd_solve(prob, f)
    assert np.max(np.abs(u - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref))), np.max(np.abs(u - ref))


@pytest.mark.parametrize("k,ne,bc", [(4, 250, "dirichlet"), (5, 200, "periodic"), (4, 64, "neumann"),
                                     (1, 1, "neumann"), (1, 2, "dirichlet"), (2, 1, "periodic"), (1, 1, "periodic")])
def test_folded_factors_structure(P, k, ne, bc):
    """Counts of the split, eigenvalues equal to the natural ones as a multiset, and
    the folded 1D solve equal to the natural one."""
    d = P.axis_fold_host(k, ne, -1.0, 1.0, bc)
    nat = P.axis_host(k, ne, -1.0, 1.0, bc)
    n = nat["lam"].size
    per = bc == "periodic"
    assert d["nrep"] == (n // 2 + 1 if per else (n + 1) // 2)
    assert d["nrep"] + d["nodd"] == n
    np.testing.assert_allclose(np.sort(d["lam_fold"]), nat["lam"], rtol=1e-15, atol=1e-15 * nat["lam"][-1])
    rng = np.random.default_rng(5)
    v = rng.standard_normal(n)
    alpha = 0.5
    ref = nat["S"] @ ((nat["F"] @ v) / (nat["lam"] + alpha))
    vf = fold_last(v, d["nrep"], per)
    nr = d["nrep"]
    c = np.concatenate([d["ffold"][:nr] @ vf[:nr], d["ffold"][nr:] @ vf[nr:]]) / (d["lam_fold"] + alpha)
    e = d["bfold_sym"] @ c[:nr]
    o = d["bfold_anti"] @ c[nr:] if d["nodd"] else np.zeros(nr)
    m = refl(n, per)
    u = np.zeros(n)
    for r in range(nr):
        u[r] = e[r] + o[r]
        if m[r] != r:
            u[m[r]] = e[r] - o[r]
    assert np.max(np.abs(u - ref)) <= 1e-13 * np.max(np.abs(ref)), np.max(np.abs(u - ref))
