"""Launch-shape tuning of the low-precision mode products (sem_plan_tune and
friends): the chosen shapes are valid, no shape changes a result bit, and the
tuning cache file written by one process is read back by the next (needs an
MI355X)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from workloads import normal_noise

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
VALID = {"f32": {128, 96, 64, 32}, "bf16": {1, 2, 4, 17, 18, 20}, "bf16x3": {1, 2, 4, 17, 18, 20}}
BOX = (-1, 1, -1, 1, -1, 1)


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


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
def test_tuned_choices_are_candidates(torch, P, prec):
    _log(f"[tune] choices {prec}")
    plan = P.Plan(4, (30, 27, 33), BOX, 1.0, "dirichlet")
    assert plan.tuning(prec) is None
    ch = plan.tune(prec)
    assert ch is not None and len(ch) == 6 and set(ch) <= VALID[prec], ch
    # a solve after tuning keeps the choices
    f = torch.from_numpy(normal_noise(plan.shape, seed=3)).to("cuda")
    plan.solve_lowp(f, prec=prec)
    assert plan.tuning(prec) == ch


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
@pytest.mark.parametrize("case", [(4, (30, 27, 33), "dirichlet"), (3, (21, 16, 25), "periodic"),
                                  (5, (9, 40, 14), "neumann")], ids=lambda c: f"k{c[0]}-{c[2]}")
def test_every_shape_gives_the_same_bits(torch, P, prec, case):
    k, ne, bc = case
    _log(f"[tune] bitwise {prec} k={k} ne={ne} {bc}")
    plan = P.Plan(k, ne, BOX, 0.5, bc)
    f = torch.from_numpy(normal_noise(plan.shape, seed=11 + k)).to("cuda")
    ref = None
    for c in sorted(VALID[prec]):
        plan.set_tuning(prec, [c] * 6)
        u = plan.solve_lowp(f, prec=prec)
        ur, it, rel, st = plan.solve_refined(f, prec=prec, tol=1e-12, max_iter=30)
        assert st == 0
        got = (u.cpu().numpy(), ur.cpu().numpy(), it)
        if ref is None:
            ref = got
            continue
        assert np.array_equal(got[0], ref[0]), (c, np.max(np.abs(got[0] - ref[0])))
        assert np.array_equal(got[1], ref[1]) and got[2] == ref[2], c
    # mixed shapes per pass as well
    mixed = [sorted(VALID[prec])[i % len(VALID[prec])] for i in range(6)]
    plan.set_tuning(prec, mixed)
    assert np.array_equal(plan.solve_lowp(f, prec=prec).cpu().numpy(), ref[0])


def test_set_tuning_rejects_invalid(torch, P):
    plan = P.Plan(3, (6, 6, 6), BOX, 1.0, "dirichlet")
    for prec, bad in [("f32", [128, 96, 64, 32, 16, 128]), ("bf16", [1, 2, 3, 1, 1, 1]), ("bf16x3", [0] * 6),
                      ("bf16x3", [16] * 6), ("bf16", [19] * 6), ("f64", [1] * 6)]:
        with pytest.raises(P.SemError):
            plan.set_tuning(prec, bad)
    with pytest.raises(P.SemError):
        plan.tune("f64")
    assert plan.tuning("bf16") is None


_CHILD = r"""
import json, sys
sys.path.insert(0, {root!r})
import torch
import paper_2310_00226_amd as P
plan = P.Plan(4, (26, 29, 24), (-1, 1, -1, 1, -1, 1), 1.0, "dirichlet")
out = {{p: plan.tune(p) for p in ("f32", "bf16x3")}}
out["stats"] = P.tune_stats()
print("RESULT " + json.dumps(out), flush=True)
"""


def _child(path):
    env = dict(os.environ, SEM_TUNE_CACHE=path)
    r = subprocess.run([sys.executable, "-c", _CHILD.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("RESULT ")][-1]
    return json.loads(line[len("RESULT "):])


def test_cache_file_is_written_and_read_by_a_fresh_process(torch, P, tmp_path):
    path = str(tmp_path / "semfd_tune.json")
    _log("[tune] cache: first process")
    first = _child(path)
    assert os.path.exists(path)
    with open(path) as fh:
        saved = json.load(fh)
    assert saved["version"] == 1 and len(saved["entries"]) >= 2
    assert first["stats"]["misses"] >= 2 and first["stats"]["entries"] == len(saved["entries"])
    _log("[tune] cache: second process")
    second = _child(path)
    # every pass geometry was found in the file: no timing, the same choices
    assert second["stats"]["misses"] == 0 and second["stats"]["hits"] == 12, second["stats"]
    assert second["f32"] == first["f32"] and second["bf16x3"] == first["bf16x3"]


def test_second_batch_reads_its_tiles_from_the_cache(torch, P):
    """A second sem_batch_create over the same problems finds every length bucket
    in the tuning cache (no new misses, no new entries) and keeps the first one's
    choices."""
    _log("[tune] batch warm cache")
    plans = [P.Plan(3, (6, 7, 5), BOX, 1.0, "dirichlet"), P.Plan(5, (12, 9, 14), BOX, 0.5, "neumann"),
             P.Plan(2, (40, 33, 30), BOX, 2.0, "dirichlet")]
    b1 = P.Batch(plans)
    s1 = P.tune_stats()
    b2 = P.Batch(plans)
    s2 = P.tune_stats()
    assert s2["misses"] == s1["misses"] and s2["entries"] == s1["entries"], (s1, s2)
    assert s2["hits"] > s1["hits"]
    assert b2.tile_rows() == b1.tile_rows()
    assert set(r for r in b1.tile_rows() if r) <= VALID["f32"]


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_cahn_hilliard_steps_with_tuned_shapes(torch, P, prec):
    """The stepper's plan is tuned at creation (outside any capture), and its graphs
    replay those shapes."""
    _log(f"[tune] CH {prec}")
    ch = P.CahnHilliard(3, (10, 10, 10), (0, 6.283185307179586) * 3, 0.05, 0.02, 1e-4, prec=prec,
                        refine_sweeps=2)
    ch_shapes = ch.tuning()
    assert ch_shapes is not None and len(ch_shapes) == 6 and set(ch_shapes) <= VALID[prec], ch_shapes
    rng = np.random.default_rng(4)
    phi = torch.from_numpy(rng.uniform(-0.05, 0.05, ch.shape)).to("cuda")
    prev = phi.clone()
    ch.step(phi, prev, 3)
    assert bool(torch.isfinite(phi).all())
    assert ch.tuning() == ch_shapes
    f64 = P.CahnHilliard(3, (4, 4, 4), (0, 6.283185307179586) * 3, 0.05, 0.02, 1e-4, prec="f64", refine_sweeps=0)
    assert f64.tuning() is None


@pytest.mark.parametrize("prec", ["f32", "bf16", "bf16x3"])
def test_single_pass_launches(torch, P, prec):
    """sem_lowp_pass runs every pass on the plan workspace; solves before and
    after it give identical bits (the workspace is scratch)."""
    _log(f"[tune] single passes {prec}")
    plan = P.Plan(3, (14, 11, 17), BOX, 1.0, "periodic")
    f = torch.from_numpy(normal_noise(plan.shape, seed=21)).to("cuda")
    u0 = plan.solve_lowp(f, prec=prec).cpu().numpy()
    for s in range(6):
        plan.lowp_pass(prec, s, 2)
    torch.cuda.synchronize()
    assert np.array_equal(plan.solve_lowp(f, prec=prec).cpu().numpy(), u0)
    for bad in [(-1, 1), (6, 1), (0, 0)]:
        with pytest.raises(P.SemError):
            plan.lowp_pass(prec, *bad)
    with pytest.raises(P.SemError):
        plan.lowp_pass("f64", 0, 1)
