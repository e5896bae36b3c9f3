"""Schedule registry and autotuner: a tuned schedule changes launch shapes and
radix orders only, so results stay within rounding of the default schedule
and of the CPU oracle; invalid schedules are rejected; the JSON-lines cache
round-trips."""

import numpy as np
import pytest

from oracle import lshom_oracle as o
from paper_1004_1122_amd import microstructure as ms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("shape,precision", [((81, 81), 0), ((81, 81), 1), ((45, 27), 0), ((15, 15, 15), 0),
                                             ((15, 15, 15), 1)],
                         ids=["81x81-fp64", "81x81-mixed", "45x27-fp64", "15^3-fp64", "15^3-mixed"])
def test_autotuned_solve_matches_oracle(shape, precision):
    from paper_1004_1122_amd import lshom
    rng = np.random.default_rng(11)
    phase = (rng.random(shape) < 0.35).astype(np.uint8)
    cond = [1.0, 200.0]
    s = lshom.Solver(phase, cond)
    E = (1.0,) + (0.0,) * (len(shape) - 1)
    e0, l0_eff, i0 = s.solve(E, tol=1e-9, precision=precision)
    sched = s.autotune(precision=precision, reps=3)
    assert sched["N"] == list(shape) and sched["ms_per_iter"] > 0
    assert sched["rows_per_block"] % 2 == 0
    for a, rad in enumerate(sched["radix"]):
        assert int(np.prod(rad)) == shape[a]
    assert s.get_schedule(precision)["radix"] == sched["radix"]
    e1, l1_eff, i1 = s.solve(E, tol=1e-9, precision=precision)
    assert abs(i1["iterations"] - i0["iterations"]) <= 1
    e1 = e1.cpu().numpy()
    assert _rel(e1, e0.cpu().numpy()) < (1e-10 if precision == 0 else 1e-7)
    if precision == 0:
        lam = ms.lam_field(phase, cond)
        ref = o.cg(lam, o.optimal_reference(lam), E, n_iter=i1["iterations"])
        assert _rel(e1, ref["e"]) < 1e-10


def test_set_schedule_rejects_invalid():
    from paper_1004_1122_amd import lshom
    phase = np.zeros((27, 27), np.uint8)
    s = lshom.Solver(phase, [1.0])
    good = s.get_schedule(0)
    bad = dict(good, radix=[[3, 3, 2], good["radix"][1]])
    with pytest.raises(lshom.LshomError) as ei:
        s.set_schedule(bad)
    assert ei.value.status == lshom.LSHOM_ERR_INVALID_ARG
    with pytest.raises(lshom.LshomError):
        s.set_schedule(dict(good, rows_per_block=3))
    with pytest.raises(lshom.LshomError):
        s.set_schedule(dict(good, rows_per_block=4096))
    with pytest.raises(lshom.LshomError):
        s.set_schedule(dict(good, radix=[[27], good["radix"][1]]))  # radix above 9
    with pytest.raises(lshom.LshomError):
        s.set_schedule(dict(good, threads_row=64))
    # forced 256-thread blocks are accepted and give the same field up to rounding
    e0, _, _ = s.solve((1.0, 0.0), tol=1e-10)
    s.set_schedule(dict(good, threads_row=256, threads_col=256))
    assert s.get_schedule(0)["threads_row"] == 256
    e1, _, _ = s.solve((1.0, 0.0), tol=1e-10)
    assert float((e1 - e0).norm() / e0.norm()) < 1e-12
    # a valid reordering is accepted and applied
    s.set_schedule(dict(good, radix=[[3, 9], [9, 3]], rows_per_block=6))
    now = s.get_schedule(0)
    assert now["radix"] == [[3, 9], [9, 3]] and now["rows_per_block"] == 6


def test_schedule_cache_roundtrip(tmp_path):
    from paper_1004_1122_amd import lshom
    phase = (np.random.default_rng(1).random((27, 45)) < 0.5).astype(np.uint8)
    s = lshom.Solver(phase, [1.0, 10.0])
    s.set_schedule(dict(s.get_schedule(1), radix=[[3, 9], [5, 9]], rows_per_block=4, tile0=2))
    path = tmp_path / "sched.jsonl"
    s.save_schedules(str(path))
    text = path.read_text()
    assert '"N": [27, 45, 1]' in text and '"precision": 1' in text
    s2 = lshom.Solver(phase, [1.0, 10.0])
    s2.load_schedules(str(path))
    got = s2.get_schedule(1)
    assert got["radix"] == [[3, 9], [5, 9]] and got["rows_per_block"] == 4 and got["tile0"] == 2
    # the FP64 schedule was not in the file
    assert s2.get_schedule(0) == s.get_schedule(0) or s2.get_schedule(0)["radix"] != [[3, 9], [5, 9]]
    e1, _, i1 = s.solve((1.0, 0.0), tol=1e-8, precision=1)
    e2, _, i2 = s2.solve((1.0, 0.0), tol=1e-8, precision=1)
    assert i1["iterations"] == i2["iterations"] and torch.equal(e1, e2)


def test_batched_autotune_keeps_results():
    from paper_1004_1122_amd import lshom
    probs = []
    for i, (n, rho) in enumerate([(27, 10.0), (27, 1e3), (81, 1e2), (81, 1e4)]):
        m = ms.grf_two_phase(n, 0.1, 0.4, rho, seed=300 + i)
        probs.append(dict(phase=m.phase, cond=[1.0, rho], E=(1.0, 0.0), tol=1e-9, want_field=True))
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    f0, leff0, inf0 = bs.run(precision=0)
    f0 = [f.clone() for f in f0]
    scheds = bs.autotune(reps=3)
    assert sorted(tuple(s["N"]) for s in scheds) == [(27, 27), (81, 81)]
    f1, leff1, inf1 = bs.run(precision=0)
    for i in range(len(probs)):
        assert abs(inf1[i]["iterations"] - inf0[i]["iterations"]) <= 1
        assert _rel(f1[i].cpu().numpy(), f0[i].cpu().numpy()) < 1e-10
        assert np.allclose(leff1[i], leff0[i], rtol=1e-10, atol=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_pass_timing_inside_solves(precision):
    """Eager solves with per-launch events give the graph solve's results bit for
    bit; the timer's bytes are the per-pass model bytes times the iterations."""
    from paper_1004_1122_amd import lshom
    probs = []
    for i, rho in enumerate([10.0, 1e3, 1e2]):
        m = ms.grf_two_phase(81, 0.1, 0.4, rho, seed=500 + i)
        probs.append(dict(phase=m.phase, cond=[1.0, rho], E=(1.0, 0.0), tol=1e-8, want_field=True))
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    f0, leff0, inf0 = bs.run(precision=precision)
    f0 = [f.clone() for f in f0]
    bs.set_pass_timing(True)
    f1, leff1, inf1 = bs.run(precision=precision)
    t = bs.pass_timing()
    bs.set_pass_timing(False)
    for i in range(len(probs)):
        assert torch.equal(f0[i], f1[i]) and inf0[i]["iterations"] == inf1[i]["iterations"]
    assert set(t) == {"axis0_inverse", "row", "axis0_forward", "update"}
    iters = sum(i["iterations"] for i in inf1)
    s = lshom.Solver(probs[0]["phase"], probs[0]["cond"])
    unit = {k: b for k, (_, b) in s.time_passes(precision, reps=1).items()}
    for k, (ms_, by, n) in t.items():
        assert ms_ > 0 and n >= max(i["iterations"] for i in inf1)
        assert by == pytest.approx(iters * unit[k], rel=1e-12), k


def test_last_block_covers_the_remaining_iterations():
    """Once the residual has fallen over a block, the next block is sized to
    the iterations still needed at that rate: a single solve launches its
    passes for little more than its own iteration count (counted with pass
    timing, where blocks are queued directly), with the same result as fixed
    blocks of 16 in a graph."""
    from paper_1004_1122_amd import lshom
    m = ms.grf_two_phase(81, 0.1, 0.4, 10.0, seed=520)
    s = lshom.Solver(m.phase, [1.0, 10.0])
    e_graph, _, i_graph = s.solve((1.0, 0.0), tol=1e-6)
    s.set_pass_timing(True)
    e_eager, _, i_eager = s.solve((1.0, 0.0), tol=1e-6)
    t = s.pass_timing()
    s.set_pass_timing(False)
    assert i_graph["iterations"] == i_eager["iterations"] and torch.equal(e_graph, e_eager)
    n_it = i_eager["iterations"]
    # 18 iterations here (the oracle's count): the first block of 16 has no
    # rate yet, the second is sized to what the residual still needs (about
    # 2 at the rate of the first block) instead of another 16
    assert 16 < n_it <= 20
    for k, (_, _, n) in t.items():
        assert n_it <= n <= n_it + 4, (k, n, n_it)
