"""Batched solves (one launch per pass for all problems of a grid) against
single solves and the CPU oracle."""

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


def _problems():
    probs = []
    for i, (n, rho, E, tol) in enumerate([(27, 10.0, (1.0, 0.0), 1e-9), (27, 1e3, (0.3, -1.0), 1e-7),
                                         (81, 1e2, (1.0, 0.0), 1e-8), (81, 1e4, (0.0, 1.0), 1e-6),
                                         (27, 50.0, (0.0, 0.0), 1e-8)]):
        m = ms.grf_two_phase(n, 0.1, 0.4, rho, seed=100 + i)
        probs.append(dict(phase=m.phase, cond=[1.0, rho], E=E, tol=tol, want_field=True))
    rng = np.random.default_rng(3)
    probs.append(dict(phase=rng.integers(0, 3, (45, 27)).astype(np.uint8), cond=[1.0, 7.0, 30.0],
                      E=(0.5, 0.5), tol=1e-9, l0=20.0, want_field=True))
    probs.append(dict(phase=(rng.random((15, 15, 15)) < 0.3).astype(np.uint8), cond=[1.0, 100.0],
                      E=(1.0, 0.0, 0.5), tol=1e-8, want_field=True))
    probs.append(dict(phase=(rng.random((15, 15, 15)) < 0.5).astype(np.uint8), cond=[2.0, 5.0],
                      E=(0.0, 1.0, 0.0), tol=1e-10, want_field=True))
    return probs


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_single(precision):
    from paper_1004_1122_amd import lshom
    probs = _problems()
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    fields, leff, infos = bs.run(precision=precision)
    for i, pr in enumerate(probs):
        s = lshom.Solver(pr["phase"], pr["cond"])
        if pr.get("l0"):
            s.set_reference(pr["l0"])
        e, l1, info = s.solve(pr["E"], tol=pr["tol"], precision=precision)
        assert infos[i]["iterations"] == info["iterations"], i
        assert infos[i]["status"] == 0
        d = len(pr["E"])
        # same kernels, block shapes and reduction order: bit-identical
        assert torch.equal(fields[i], e), i
        assert np.array_equal(leff[i][:d], l1), i


def test_batched_matches_oracle_equal_iterations():
    from paper_1004_1122_amd import lshom
    probs = _problems()
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    fields, leff, infos = bs.run(precision=0)
    for i, pr in enumerate(probs):
        lam = ms.lam_field(pr["phase"], pr["cond"])
        l0 = pr.get("l0") or o.optimal_reference(lam)
        ref = o.cg(lam, l0, pr["E"], n_iter=infos[i]["iterations"])
        e = fields[i].cpu().numpy()
        if not np.any(pr["E"]):
            assert infos[i]["iterations"] == 0 and not np.any(e)
            continue
        assert np.linalg.norm(e - ref["e"]) / np.linalg.norm(ref["e"]) < 1e-10, i
        assert infos[i]["rel_res"] <= pr["tol"]


def test_batched_rejects_bad_phase():
    from paper_1004_1122_amd import lshom
    probs = _problems()[:2]
    bad = probs[1]["phase"].copy()
    bad[0, 0] = 2
    probs[1]["phase"] = bad
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    with pytest.raises(lshom.LshomError):
        bs.run(precision=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_with_uneven_convergence_equals_single(precision):
    """Eight problems of one grid whose iteration counts spread over an order
    of magnitude: as problems finish, the launches shrink to the unfinished
    ones (rows 8, 6, 4, 3, 2, 1), which must not change any result."""
    from paper_1004_1122_amd import lshom
    probs = []
    for i, rho in enumerate(np.geomspace(2.0, 3e4, 8)):
        m = ms.grf_two_phase(27, 0.15, 0.4, float(rho), seed=700 + i)
        probs.append(dict(phase=m.phase, cond=[1.0, float(rho)], E=(1.0, 0.5) if i % 2 else (0.0, 1.0),
                          tol=1e-9, want_field=True))
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    fields, leff, infos = bs.run(precision=precision, graph_block=4)
    iters = [inf["iterations"] for inf in infos]
    assert max(iters) > 4 * min(iters), iters
    for i, pr in enumerate(probs):
        s = lshom.Solver(pr["phase"], pr["cond"])
        e, l1, info = s.solve(pr["E"], tol=pr["tol"], precision=precision, graph_block=4)
        assert infos[i]["status"] == 0
        assert infos[i]["iterations"] == info["iterations"], i
        assert torch.equal(fields[i], e), i
        assert np.array_equal(leff[i][:2], l1), i


@pytest.mark.parametrize("precision", [0, 1])
def test_tail_schedules(precision, tmp_path):
    """The batched autotuner also tunes the launches that cover only the last
    two unfinished problems; a batch that switches to that schedule in its
    tail still meets the FP64 bar, also with an explicitly set tail shape."""
    from paper_1004_1122_amd import lshom
    probs = []
    for i, rho in enumerate(np.geomspace(2.0, 500.0, 6)):
        m = ms.grf_two_phase(27, 0.15, 0.4, float(rho), seed=900 + i)
        probs.append(dict(phase=m.phase, cond=[1.0, float(rho)], E=(1.0, 0.0), tol=1e-8, want_field=True))
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    scheds = bs.autotune(precision=precision, reps=2)
    assert [s["tail_rows"] for s in scheds] == [0, 2]
    fields, _, infos = bs.run(precision=precision, graph_block=4)
    for i, pr in enumerate(probs):
        assert infos[i]["status"] == 0
        if precision == 0:
            lam = ms.lam_field(pr["phase"], pr["cond"])
            ref = o.cg(lam, o.optimal_reference(lam), pr["E"], n_iter=infos[i]["iterations"])
            assert np.linalg.norm(fields[i].cpu().numpy() - ref["e"]) / np.linalg.norm(ref["e"]) < 1e-10, i
        else:
            assert infos[i]["rel_res_true"] <= 1.01e-8
    # a different tail shape: same answers within the bar
    main = scheds[0]
    bs.set_schedule(dict(main, rows_per_block=2, threads_row=128, row_split=0, tail_rows=2))
    f2, _, inf2 = bs.run(precision=precision, graph_block=4)
    for i in range(len(probs)):
        assert abs(inf2[i]["iterations"] - infos[i]["iterations"]) <= 1
        ref = fields[i].cpu().numpy()
        tol = 1e-9 if precision == 0 else 1e-6
        assert np.linalg.norm(f2[i].cpu().numpy() - ref) / np.linalg.norm(ref) < tol, i
    path = tmp_path / "sched.jsonl"
    bs.save_schedules(str(path))
    assert '"tail_rows": 2' in path.read_text()


def test_bench_sweep_full_size():
    """The measured workload itself: the 729^2 circle cell (seed 2), rho = 1e1 .. 1e4, E = e1 and
    e2, one batch per form with autotuned schedules, as the benchmark runs it.  At this size the
    oracle checks every returned field through its own FP64 evaluation of the residual and of
    <L e> (one apply each); the FP64 field of rho = 10, E = e1 equals the oracle's CG at the same
    iteration count; both forms give the same effective conductivities."""
    from paper_1004_1122_amd import lshom
    m = ms.circles_729(seed=2)
    probs = [dict(phase=m.phase, cond=[1.0, rho], E=E, tol=1e-6, want_field=True)
             for rho in (1e1, 1e2, 1e3, 1e4) for E in ((1.0, 0.0), (0.0, 1.0))]
    leffs = {}
    for prec in (0, 1):
        bs = lshom.BatchSolver()
        bs.prepare(probs, precision=prec)
        bs.autotune(precision=prec, reps=1)
        fields, leff, infos = bs.run(precision=prec)
        for i, pr in enumerate(probs):
            lam = ms.lam_field(pr["phase"], pr["cond"])
            l0 = o.optimal_reference(lam)
            e = fields[i].cpu().numpy()
            assert infos[i]["status"] == 0, (prec, i)
            true = o.true_residual(lam, l0, pr["E"], e)
            assert true <= 1.5e-6, (prec, i, true)
            assert abs(true - infos[i]["rel_res_true"]) <= 1e-3 * true, (prec, i)
            np.testing.assert_allclose(leff[i][:2], o.leff(lam, e), rtol=1e-10, atol=1e-13)
            if prec == 0 and i == 0:
                ref = o.cg(lam, l0, pr["E"], n_iter=infos[i]["iterations"])
                assert np.linalg.norm(e - ref["e"]) / np.linalg.norm(ref["e"]) < 1e-10
        leffs[prec] = np.array([x[:2] for x in leff])
        bs.close()
    # diagonal entries are second order in the field error, off-diagonal ones first order
    np.testing.assert_allclose(leffs[1], leffs[0], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("tiles", [(1, 2), (4, 4), (16, 8)], ids=["t1x2", "t4x4", "t16x8"])
def test_column_tiles_3d_batch(precision, tiles):
    """3-D column passes with tiles narrower than one 128-byte line (their
    blocks then run in XCD-grouped order) and as wide as one line (dispatch
    order): a batch of three problems that converge at different iterations
    equals the single solves under the same schedule bit for bit, and FP64
    meets the oracle at an equal iteration count."""
    from paper_1004_1122_amd import lshom
    shape = (15, 21, 9)
    rng = np.random.default_rng(31)
    probs = [dict(phase=(rng.random(shape) < f).astype(np.uint8), cond=[1.0, rho], E=E, tol=1e-9, want_field=True)
             for f, rho, E in ((0.3, 50.0, (1.0, 0.0, 0.0)), (0.4, 400.0, (0.0, 1.0, 0.5)),
                               (0.2, 4.0, (0.3, 0.0, 1.0)))]
    sched = dict(lshom.Solver(probs[0]["phase"], probs[0]["cond"]).get_schedule(precision),
                 tile0=tiles[0], tile1=tiles[1])
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    bs.set_schedule(sched)
    fields, leff, infos = bs.run(precision=precision)
    iters = [inf["iterations"] for inf in infos]
    assert len(set(iters)) > 1, iters
    for i, pr in enumerate(probs):
        s = lshom.Solver(pr["phase"], pr["cond"])
        s.set_schedule(sched)
        assert s.get_schedule(precision)["tile0"] == tiles[0]
        e, l1, info = s.solve(pr["E"], tol=pr["tol"], precision=precision)
        assert infos[i]["status"] == 0 and infos[i]["iterations"] == info["iterations"], i
        assert torch.equal(fields[i], e), i
        assert np.array_equal(leff[i][:3], l1), i
        if precision == 0:
            lam = ms.lam_field(pr["phase"], pr["cond"])
            ref = o.cg(lam, o.optimal_reference(lam), pr["E"], n_iter=info["iterations"])
            got = e.cpu().numpy()
            assert np.linalg.norm(got - ref["e"]) / np.linalg.norm(ref["e"]) < 1e-10, i
        else:
            assert info["rel_res_true"] <= 1.01e-9, i


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_grid_subset_concurrent_groups(precision):
    """The first 24 problems of the 512-problem generator (grids of 81^2,
    243^2 and 729^2, contrasts 10 to 1e4): the three grid groups run on
    streams of their own at once, and every problem equals its single solve
    bit for bit; the 81^2 fields match the oracle at equal iterations."""
    from paper_1004_1122_amd import lshom
    items = [ms.batched_problem(i) for i in range(24)]
    sizes = {m.phase.shape[0] for m in items}
    assert sizes == {81, 243, 729}, sizes
    probs = [dict(phase=m.phase, cond=list(m.cond), E=(1.0, 0.0), tol=1e-6, want_field=True) for m in items]
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    fields, leff, infos = bs.run(precision=precision)
    for i, pr in enumerate(probs):
        print("problem", i, pr["phase"].shape, flush=True)
        s = lshom.Solver(pr["phase"], pr["cond"])
        e, l1, info = s.solve(pr["E"], tol=pr["tol"], precision=precision)
        assert infos[i]["status"] == 0 and info["status"] == 0, i
        assert infos[i]["iterations"] == info["iterations"], i
        assert torch.equal(fields[i], e), i
        assert np.array_equal(leff[i][:2], l1), i
        s.close()
        if precision == 0 and pr["phase"].shape[0] == 81:
            lam = ms.lam_field(pr["phase"], pr["cond"])
            ref = o.cg(lam, o.optimal_reference(lam), pr["E"], n_iter=infos[i]["iterations"])
            err = np.linalg.norm(fields[i].cpu().numpy() - ref["e"]) / np.linalg.norm(ref["e"])
            assert err < 1e-10, (i, err)
    bs.close()
