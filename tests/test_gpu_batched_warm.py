"""Warm starts inside batched solves (lshom_problem.x0_dev) against single
warm-started solves and the oracle, batched network inference feeding a
batched solve, and a batch solver reused across cells."""

import os

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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _warm_cases():
    """81^2 problems with a good warm start (a few oracle CG steps, perturbed),
    a useless one (NaN: rejected) and none."""
    out = []
    rng = np.random.default_rng(41)
    for i, (rho, kind) in enumerate([(1e2, "good"), (1e3, "nan"), (3e3, "good"), (10.0, "none"),
                                     (5e2, "good"), (2e4, "good")]):
        m = ms.grf_two_phase(81, 0.1, 0.45, rho, seed=1200 + i)
        lam = m.lam()
        l0 = o.optimal_reference(lam)
        x0 = None
        if kind == "good":
            x0 = o.cg(lam, l0, (1.0, 0.0), n_iter=6)["e"] + 1e-3 * rng.standard_normal((2, 81, 81))
        elif kind == "nan":
            x0 = np.full((2, 81, 81), np.nan)
        out.append(dict(phase=m.phase, cond=[1.0, rho], E=(1.0, 0.0), tol=1e-8, want_field=True,
                        x0=None if x0 is None else torch.from_numpy(x0), kind=kind))
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_warm_equals_single(precision):
    from paper_1004_1122_amd import lshom
    probs = _warm_cases()
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=1)
    fields, leff, infos = bs.run(precision=precision)
    for i, pr in enumerate(probs):
        s = lshom.Solver(pr["phase"], pr["cond"])
        e, l1, info = s.solve(pr["E"], tol=pr["tol"], precision=precision, x0=pr["x0"])
        assert infos[i]["status"] == 0, i
        assert infos[i]["warm_start_used"] == (1 if pr["kind"] == "good" else 0), i
        assert info["warm_start_used"] == infos[i]["warm_start_used"], i
        if pr["kind"] == "good":
            # the same kernels on the same data: bit for bit
            assert infos[i]["iterations"] == info["iterations"], i
            assert torch.equal(fields[i], e), i
            assert np.array_equal(leff[i][:2], l1), i
        else:
            # started from e = E inside a batch whose other problems were warm
            # (the residual of E formed by the general pass): the cold answer
            assert abs(infos[i]["iterations"] - info["iterations"]) <= 1, i
            lam = ms.lam_field(pr["phase"], pr["cond"])
            if precision == 0:
                ref = o.cg(lam, o.optimal_reference(lam), pr["E"], n_iter=infos[i]["iterations"])
                assert _rel(fields[i].cpu().numpy(), ref["e"]) < 1e-10, i
            else:
                assert infos[i]["rel_res_true"] <= 1.01 * pr["tol"], i
    # every answer is within the a-posteriori bound of the converged oracle
    for i, pr in enumerate(probs):
        lam = ms.lam_field(pr["phase"], pr["cond"])
        l0 = o.optimal_reference(lam)
        ref = o.cg(lam, l0, pr["E"], tol=1e-13)["e"]
        bound = (l0 / lam.min()) * pr["tol"] * 2.0
        assert _rel(fields[i].cpu().numpy(), ref) <= bound, i


def test_batched_warm_all_rejected_is_the_cold_batch():
    from paper_1004_1122_amd import lshom
    probs = [p for p in _warm_cases() if p["kind"] != "nan"][:3]
    cold = [dict(p, x0=None) for p in probs]
    bad = [dict(p, x0=torch.full((2, 81, 81), float("nan"), dtype=torch.float64)) for p in probs]
    bs = lshom.BatchSolver()
    bs.prepare(cold, precision=0)
    f_c, l_c, i_c = bs.run(precision=0)
    f_c = [f.clone() for f in f_c]
    bs.prepare(bad, precision=0)
    f_b, l_b, i_b = bs.run(precision=0)
    for i in range(len(probs)):
        assert i_b[i]["warm_start_used"] == 0
        assert i_b[i]["iterations"] == i_c[i]["iterations"]
        assert torch.equal(f_b[i], f_c[i])
        assert np.array_equal(l_b[i], l_c[i])


def test_batched_warm_start_rejects_other_methods():
    from paper_1004_1122_amd import lshom
    probs = [p for p in _warm_cases() if p["kind"] == "good"][:1]
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    with pytest.raises(lshom.LshomError):
        bs.run(precision=0, method=lshom.METHOD_FFTH)


def test_batched_network_inference_feeds_batched_solve():
    """One network call over many images (held-out 243^2 problems), its
    predictions handed to one batched solve: each result equals the single
    warm-started solve bit for bit and stays within the a-posteriori bound of
    the cold answer."""
    from paper_1004_1122_amd import cnn, lshom
    if not os.path.exists(cnn.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    net = cnn.WarmStartNet.load(cnn.DEFAULT_WEIGHTS)
    items = [ms.warmstart_eval_problem(i, 243) for i in range(6)]
    phases = np.stack([m.phase for m in items])
    x0 = net.forward(phases, np.array([m.info["log10_rho"] for m in items]))
    assert tuple(x0.shape) == (6, 2, 243, 243)
    probs = [dict(phase=m.phase, cond=m.cond, E=(1.0, 0.0), tol=1e-6, want_field=True, x0=x0[b])
             for b, m in enumerate(items)]
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    fields, leff, infos = bs.run(precision=0)
    for b, m in enumerate(items):
        s = lshom.Solver(m.phase, m.cond)
        e_w, l_w, i_w = s.solve((1.0, 0.0), tol=1e-6, x0=x0[b])
        e_c, _, i_c = s.solve((1.0, 0.0), tol=1e-6)
        assert infos[b]["status"] == 0
        assert infos[b]["warm_start_used"] == i_w["warm_start_used"]
        if i_w["warm_start_used"]:
            assert infos[b]["iterations"] == i_w["iterations"]
            assert torch.equal(fields[b], e_w)
        bound = 2.0 * (0.5 * (1.0 + m.info["rho"])) * 1e-6
        assert float((fields[b] - e_c).norm() / e_c.norm()) <= bound, b
    net.close()


def test_batch_solver_reused_across_cells():
    """One BatchSolver (one workspace, cached iteration graphs) solves the same
    grid first on the unit cell, then on a cell of side lengths (1, 3): both
    runs equal single solves on those cells and the oracle's CG at the same
    iteration count (the wave vector xi = k / Y of Sec. 2.1 changes with the
    cell)."""
    from paper_1004_1122_amd import lshom
    base = []
    for i in range(3):
        m = ms.grf_two_phase(45, 0.12, 0.4, 50.0 * (i + 1), seed=1300 + i)
        base.append(dict(phase=m.phase, cond=[1.0, 50.0 * (i + 1)], E=(1.0, 0.5), tol=1e-9, want_field=True))
    bs = lshom.BatchSolver()
    for cell in (None, (1.0, 3.0)):
        probs = [dict(p, cell=cell) for p in base]
        bs.prepare(probs, precision=0)
        fields, leff, infos = bs.run(precision=0, graph_block=4)
        for i, pr in enumerate(probs):
            s = lshom.Solver(pr["phase"], pr["cond"], cell=cell)
            e, l1, info = s.solve(pr["E"], tol=pr["tol"], graph_block=4)
            assert infos[i]["iterations"] == info["iterations"], (cell, i)
            assert torch.equal(fields[i], e), (cell, i)
            lam = ms.lam_field(pr["phase"], pr["cond"])
            med = o.Medium(lam, cell=cell)
            ref = o.cg(med, o.optimal_reference(med), pr["E"], n_iter=infos[i]["iterations"])
            assert _rel(fields[i].cpu().numpy(), ref["e"]) < 1e-10, (cell, i)
