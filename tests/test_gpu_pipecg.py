"""Pipelined CG on the GPU (one reduction per iteration: (r, r) and (w, r)
from the update pass; w = A r, s = A p, z = A s carried as spectral vectors),
through the C ABI, against the oracle's pipelined CG and against CG.

FP64 bars: fields within 1e-10 of the oracle's pipelined CG at an equal
iteration count; stopping iteration within one of the oracle's; the iterates
of the GPU's CG within 1e-9 at equal counts (the same Krylov iterates).
"""

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


def _cases():
    rng = np.random.default_rng(8)
    return [("square63_rho10", ms.square_inclusion(rho=10.0).phase, [1.0, 10.0], (1.0, 0.0)),
            ("grf45_rho100", ms.grf_two_phase(45, 0.15, 0.4, 100.0, seed=12).phase, [1.0, 100.0], (0.6, -0.8)),
            ("rand16x12_3ph", rng.integers(0, 3, (16, 12)).astype(np.uint8), [1.0, 4.0, 20.0], (1.0, 1.0)),
            ("cube15_rho20", (rng.random((15, 15, 15)) < 0.3).astype(np.uint8), [1.0, 20.0], (0.0, 1.0, 0.5)),
            ("box18x10x12_rho50", (rng.random((18, 10, 12)) < 0.4).astype(np.uint8), [1.0, 50.0], (1.0, 0.0, 0.0))]


CASES = _cases()
IDS = [c[0] for c in CASES]


def _solver(phase, cond):
    from paper_1004_1122_amd import lshom
    return lshom.Solver(np.ascontiguousarray(phase, dtype=np.uint8), cond)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_pipecg_matches_oracle(case):
    from paper_1004_1122_amd import lshom
    _, phase, cond, E = case
    lam = ms.lam_field(phase, cond)
    l0 = o.optimal_reference(lam)
    s = _solver(phase, cond)
    e, leff, info = s.solve(E, tol=1e-8, method=lshom.METHOD_PIPECG)
    assert info["status"] == 0
    ref = o.pipelined_cg(lam, l0, E, n_iter=info["iterations"])
    assert _rel(e.cpu().numpy(), ref["e"]) < 1e-10
    full = o.pipelined_cg(lam, l0, E, tol=1e-8)
    assert abs(info["iterations"] - full["iterations"]) <= 1
    lref = o.leff(lam, ref["e"])
    np.testing.assert_allclose(leff, lref, rtol=1e-10, atol=1e-12 * np.abs(lref).max())
    assert info["rel_res"] <= 1e-8 and info["rel_res_true"] <= 1.5e-8
    assert abs(info["rel_res_true"] - o.true_residual(lam, l0, E, e.cpu().numpy())) <= 1e-3 * info["rel_res_true"]


@pytest.mark.parametrize("case", CASES[:2] + CASES[3:4], ids=IDS[:2] + IDS[3:4])
def test_pipecg_iterates_equal_cg(case):
    from paper_1004_1122_amd import lshom
    _, phase, cond, E = case
    s = _solver(phase, cond)
    for k in (1, 3, 8):
        e_cg, _, _ = s.solve(E, tol=0.0, max_iter=k, allow_fail=True)
        e_pc, _, info = s.solve(E, tol=0.0, max_iter=k, allow_fail=True, method=lshom.METHOD_PIPECG)
        assert info["iterations"] == k and info["status"] == lshom.LSHOM_ERR_NOT_CONVERGED
        assert _rel(e_pc.cpu().numpy(), e_cg.cpu().numpy()) < 1e-9, k
    _, _, i_cg = s.solve(E, tol=1e-8)
    _, _, i_pc = s.solve(E, tol=1e-8, method=lshom.METHOD_PIPECG)
    assert abs(i_cg["iterations"] - i_pc["iterations"]) <= 1


def test_pipecg_graph_equals_eager_and_options():
    from paper_1004_1122_amd import lshom
    _, phase, cond, E = CASES[1]
    s = _solver(phase, cond)
    a, _, ia = s.solve(E, tol=1e-9, method=lshom.METHOD_PIPECG)
    b, _, ib = s.solve(E, tol=1e-9, method=lshom.METHOD_PIPECG, graph_block=0)
    c, _, ic = s.solve(E, tol=1e-9, method=lshom.METHOD_PIPECG, graph_block=3)
    assert ia["iterations"] == ib["iterations"] == ic["iterations"]
    assert torch.equal(a, b) and torch.equal(a, c)
    z, lz, iz = s.solve((0.0, 0.0), tol=1e-9, method=lshom.METHOD_PIPECG)
    assert iz["iterations"] == 0 and float(z.abs().max()) == 0.0
    for kw, status in ((dict(precision=1), lshom.LSHOM_ERR_UNSUPPORTED),
                       (dict(norm=lshom.NORM_EQUILIBRIUM), lshom.LSHOM_ERR_UNSUPPORTED),
                       (dict(x0=torch.zeros((2, 45, 45), dtype=torch.float64)), lshom.LSHOM_ERR_UNSUPPORTED)):
        with pytest.raises(lshom.LshomError) as ex:
            s.solve(E, tol=1e-6, method=lshom.METHOD_PIPECG, **kw)
        assert ex.value.status == status
    bs = lshom.BatchSolver()
    bs.prepare([dict(phase=phase, cond=cond, E=E, tol=1e-6)], precision=0)
    with pytest.raises(lshom.LshomError) as ex:
        bs.run(method=lshom.METHOD_PIPECG)
    assert ex.value.status == lshom.LSHOM_ERR_UNSUPPORTED
    # CG still runs on the grown workspace
    _, _, icg = s.solve(E, tol=1e-9, precision=1)
    assert icg["status"] == 0


def test_pipecg_not_converged_and_general_reference():
    from paper_1004_1122_amd import lshom
    _, phase, cond, E = CASES[1]
    lam = ms.lam_field(phase, cond)
    s = _solver(phase, cond)
    e, _, info = s.solve(E, tol=1e-12, max_iter=5, method=lshom.METHOD_PIPECG, allow_fail=True)
    assert info["status"] == lshom.LSHOM_ERR_NOT_CONVERGED and info["iterations"] == 5
    ref = o.pipelined_cg(lam, o.optimal_reference(lam), E, n_iter=5)
    assert _rel(e.cpu().numpy(), ref["e"]) < 1e-10
    # an anisotropic reference: energy products of L0, as CG
    L0 = np.array([[60.0, 12.0], [12.0, 35.0]])
    s.set_reference(L0)
    e, _, info = s.solve(E, tol=1e-9, method=lshom.METHOD_PIPECG)
    assert info["status"] == 0
    ref = o.pipelined_cg(lam, L0, E, n_iter=info["iterations"])
    assert _rel(e.cpu().numpy(), ref["e"]) < 1e-10
    assert abs(info["iterations"] - o.cg(lam, L0, E, tol=1e-9)["iterations"]) <= 1
