"""Parity of the HIP solver (through the C ABI) with the CPU FP64 oracle.

FP64 bar: relative L2 field error <= 1e-10 and |dL_eff| / |L_eff| <= 1e-10 at
an equal iteration count (the oracle is rerun for exactly the GPU's count).
"""

import math

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


def _solver(phase, cond):
    from paper_1004_1122_amd import lshom
    return lshom.Solver(np.ascontiguousarray(phase, dtype=np.uint8), cond)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _random_phases(shape, n_phases, seed, lo=1.0, hi=50.0):
    rng = np.random.default_rng(seed)
    phase = rng.integers(0, n_phases, size=shape).astype(np.uint8)
    cond = rng.uniform(lo, hi, size=n_phases)
    return phase, cond


# ---------------------------------------------------------------------------
# One operator apply on arbitrary real fields
# ---------------------------------------------------------------------------

APPLY_SHAPES = [(63, 63), (81, 81), (45, 27), (27, 45), (7, 5), (16, 12), (10, 14), (729, 729),
                (15, 15, 15), (9, 15, 21), (8, 6, 10), (27, 27, 27), (5, 7, 3),
                # prime factors 11, 13, 17 (the paper's 255 = 3 5 17 grid)
                (255, 255), (33, 39), (17, 26), (13, 11, 17), (34, 22, 12)]


@pytest.mark.parametrize("shape", APPLY_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_apply_matches_oracle(shape):
    phase, cond = _random_phases(shape, 4, seed=sum(shape))
    s = _solver(phase, cond)
    l0 = 0.37 * float(cond.max() + cond.min())
    s.set_reference(l0)
    rng = np.random.default_rng(7)
    p = rng.standard_normal((len(shape),) + shape)
    q = s.apply(torch.from_numpy(p)).cpu().numpy()
    ref = o.apply_A(p, ms.lam_field(phase, cond), l0)
    err = np.abs(q - ref).max() / np.abs(ref).max()
    assert err < 1e-13, err


# ---------------------------------------------------------------------------
# CG solves at an equal iteration count
# ---------------------------------------------------------------------------

def _parity_case(m, E, tol, l0=None, **kw):
    s = _solver(m.phase, m.cond)
    lam = m.lam()
    if l0 is not None:
        s.set_reference(l0)
    else:
        l0 = o.optimal_reference(lam)
    e, leff, info = s.solve(E, tol=tol, **kw)
    ref = o.cg(lam, l0, E, n_iter=info["iterations"])
    e_np = e.cpu().numpy()
    return s, lam, l0, e_np, leff, info, ref


def _assert_parity(e, leff, info, ref, lam, field_tol=1e-10):
    assert info["status"] == 0
    err = _rel(e, ref["e"])
    assert err < field_tol, err
    Lref = o.leff(lam, ref["e"])
    assert np.abs(leff - Lref).max() <= 1e-10 * np.abs(Lref).max()
    # recursive residual norms agree as well
    assert abs(info["rel_res"] - ref["rel_res"]) <= 1e-6 * ref["rel_res"] + 1e-15


def test_square_inclusion_63():
    m = ms.square_inclusion()
    s, lam, l0, e, leff, info, ref = _parity_case(m, [1.0, 0.0], 1e-8, l0=5.5)
    _assert_parity(e, leff, info, ref, lam)
    full = o.cg(lam, 5.5, [1.0, 0.0], tol=1e-8)
    assert info["iterations"] == full["iterations"] == 21
    assert info["rel_res_true"] <= 1.01e-8
    assert abs(info["eta_r"] - 5.5 * info["rel_res"]) < 1e-15


@pytest.mark.parametrize("n,rho,tol", [(81, 1e3, 1e-6), (243, 1e2, 1e-6), (81, 1e4, 1e-7)])
def test_grf_2d(n, rho, tol):
    m = ms.grf_two_phase(n, 0.1, 0.4, rho, seed=11 + n)
    s, lam, l0, e, leff, info, ref = _parity_case(m, [0.6, -0.8], tol)
    _assert_parity(e, leff, info, ref, lam)
    full = o.cg(lam, l0, [0.6, -0.8], tol=tol)
    assert abs(info["iterations"] - full["iterations"]) <= 1


def test_non_square_and_even_grids():
    for shape in [(45, 27), (27, 45), (16, 24)]:
        phase, cond = _random_phases(shape, 3, seed=shape[0])
        m = ms.Microstructure(phase, cond)
        s, lam, l0, e, leff, info, ref = _parity_case(m, [1.0, 0.5], 1e-9)
        _assert_parity(e, leff, info, ref, lam)


@pytest.mark.parametrize("shape,rho", [((15, 15, 15), 10.0), ((27, 27, 27), 1e3), ((9, 15, 21), 100.0),
                                       ((12, 10, 8), 50.0)])
def test_3d(shape, rho):
    phase = ms.rsa_inclusions(shape[0], 3, 5, 0.1, 0.2, seed=3, rho=rho).phase
    if phase.shape != shape:
        rng = np.random.default_rng(5)
        phase = (rng.random(shape) < 0.3).astype(np.uint8)
    m = ms.Microstructure(phase, np.array([1.0, rho]))
    s, lam, l0, e, leff, info, ref = _parity_case(m, [0.3, -1.0, 0.5], 1e-7)
    _assert_parity(e, leff, info, ref, lam)


@pytest.mark.parametrize("rho", [10.0, 1e3])
def test_paper_circle_array_255(rho):
    """The workload of Sec. 3 at its own grid (255 = 3 5 17: radix-17 stages)."""
    m = ms.circle_array(n=255, vf=0.5, rho=rho)
    s, lam, l0, e, leff, info, ref = _parity_case(m, [1.0, 0.0], 1e-8)
    _assert_parity(e, leff, info, ref, lam)


def test_wide_prime_grids_3d():
    phase, cond = _random_phases((13, 11, 17), 3, seed=17)
    m = ms.Microstructure(phase, cond)
    s, lam, l0, e, leff, info, ref = _parity_case(m, [0.2, 1.0, -0.4], 1e-9)
    _assert_parity(e, leff, info, ref, lam)


def test_full_size_729_low_contrast():
    m = ms.circles_729(2, rho=10.0)
    s, lam, l0, e, leff, info, ref = _parity_case(m, [1.0, 0.0], 1e-6)
    _assert_parity(e, leff, info, ref, lam)
    assert 10 <= info["iterations"] <= 25


def test_homogenize_square_symmetric():
    m = ms.square_inclusion()
    s = _solver(m.phase, m.cond)
    s.set_reference(5.5)
    L, infos = s.homogenize(tol=1e-10)
    Lref, _ = o.homogenize(m.lam(), 5.5, tol=1e-10)
    assert np.abs(L - Lref).max() < 1e-9
    assert abs(L[0, 1]) < 1e-12 and abs(L[0, 0] - L[1, 1]) < 1e-10
    assert all(i["status"] == 0 for i in infos)


# ---------------------------------------------------------------------------
# Closed forms and degenerate cases
# ---------------------------------------------------------------------------

def test_laminate_one_iteration():
    layers = (np.arange(27) % 3 == 0).astype(np.uint8)
    phase = ms.laminate((27, 27), layers)
    s = _solver(phase, [1.0, 100.0])
    e, leff, info = s.solve([1.0, 0.0], tol=1e-12)
    lam = ms.lam_field(phase, [1.0, 100.0])
    harmonic = 1.0 / np.mean(1.0 / lam)
    assert info["iterations"] == 1
    assert abs(leff[0] - harmonic) < 1e-12 * harmonic
    e, leff, info = s.solve([0.0, 1.0], tol=1e-12)
    assert info["iterations"] == 0 and abs(leff[1] - lam.mean()) < 1e-13 * lam.mean()


def test_homogeneous_medium_exact():
    phase = np.zeros((21, 15, 9), dtype=np.uint8)
    s = _solver(phase, [2.5])
    e, leff, info = s.solve([1.0, 2.0, -1.0], tol=1e-12)
    assert info["iterations"] == 0
    E = np.array([1.0, 2.0, -1.0]).reshape(3, 1, 1, 1)
    assert np.abs(e.cpu().numpy() - E).max() == 0.0
    np.testing.assert_allclose(leff, 2.5 * E.ravel(), rtol=1e-15)


def test_zero_load():
    m = ms.square_inclusion()
    s = _solver(m.phase, m.cond)
    e, leff, info = s.solve([0.0, 0.0], tol=1e-8)
    assert info["iterations"] == 0 and not torch.any(e != 0) and not np.any(leff)


def test_not_converged_returns_iterate():
    from paper_1004_1122_amd import lshom
    m = ms.square_inclusion()
    s = _solver(m.phase, m.cond)
    s.set_reference(5.5)
    with pytest.raises(lshom.LshomError) as ex:
        s.solve([1.0, 0.0], tol=1e-8, max_iter=3)
    assert ex.value.status == lshom.LSHOM_ERR_NOT_CONVERGED
    e, leff, info = s.solve([1.0, 0.0], tol=1e-8, max_iter=3, allow_fail=True)
    assert info["status"] == lshom.LSHOM_ERR_NOT_CONVERGED and info["iterations"] == 3
    ref = o.cg(m.lam(), 5.5, [1.0, 0.0], n_iter=3)
    assert _rel(e.cpu().numpy(), ref["e"]) < 1e-12


def test_warm_start_from_solution_and_garbage():
    m = ms.grf_two_phase(81, 0.1, 0.4, 100.0, seed=4)
    lam = m.lam()
    l0 = o.optimal_reference(lam)
    s = _solver(m.phase, m.cond)
    cold_e, cold_l, cold = s.solve([1.0, 0.0], tol=1e-8)
    ref = o.cg(lam, l0, [1.0, 0.0], tol=1e-12)
    # from (nearly) the solution: accepted, almost no iterations
    e, leff, info = s.solve([1.0, 0.0], tol=1e-8, x0=torch.from_numpy(ref["e"]))
    assert info["warm_start_used"] == 1 and info["iterations"] <= 1
    assert _rel(e.cpu().numpy(), ref["e"]) < 1e-7
    # garbage is rejected and the cold answer comes back bit for bit
    bad = torch.full((2, 81, 81), float("nan"), dtype=torch.float64)
    e2, l2, info2 = s.solve([1.0, 0.0], tol=1e-8, x0=bad)
    assert info2["warm_start_used"] == 0 and info2["iterations"] == cold["iterations"]
    assert torch.equal(e2, cold_e)
    # a perturbed start keeps the answer within the a-posteriori bound
    x0 = torch.from_numpy(ref["e"] + 0.01 * np.random.default_rng(1).standard_normal(ref["e"].shape))
    e3, l3, info3 = s.solve([1.0, 0.0], tol=1e-8, x0=x0)
    bound = (l0 / lam.min()) * 1e-8 * 2
    assert _rel(e3.cpu().numpy(), ref["e"]) < bound


def test_deterministic_and_graph_equals_eager():
    m = ms.grf_two_phase(243, 0.08, 0.5, 1e3, seed=9)
    s = _solver(m.phase, m.cond)
    a, la, ia = s.solve([1.0, 0.0], tol=1e-6)
    b, lb, ib = s.solve([1.0, 0.0], tol=1e-6)
    c, lc, ic = s.solve([1.0, 0.0], tol=1e-6, graph_block=0)
    d_, ld, id_ = s.solve([1.0, 0.0], tol=1e-6, graph_block=5)
    assert torch.equal(a, b) and torch.equal(a, c) and torch.equal(a, d_)
    assert ia["iterations"] == ib["iterations"] == ic["iterations"] == id_["iterations"]


def test_reference_invariance():
    m = ms.square_inclusion()
    s = _solver(m.phase, m.cond)
    fields = []
    for l0 in (2.0, 5.5, 20.0):
        s.set_reference(l0)
        e, leff, info = s.solve([1.0, 0.0], tol=0.0, max_iter=12, allow_fail=True)
        fields.append(e.cpu().numpy())
    for f in fields[1:]:
        assert _rel(f, fields[0]) < 1e-9


def test_call_order_errors():
    from paper_1004_1122_amd import lshom
    import ctypes
    lib = lshom.load()
    ctx = lshom.lshom_create(0, None)
    try:
        E = (ctypes.c_double * 2)(1.0, 0.0)
        assert lib.lshom_solve(ctx, E, 1e-6, None, None, None, None, None) == lshom.LSHOM_ERR_STATE
        assert lib.lshom_set_reference(ctx, 1.0) == lshom.LSHOM_ERR_STATE
        phase = torch.zeros((9, 9), dtype=torch.uint8, device="cuda")
        N = (ctypes.c_int64 * 2)(9, 9)
        cond = (ctypes.c_double * 1)(1.0)
        assert lib.lshom_set_microstructure(ctx, 2, N, ctypes.c_void_p(phase.data_ptr()), 1, cond) == 0
        assert lib.lshom_solve(ctx, E, 1e-6, None, None, None, None, None) == lshom.LSHOM_ERR_WORKSPACE
        assert lib.lshom_set_reference(ctx, -1.0) == lshom.LSHOM_ERR_INVALID_ARG
        assert lib.lshom_set_reference(ctx, float("nan")) == lshom.LSHOM_ERR_INVALID_ARG
        assert lib.lshom_set_workspace(ctx, ctypes.c_void_p(phase.data_ptr()), 16) == lshom.LSHOM_ERR_WORKSPACE
        assert b"workspace" in lib.lshom_last_error(ctx)
    finally:
        lshom.lshom_destroy(ctx)


def test_out_of_range_phase_is_loud():
    from paper_1004_1122_amd import lshom
    phase = np.zeros((27, 27), dtype=np.uint8)
    phase[3, 3] = 5                       # only 2 phases declared
    with pytest.raises(lshom.LshomError) as ex:
        _solver(phase, [1.0, 3.0])        # rejected when the workspace is attached
    assert ex.value.status == lshom.LSHOM_ERR_INVALID_ARG and "n_phases" in str(ex.value)


# ---------------------------------------------------------------------------
# Mixed precision (FP32 operator and vectors, FP64 dots and refreshes)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,rho", [((243, 243), 1e4), ((81, 81), 1e2), ((27, 27, 27), 1e3),
                                       ((45, 27), 10.0)])
def test_mixed_matches_converged_oracle(shape, rho):
    """R18 bar: stop when the FP64 true residual <= 1e-6 lambda_min / l0, then
    the field is within 1e-6 of the exact discrete solution."""
    rng = np.random.default_rng(21)
    if len(shape) == 2 and shape[0] == shape[1]:
        m = ms.grf_two_phase(shape[0], 0.1, 0.4, rho, seed=21)
        phase = m.phase
    else:
        phase = (rng.random(shape) < 0.35).astype(np.uint8)
    cond = [1.0, rho]
    lam = ms.lam_field(phase, cond)
    l0 = o.optimal_reference(lam)
    tol = 1e-6 * lam.min() / l0
    s = _solver(phase, cond)
    E = [1.0, -0.5, 0.25][:len(shape)]
    e, leff, info = s.solve(E, tol=tol, precision=1)
    assert info["status"] == 0 and info["refreshes"] >= 1 and info["applies_fp32"] == info["iterations"]
    assert info["rel_res_true"] <= tol * 1.0001
    exact = o.cg(lam, l0, E, tol=1e-13, max_iter=20000)
    err = _rel(e.cpu().numpy(), exact["e"])
    assert err <= 1e-6, err
    Lx = o.leff(lam, exact["e"])
    assert np.abs(leff - Lx).max() <= 1e-6 * np.abs(Lx).max()
    # the FP64 refreshes keep the iteration count close to plain FP64 CG
    e64, l64, i64 = s.solve(E, tol=tol)
    assert info["iterations"] <= 1.25 * i64["iterations"] + 5


def test_mixed_reports_and_limits():
    from paper_1004_1122_amd import lshom
    m = ms.square_inclusion()
    s = _solver(m.phase, m.cond)
    e, leff, info = s.solve([1.0, 0.0], tol=1e-6, precision=1, refresh_every=5)
    assert info["refreshes"] >= info["iterations"] // 5
    e, leff, info = s.solve([1.0, 0.0], tol=1e-9, precision=1, max_iter=4, allow_fail=True)
    assert info["status"] == lshom.LSHOM_ERR_NOT_CONVERGED and info["iterations"] == 4
    e, leff, info = s.solve([0.0, 0.0], tol=1e-6, precision=1)
    assert info["iterations"] == 0
    homog = _solver(np.zeros((9, 9, 9), np.uint8), [3.0])
    e, leff, info = homog.solve([1.0, 1.0, 1.0], tol=1e-10, precision=1)
    assert info["iterations"] == 0 and np.allclose(leff, 3.0, rtol=1e-15)


@pytest.mark.parametrize("precision", [0, 1])
def test_solver_reuse_across_load_cases(precision):
    """Solves with different E on one context (cached iteration graphs) equal
    solves on fresh contexts bit for bit."""
    from paper_1004_1122_amd import lshom
    m = ms.grf_two_phase(81, 0.1, 0.4, 1e3, seed=77)
    loads = [(1.0, 0.0), (0.0, 1.0), (0.6, -0.8), (1.0, 0.0)]
    s = lshom.Solver(m.phase, m.cond)
    for E in loads:
        e1, l1, i1 = s.solve(E, tol=1e-8, precision=precision)
        f = lshom.Solver(m.phase, m.cond)
        e2, l2, i2 = f.solve(E, tol=1e-8, precision=precision)
        assert i1["iterations"] == i2["iterations"] and i1["status"] == 0
        assert torch.equal(e1, e2) and np.array_equal(l1, l2)
    t, infos = s.homogenize(tol=1e-8, precision=precision)
    for b in range(2):
        E = (1.0, 0.0) if b == 0 else (0.0, 1.0)
        _, l, _ = lshom.Solver(m.phase, m.cond).solve(E, tol=1e-8, precision=precision)
        assert np.array_equal(t[:, b], l)


@pytest.mark.parametrize("shape", [(1331, 1331), (1600, 1600), (1728, 1728), (975, 9, 9), (1377, 9, 9), (1024, 9, 9)],
                         ids=["1331^2", "1600^2", "1728^2", "975x9x9", "1377x9x9", "1024x9x9"])
def test_set_up_agrees_with_host_check(shape):
    """The device set-up accepts exactly the grids the host-only check accepts
    (the LDS fit of the pass kernels bounds the axis lengths)."""
    from paper_1004_1122_amd import lshom
    want = lshom.lshom_check_problem(len(shape), shape, [1.0, 10.0])
    phase = np.zeros(shape, np.uint8)
    phase.flat[::7] = 1
    if want == 0:
        s = lshom.Solver(phase, [1.0, 10.0])
        e, _, info = s.solve((1.0,) + (0.0,) * (len(shape) - 1), tol=1e-3)
        assert info["status"] == 0 and bool(torch.isfinite(e).all())
    else:
        assert want == lshom.LSHOM_ERR_UNSUPPORTED
        with pytest.raises(lshom.LshomError) as ex:
            lshom.Solver(phase, [1.0, 10.0])
        assert ex.value.status == lshom.LSHOM_ERR_UNSUPPORTED
