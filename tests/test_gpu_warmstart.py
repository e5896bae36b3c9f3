"""The trained warm-start network (paper_1004_1122_amd/weights) on held-out
problems: the converged answer stays within the a-posteriori bound of the
cold start, and the mean iteration count drops at the training scale."""

import os

import numpy as np
import pytest

from paper_1004_1122_amd import microstructure as ms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def net():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1004_1122_amd import cnn
    if not os.path.exists(cnn.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    return cnn.WarmStartNet.load(cnn.DEFAULT_WEIGHTS)


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_start_held_out_243(net, precision):
    from paper_1004_1122_amd import lshom
    saved = []
    for i in range(8):
        m = ms.warmstart_eval_problem(i, 243)
        s = lshom.Solver(m.phase, m.cond)
        tol = 1e-6
        e_c, l_c, i_c = s.solve((1.0, 0.0), tol=tol, precision=precision)
        x0 = net.forward(m.phase, m.info["log10_rho"])[0]
        e_w, l_w, i_w = s.solve((1.0, 0.0), tol=tol, precision=precision, x0=x0)
        assert i_c["status"] == 0 and i_w["status"] == 0
        assert i_w["rel_res_true"] <= tol * 1.01
        # both are within (l0 / lambda_min) tol of the exact solution
        bound = 2.0 * (0.5 * (1.0 + m.info["rho"])) * tol
        err = float((e_w - e_c).norm() / e_c.norm())
        assert err <= bound, (i, err, bound)
        # |<lambda de>| <= lambda_max ||de||_rms
        rms = float(e_c.norm()) / np.sqrt(e_c.numel() / 2)
        assert np.abs(l_w - l_c).max() <= m.info["rho"] * err * rms * 1.0001 + 1e-15
        saved.append(i_c["iterations"] - i_w["iterations"])
    print("iterations saved per problem:", saved)
    assert np.mean(saved) > 0, saved


def test_warm_start_load_case_e2(net):
    """The e2 prediction (transposed image) is used and gives the same answer."""
    from paper_1004_1122_amd import lshom
    m = ms.warmstart_eval_problem(3, 243)
    s = lshom.Solver(m.phase, m.cond)
    e_c, l_c, i_c = s.solve((0.0, 1.0), tol=1e-6)
    x0 = net.forward(m.phase, m.info["log10_rho"], load_axis=1)[0]
    e_w, l_w, i_w = s.solve((0.0, 1.0), tol=1e-6, x0=x0)
    assert i_w["warm_start_used"] == 1 and i_w["status"] == 0
    bound = 2.0 * (0.5 * (1.0 + m.info["rho"])) * 1e-6
    assert float((e_w - e_c).norm() / e_c.norm()) <= bound
