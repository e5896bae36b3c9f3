"""Several contexts solving from several host threads at once (each context
has its own stream and captures its own iteration graphs): every result
equals the same solve run alone, bit for bit."""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from paper_1004_1122_amd import microstructure as ms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_concurrent_batches_match_sequential():
    from paper_1004_1122_amd import lshom
    batches = []
    for j in range(4):
        probs = []
        for i, rho in enumerate((10.0, 1e3, 1e2)):
            m = ms.grf_two_phase(81, 0.1, 0.4, rho, seed=900 + 10 * j + i)
            probs.append(dict(phase=m.phase, cond=m.cond, E=(1.0, 0.0) if j % 2 == 0 else (0.0, 1.0), tol=1e-8,
                              want_field=True))
        batches.append(probs)
    precisions = [0, 1, 0, 1]
    solvers = []
    for probs, prec in zip(batches, precisions):
        bs = lshom.BatchSolver()
        bs.prepare(probs, precision=prec)
        solvers.append(bs)
    alone = []
    for bs, prec in zip(solvers, precisions):
        f, l, inf = bs.run(precision=prec)
        alone.append(([x.clone() for x in f], l.copy(), [i["iterations"] for i in inf]))
    with ThreadPoolExecutor(4) as ex:
        for rep in range(3):
            futs = [ex.submit(bs.run, precision=prec) for bs, prec in zip(solvers, precisions)]
            for k, fu in enumerate(futs):
                f, l, inf = fu.result()
                assert [i["iterations"] for i in inf] == alone[k][2], (rep, k)
                assert np.array_equal(l, alone[k][1]), (rep, k)
                for a, b in zip(f, alone[k][0]):
                    assert torch.equal(a, b), (rep, k)
