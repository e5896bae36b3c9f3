"""Seeded input generators: determinism and the stated geometric facts."""

import numpy as np

from paper_1004_1122_amd import microstructure as ms


def test_square_inclusion_nodes():
    m = ms.square_inclusion()
    assert m.phase.shape == (63, 63) and m.phase.dtype == np.uint8
    assert int(m.phase.sum()) == 961
    assert m.phase[31, 31] == 1 and m.phase[16, 16] == 1 and m.phase[15, 16] == 0
    np.testing.assert_array_equal(m.phase, m.phase.T)
    np.testing.assert_array_equal(m.phase, m.phase[::-1, :])


def test_rsa_deterministic_and_non_overlapping():
    a = ms.rsa_inclusions(81, 2, 12, 0.02, 0.06, seed=7)
    b = ms.rsa_inclusions(81, 2, 12, 0.02, 0.06, seed=7)
    np.testing.assert_array_equal(a.phase, b.phase)
    c, r = a.info["centres"], a.info["radii"]
    for i in range(len(r)):
        for j in range(i):
            diff = np.abs(c[i] - c[j])
            diff = np.minimum(diff, 1 - diff)
            assert np.sqrt((diff ** 2).sum()) >= r[i] + r[j]
    assert r.min() >= 0.02 and r.max() <= 0.06 and len(r) == 12


def test_rsa_rasterisation_periodic():
    m = ms.rsa_inclusions(31, 3, 3, 0.1, 0.15, seed=1)
    # every centre node is inside its own ball
    for c in m.info["centres"]:
        j = tuple(int(round(v * 31)) % 31 for v in c)
        assert m.phase[j] == 1


def test_workload_geometries():
    c2 = ms.circles_729(2)
    assert c2.phase.shape == (729, 729) and c2.info["count"] == 40
    assert 0.1 < c2.info["vf"] < 0.35


def test_grf_exact_volume_fraction():
    m = ms.grf_two_phase(81, 0.1, 0.37, 100.0, seed=3)
    assert int(m.phase.sum()) == int(round(0.37 * 81 * 81))


def test_batched_problem_draws():
    sizes = [ms.batched_problem(i).info["n"] for i in range(24)]
    assert set(sizes) <= {81, 243, 729} and len(set(sizes)) == 3
    p = ms.batched_problem(5)
    q = ms.batched_problem(5)
    np.testing.assert_array_equal(p.phase, q.phase)
    assert 1.0 <= p.info["log10_rho"] <= 4.0 and 0.05 <= p.info["ell"] <= 0.2
    assert abs(p.info["vf"] - p.info["vf_target"]) <= 1.0 / p.phase.size


def test_warmstart_problems_forced_sizes():
    assert ms.warmstart_train_problem(0).phase.shape == (81, 81)
    assert ms.warmstart_train_problem(1).phase.shape == (243, 243)
    assert ms.warmstart_eval_problem(0, 243).phase.shape == (243, 243)
    # the forced size does not change the remaining draws
    a = ms._grf_problem_fixed_draw(123, None)
    b = ms._grf_problem_fixed_draw(123, a.info["n"])
    np.testing.assert_array_equal(a.phase, b.phase)
