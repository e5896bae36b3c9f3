"""Warm-start network on the GPU (through the C ABI of include/lshom_cnn.h)
against the CPU oracle of oracle/cnn_oracle.py.

The GPU stores weights and activations in bfloat16 and accumulates in FP32.
The oracle is run on the same bfloat16-rounded weights and input, rounding
every stored activation to bfloat16 and every pre-activation gradient (the
operand of the gradient products) to bfloat16 at the same points as the GPU.
Each operation on identical operands agrees to about 1e-7 of the sum of
the magnitudes of its terms (tests/test_gpu_cnn_ops.py); through the whole
network the two differ where an FP32 and an FP64 sum round to different
bfloat16 values (one unit in the last place, 2^-8 relative), and such flips
propagate: the forward output agrees to about 1e-4 and the gradients to
about 5e-3 (relative L2), hence the network-level bars of 1e-3 and 1.5e-2.
"""

import numpy as np
import pytest

from oracle import cnn_oracle as co
from paper_1004_1122_amd import microstructure as ms

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


C0 = 8


def _setup(N=27, B=2, seed=0):
    from paper_1004_1122_amd import cnn
    rng = np.random.default_rng(seed)
    params = co.init_params(C0, seed=seed)
    for name in params:
        params[name][1] = rng.standard_normal(params[name][1].shape) * 0.05
    vec = cnn.pack(params, C0)
    # what the GPU computes with: bf16 weights, FP32 biases
    used = cnn.unpack(vec, C0)
    for name in used:
        used[name][0] = co.bf16(used[name][0])
    phase = (rng.random((B, N, N)) < 0.4).astype(np.uint8)
    lrho = rng.uniform(1.0, 4.0, size=B).astype(np.float32)
    x = np.stack([phase.astype(np.float64), np.broadcast_to(co.bf16(lrho * np.float32(0.25))[:, None, None],
                                                            phase.shape)], axis=-1)
    net = cnn.WarmStartNet(C0, params=vec)
    return net, used, phase, lrho, x


def _oracle_out(used, x):
    y, acts = co.forward(used, x, C0, round_act=co.bf16)
    w, b = used["head"]
    return co.conv1(acts["dec0b"], w, b), acts


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("N,B", [(27, 2), (81, 1)])
def test_forward_matches_oracle(N, B):
    net, used, phase, lrho, x = _setup(N, B)
    e, raw = net.forward(phase, lrho, want_raw=True)
    ref, _ = _oracle_out(used, x)
    got = raw.cpu().numpy().astype(np.float64)
    print(f"forward N={N} B={B}: rel-L2 {_rel(got, ref):.3e}", flush=True)
    assert _rel(got, ref) < 1e-3, _rel(got, ref)
    # the field output is E + prediction, planar
    ef = e.cpu().numpy()
    np.testing.assert_allclose(ef[:, 0], 1.0 + got[..., 0], rtol=0, atol=1e-7)
    np.testing.assert_allclose(ef[:, 1], got[..., 1], rtol=0, atol=1e-7)


def test_transposed_load_case():
    net, used, phase, lrho, x = _setup(27, 2, seed=3)
    e2 = net.forward(phase, lrho, load_axis=1).cpu().numpy()
    e1t = net.forward(np.ascontiguousarray(np.swapaxes(phase, 1, 2)), lrho, load_axis=0).cpu().numpy()
    # e^(I, e2)_1(x1, x2) = e^(I^T, e1)_2(x2, x1), e^(I, e2)_2 = e^(I^T, e1)_1 (transposed), E = e2
    np.testing.assert_array_equal(e2[:, 0], np.swapaxes(e1t[:, 1], 1, 2))
    np.testing.assert_array_equal(e2[:, 1], np.swapaxes(e1t[:, 0], 1, 2))


def test_gradients_match_oracle():
    net, used, phase, lrho, x = _setup(27, 2, seed=1)
    rng = np.random.default_rng(9)
    tgt = rng.standard_normal((2, 2, 27, 27)) * 0.3
    tgt[:, 0] += 1.0  # fields around E = e1
    loss = net.train_step(phase, lrho, torch.from_numpy(tgt), update=False)
    g = net.get_grads()
    from paper_1004_1122_amd import cnn
    gg = cnn.unpack(g, C0)
    y, acts = _oracle_out(used, x)
    t = np.moveaxis(tgt - np.array([1.0, 0.0])[None, :, None, None], 1, -1)
    ref_loss, gy = co.rel_mse(y, t)
    assert loss == pytest.approx(ref_loss, rel=1e-3)
    ref = co.backward(used, acts, gy, C0, round_grad=co.bf16)
    worst = 0.0
    for name in used:
        for k in (0, 1):
            err = _rel(gg[name][k], ref[name][k])
            worst = max(worst, err)
            assert err < 1.5e-2, (name, k, err)
    print(f"gradients: worst rel-L2 {worst:.3e}", flush=True)


def test_adam_step_matches_oracle():
    net, used, phase, lrho, x = _setup(27, 2, seed=2)
    rng = np.random.default_rng(4)
    tgt = rng.standard_normal((2, 2, 27, 27))
    before = net.get_params().astype(np.float64)
    net.train_step(phase, lrho, torch.from_numpy(tgt), lr=1e-3, update=True)
    after = net.get_params().astype(np.float64)
    g = net.get_grads().astype(np.float64)
    want, _, _ = co.adam_step(before, g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    np.testing.assert_allclose(after, want, rtol=1e-5, atol=1e-7)


def test_training_reduces_loss_on_solved_fields():
    """A few Adam steps on GPU-solved fields lower the loss (overfitting one batch)."""
    from paper_1004_1122_amd import cnn, lshom
    probs = []
    for i in range(4):
        m = ms.grf_two_phase(27, 0.15, 0.4, 30.0, seed=700 + i)
        probs.append(dict(phase=m.phase, cond=m.cond, E=(1.0, 0.0), tol=1e-8, want_field=True))
    bs = lshom.BatchSolver()
    bs.prepare(probs, precision=0)
    fields, _, _ = bs.run(precision=0)
    tgt = torch.stack(fields)
    phase = np.stack([p["phase"] for p in probs])
    net = cnn.WarmStartNet(C0, seed=5)
    lrho = np.full(4, np.log10(30.0), np.float32)
    first = net.train_step(phase, lrho, tgt, lr=3e-3)
    last = first
    for _ in range(60):
        last = net.train_step(phase, lrho, tgt, lr=3e-3)
    assert np.isfinite(first) and last < 0.5 * first, (first, last)


def test_bad_prediction_falls_back_to_cold_start():
    """NaN weights give a NaN prediction: the solver rejects it and returns the
    cold-start answer."""
    from paper_1004_1122_amd import cnn, lshom
    m = ms.grf_two_phase(81, 0.1, 0.4, 1e2, seed=11)
    net = cnn.WarmStartNet(C0, seed=0)
    p = net.get_params()
    p[:] = np.nan
    net.set_params(p)
    e_pred = net.forward(m.phase, np.log10(1e2))
    s = lshom.Solver(m.phase, m.cond)
    e_cold, l_cold, i_cold = s.solve((1.0, 0.0), tol=1e-8)
    e_warm, l_warm, i_warm = s.solve((1.0, 0.0), tol=1e-8, x0=e_pred[0])
    assert i_warm["warm_start_used"] == 0
    assert torch.equal(e_warm, e_cold) and i_warm["iterations"] == i_cold["iterations"]
