"""BF16-MFMA MLP kernels (through the C ABI) against the FP64 oracle MLP.

Both sides get identical inputs: weight matrices and features already rounded
to BF16 (round to nearest even), biases in FP32.  The GPU additionally rounds
the two hidden activations and the back-propagated signals to BF16 (unit
round-off 2^-9) while accumulating in FP32, so the bars are 2e-2 of the
largest output for the forward pass and 3e-2 relative L2 for the gradient
(a few BF16 round-offs per layer, three layers).
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

NF, NH, NO = 12, 128, 3
OFF_B1 = NF * NH
OFF_W2 = OFF_B1 + NH
OFF_B2 = OFF_W2 + NH * NH
OFF_W3 = OFF_B2 + NH
OFF_B3 = OFF_W3 + NH * NO


def bf16(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def weights(seed):
    rng = np.random.default_rng(seed)
    w = np.zeros(OFF_B3 + NO, np.float32)
    w[:OFF_B1] = bf16(rng.normal(0, math.sqrt(2 / NF), NF * NH))
    w[OFF_B1:OFF_W2] = rng.normal(0, 0.1, NH)
    w[OFF_W2:OFF_B2] = bf16(rng.normal(0, math.sqrt(2 / NH), NH * NH))
    w[OFF_B2:OFF_W3] = rng.normal(0, 0.1, NH)
    w[OFF_W3:OFF_B3] = bf16(rng.normal(0, math.sqrt(1 / NH), NH * NO))
    w[OFF_B3:] = rng.normal(0, 0.1, NO)
    return w


def _nb():
    import paper_1501_05810_amd as nb

    return nb


@pytest.mark.parametrize("n", [1, 64, 65, 1000, 5003])
def test_forward_matches_oracle(n):
    import torch

    nb = _nb()
    w = weights(1)
    x = bf16(np.random.default_rng(2).normal(size=(n, NF)))
    m = nb.GpuMlp()
    m.set_weights(w)
    y = m.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    ref = oracle.mlp_forward(w.astype(np.float64), x.astype(np.float64))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= 2e-2, err
    m.close()


@pytest.mark.parametrize("n", [1, 63, 300, 4096])
def test_gradient_matches_oracle(n):
    import torch

    nb = _nb()
    w = weights(3)
    rng = np.random.default_rng(4)
    x = bf16(rng.normal(size=(n, NF)))
    t = rng.normal(size=(n, NO)).astype(np.float32)
    m = nb.GpuMlp()
    m.set_weights(w)
    loss, g = m.loss_grad(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"))
    g = g.cpu().numpy()
    rloss, rg = oracle.mlp_loss_grad(w.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    assert loss == pytest.approx(rloss, rel=2e-2)
    for lo, hi, name in ((0, OFF_B1, "W1"), (OFF_B1, OFF_W2, "b1"), (OFF_W2, OFF_B2, "W2"), (OFF_B2, OFF_W3, "b2"),
                         (OFF_W3, OFF_B3, "W3"), (OFF_B3, OFF_B3 + NO, "b3")):
        rel = np.linalg.norm(g[lo:hi] - rg[lo:hi]) / max(np.linalg.norm(rg[lo:hi]), 1e-30)
        assert rel <= 3e-2, (name, rel)
    # deterministic
    loss2, g2 = m.loss_grad(torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda"))
    assert loss2 == loss and np.array_equal(g2.cpu().numpy(), g)
    m.close()


def test_weights_round_trip_and_initialisation():
    nb = _nb()
    m = nb.GpuMlp(seed=7)
    w0 = m.weights()
    assert w0.shape == (18563,) and np.all(w0[OFF_B1:OFF_W2] == 0) and np.abs(w0[:OFF_B1]).max() <= math.sqrt(0.5)
    m2 = nb.GpuMlp(seed=7)
    assert np.array_equal(m2.weights(), w0)
    w = weights(5)
    m.set_weights(w)
    assert np.array_equal(m.weights(), w)
    m.close()
    m2.close()


def test_training_fits_a_smooth_map():
    """Adam on a regression whose exact map is a small function of the inputs: the loss must fall sharply."""
    import torch

    nb = _nb()
    rng = np.random.default_rng(6)
    n = 20000
    x = rng.uniform(-1, 1, size=(n, NF)).astype(np.float32)
    t = np.stack([np.maximum(x[:, 0] + 0.5 * x[:, 1], 0), x[:, 2] * x[:, 3], 0.3 * x[:, 4] - x[:, 5]], 1)
    m = nb.GpuMlp(seed=1)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t.astype(np.float32), device="cuda")
    l0, _ = m.loss_grad(xd, td)
    lfin = m.train(xd, td, epochs=15, batch=512, lr=2e-3, seed=3)
    l1, _ = m.loss_grad(xd, td)
    assert l1 < 0.05 * l0, (l0, lfin, l1)
    m.close()


def test_adam_steps_match_oracle():
    """Three Adam steps of the training kernels against the oracle's Adam (Kingma & Ba) on the same gradient.

    One sample, one batch: the GPU gradient of nbgs_mlp_loss_grad and the one the training loop forms are then the
    same sum (one block, no summation order), so the step can be replayed by the oracle from the GPU's own weights
    and gradient; the oracle keeps its moments in FP64, the GPU in FP32 (a few FP32 round-offs of a move of lr)."""
    import torch

    nb = _nb()
    w0 = weights(8)
    rng = np.random.default_rng(9)
    x = torch.tensor(bf16(rng.normal(size=(1, NF))), device="cuda")
    t = torch.tensor(rng.normal(size=(1, NO)).astype(np.float32), device="cuda")
    m = nb.GpuMlp()
    m.set_weights(w0)
    lr = 1e-3
    wr = w0.astype(np.float64)
    mr, vr = np.zeros_like(wr), np.zeros_like(wr)
    for k in (1, 2, 3):
        _, g = m.loss_grad(x, t)
        g = g.cpu().numpy().astype(np.float64)
        assert np.count_nonzero(g) > 1000
        wprev = m.weights().astype(np.float64)
        m.train(x, t, epochs=1, batch=1, lr=lr, seed=k)
        wg = m.weights().astype(np.float64)
        wr = wprev.copy()
        oracle.mlp_adam(wr, g, mr, vr, k, lr=lr)
        moved = np.abs(wr - wprev)
        assert np.median(moved[g != 0]) > 0.5 * lr  # the steps are not vanishing
        np.testing.assert_allclose(wg, wr, rtol=3e-7, atol=1e-8 * lr / 1e-3)
    m.close()
