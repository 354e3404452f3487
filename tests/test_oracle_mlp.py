"""Pins of the FP64 MLP reference: the analytic backward pass against central
finite differences of its own forward loss (FP64, no rounding), and the
bfloat16 rounding helper against the format's definition."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_rounding_definition():
    # bfloat16 keeps the top 16 bits of a float32, rounding to nearest even
    assert mlp.bf16_round(1.0) == 1.0
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0            # tie -> even (down)
    assert mlp.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)
    assert mlp.bf16_round(1.0 + 2 ** -7) == 1.0 + 2 ** -7   # representable
    assert mlp.bf16_round(-3.0) == -3.0
    assert mlp.bf16_bits(1.0) == 0x3F80
    assert mlp.bf16_bits(-2.0) == 0xC000


def _problem(rng, n_par=7):
    fan = rng.integers(1, 5, n_par)
    seg = np.concatenate([[0], np.cumsum(fan)])
    M = int(seg[-1])
    X = rng.integers(0, 2, (M, mlp.N_IN)).astype(np.float64)
    X[:, 156:167] = rng.normal(0, 0.5, (M, 11))
    tsig = np.concatenate([rng.dirichlet(np.ones(k)) for k in fan])
    tval = rng.normal(0, 3, M)
    return X, seg, tsig, tval


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    W = mlp.init_weights(rng)
    W[1] = rng.normal(0, 0.1, 256)
    W[3] = rng.normal(0, 0.1, 256)
    W[5] = rng.normal(0, 0.1, 2)
    X, seg, tsig, tval = _problem(rng)

    def loss(Wx):
        _, _, Y = mlp.forward(Wx, X, bf16=False)
        return mlp.loss_and_dY(Y, seg, tsig, tval, 0.5)[0]

    H1, H2, Y = mlp.forward(W, X, bf16=False)
    _, dY = mlp.loss_and_dY(Y, seg, tsig, tval, 0.5)
    grads = mlp.backward(W, X, H1, H2, dY, bf16=False)
    h = 1e-6
    for wi, g in zip(range(6), grads):
        flat = W[wi].reshape(-1)
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for j in idx:
            old = flat[j]
            flat[j] = old + h
            lp = loss(W)
            flat[j] = old - h
            lm = loss(W)
            flat[j] = old
            num = (lp - lm) / (2 * h)
            assert g.reshape(-1)[j] == pytest.approx(num, rel=1e-5, abs=1e-8), (wi, j)
