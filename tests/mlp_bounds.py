"""Element-wise error bounds for the BF16 MLP against the FP64 oracle.

Every matrix product multiplies bfloat16 values (exact in FP32) and sums in
FP32, so a GPU output z differs from the FP64 sum by at most U times the sum
of |terms| (U = 2e-6, the bound the GEMM test checks directly).  A result
rounded to bfloat16 (a hidden activation or a hidden gradient) can then
differ from the oracle's rounding only where the FP64 value lies within that
band of a rounding point; there the difference is at most the distance to
the neighbouring bfloat16 value, and it is carried into the next product
through |weights|.  The bounds below add up exactly these allowances, element
by element, so an element that is not near a rounding point must match to
FP32 accumulation, and a wrong or dropped term shows as a violation."""
import numpy as np

from oracle import mlp as omlp

U = 2e-6
q = omlp.bf16_round


def rounding_allowance(z, band, relu=False):
    """Largest |bf16(z') - bf16(z)| over |z' - z| <= band (after ReLU)."""
    f = (lambda x: np.maximum(x, 0.0)) if relu else (lambda x: x)
    mid = q(f(z))
    return np.maximum(q(f(z + band)) - mid, mid - q(f(z - band)))


def layer_bounds(Hin, Wl, bl, relu):
    """One layer on given (bfloat16) inputs: the oracle's output
    (bf16(relu(Hin Wq + b)) for a hidden layer, else Hin Wq + b) and the
    per-element bound on |GPU - oracle| for the same inputs."""
    Wq = q(Wl)
    z = Hin @ Wq + bl
    band = U * (np.abs(Hin) @ np.abs(Wq) + np.abs(bl))
    if not relu:
        return z, band
    return q(np.maximum(z, 0.0)), rounding_allowance(z, band, relu=True)


def forward_bounds(W, X):
    """Oracle forward (H1, H2, Y) and per-element bounds (A1, A2, bY) on
    |GPU - oracle| for H1, H2 (bfloat16) and Y, the allowances of each layer
    carried into the next (for a GPU path whose activations are not seen)."""
    W1, b1, W2, b2, W3, b3 = W
    H1, A1 = layer_bounds(q(X), W1, b1, True)
    W2q, W3q = q(W2), q(W3)
    z2 = H1 @ W2q + b2
    band2 = U * (np.abs(H1) @ np.abs(W2q) + np.abs(b2)) + A1 @ np.abs(W2q)
    H2 = q(np.maximum(z2, 0.0))
    A2 = rounding_allowance(z2, band2, relu=True)
    Y = H2 @ W3q + b3
    bY = U * (np.abs(H2) @ np.abs(W3q) + np.abs(b3)) + A2 @ np.abs(W3q)
    return (H1, H2, Y), (A1, A2, bY)


def backward_bounds(W, X, H1, H2, dY):
    """Per-element bounds on |GPU - oracle| of (dW1, db1, dW2, db2, dW3, db3)
    for the oracle's backward pass on the same activations H1, H2 and the
    same FP32 output gradient dY (omlp.backward)."""
    W1, b1, W2, b2, W3, b3 = W
    Xq, W2q, W3q, dYq = q(X), q(W2), q(W3), q(dY)
    m2 = H2 > 0
    m1 = H1 > 0
    z2 = (dYq @ W3q.T) * m2
    band2 = U * (np.abs(dYq) @ np.abs(W3q).T) * m2
    G2q = q(z2)
    A2 = rounding_allowance(z2, band2)
    z1 = (G2q @ W2q.T) * m1
    band1 = (U * (np.abs(G2q) @ np.abs(W2q).T) + A2 @ np.abs(W2q).T) * m1
    G1q = q(z1)
    A1 = rounding_allowance(z1, band1)
    bdW1 = U * (np.abs(Xq).T @ np.abs(G1q)) + np.abs(Xq).T @ A1
    bdb1 = U * np.abs(z1).sum(axis=0) + band1.sum(axis=0)
    bdW2 = U * (np.abs(H1).T @ np.abs(G2q)) + np.abs(H1).T @ A2
    bdb2 = U * np.abs(z2).sum(axis=0) + band2.sum(axis=0)
    bdW3 = U * (np.abs(H2).T @ np.abs(dYq))
    bdb3 = U * np.abs(dY).sum(axis=0)
    return bdW1, bdb1, bdW2, bdb2, bdW3, bdb3
