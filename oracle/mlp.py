"""CPU oracle for the selector network: a 16 -> 64 -> 64 -> 1 perceptron with
ReLU hidden layers, the pinball (quantile) loss and the Adam update.

TEST INFRASTRUCTURE ONLY.  Plain float64 numpy, one row at a time where that
reads more clearly.  Parameter vector layout (5,313 entries, the library's
flat layout): W1[64][16] (row = hidden unit), b1[64], W2[64][64], b2[64],
W3[64], b3.

* Input normalisation: xn = (x - mu) / sd, with mu, sd stored beside the
  parameters (not trained).
* Forward: z1 = W1 xn + b1, h1 = max(z1, 0), z2 = W2 h1 + b2,
  h2 = max(z2, 0), y = W3 . h2 + b3.
* Loss over a batch of B rows with targets t: L = (1/B) sum rho_tau(t - y),
  rho_tau(r) = tau r for r > 0, (tau - 1) r otherwise (the quantile loss of
  Koenker and Bassett, 1978); dL/dy = -tau/B where t > y, (1 - tau)/B otherwise.
* Backward: the chain rule through the layers, ReLU derivative 1 where z > 0.
* Adam (Kingma and Ba, 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
  p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parity: the backward pass is pinned by central finite differences of the
loss, the forward pass by a hand-set network with a closed-form output, and
Adam by its first step, which moves every parameter with a non-zero gradient
by lr * g / (|g| + eps) (tests/test_oracle_mlp.py).
"""
import numpy as np

NIN, NH = 16, 64
SIZES = [("W1", (NH, NIN)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        cnt = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + cnt], dtype=np.float64).reshape(shape)
        o += cnt
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def forward(p, X, mu, sd):
    """Returns y [B] and the intermediate values of every row."""
    P = unpack(p)
    Xn = (np.asarray(X, np.float64) - mu) / sd
    Z1 = Xn @ P["W1"].T + P["b1"]
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ P["W2"].T + P["b2"]
    H2 = np.maximum(Z2, 0.0)
    y = H2 @ P["W3"] + P["b3"][0]
    return y, dict(Xn=Xn, Z1=Z1, H1=H1, Z2=Z2, H2=H2)


def pinball(y, t, tau):
    r = np.asarray(t, np.float64) - y
    return float(np.mean(np.where(r > 0, tau * r, (tau - 1.0) * r)))


def loss_grad(p, X, t, tau, mu, sd):
    """(loss, gradient of the loss w.r.t. the flat parameter vector)."""
    y, c = forward(p, X, mu, sd)
    P = unpack(p)
    B = y.shape[0]
    r = np.asarray(t, np.float64) - y
    d3 = np.where(r > 0, -tau, 1.0 - tau) / B            # dL/dy per row
    g = {"W3": c["H2"].T @ d3, "b3": np.array([d3.sum()])}
    d2 = np.outer(d3, P["W3"]) * (c["Z2"] > 0)
    g["W2"] = d2.T @ c["H1"]
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (c["Z1"] > 0)
    g["W1"] = d1.T @ c["Xn"]
    g["b1"] = d1.sum(axis=0)
    return pinball(y, t, tau), pack(g)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict_slices(y, smin=2, smax=12):
    """Slice count from the network output, rounded half up and clamped:
    clamp(floor(y + 1/2), smin, smax).  The pinball loss with tau near 1 puts
    y at an upper quantile of the integer labels, so the nearest integer is
    the prediction (a ceiling would add one slice whenever y lands just above
    the label)."""
    return np.clip(np.floor(np.asarray(y) + 0.5), smin, smax).astype(np.int64)
