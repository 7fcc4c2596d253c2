"""Plain FP64 reference of the warm-start perceptron (test infrastructure).

Only the tests and the benchmark's CPU baseline use this module; the library
never does.  Network: widths dims[0] -> ... -> dims[L], hidden activations
tanh, linear output, parameters flat [W_1 b_1 ... W_L b_L] with W_l of shape
(dims[l], dims[l-1]).  Batches are (features, samples).  Loss: mean squared
error over all outputs and samples,

    loss = sum (Y - T)^2 / (dims[L] * S).

The gradient is the chain rule written out layer by layer (reverse mode).
"""
import numpy as np


def unpack(params, dims):
    out, off = [], 0
    for l in range(len(dims) - 1):
        n_in, n_out = dims[l], dims[l + 1]
        W = params[off:off + n_in * n_out].reshape(n_out, n_in)
        off += n_in * n_out
        b = params[off:off + n_out]
        off += n_out
        out.append((W, b))
    assert off == params.size
    return out


def n_params(dims):
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))


def forward(params, dims, X):
    """Activations of every layer (the input first)."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64), dims)
    for l, (W, b) in enumerate(layers):
        z = W @ acts[-1] + b[:, None]
        acts.append(np.tanh(z) if l < len(layers) - 1 else z)
    return acts


def loss_and_grad(params, dims, X, T):
    params = np.asarray(params, dtype=np.float64)
    acts = forward(params, dims, X)
    Y = acts[-1]
    n = Y.size
    loss = float(np.sum((Y - T) ** 2) / n)
    layers = unpack(params, dims)
    grads = []
    d = 2.0 * (Y - T) / n                     # d loss / d z of the last layer
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads.append((d @ acts[l].T, d.sum(axis=1)))
        if l > 0:
            d = (W.T @ d) * (1.0 - acts[l] ** 2)   # through tanh of layer l
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat
