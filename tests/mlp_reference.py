"""Plain NumPy FP64 multilayer perceptron with the library's parameter layout
(layer by layer: W as nout x nin row-major, then b; tanh hidden layers,
linear output) and the masked mean-squared-error loss
    L = sum_{b,o} mask[b,o] (y[b,o] - t[b,o])^2 / sum mask.
Used only by tests to check the GPU forward/backward/Adam kernels."""
import numpy as np


def unpack(w, dims):
    out, k = [], 0
    for nin, nout in zip(dims[:-1], dims[1:]):
        W = w[k:k + nin * nout].reshape(nout, nin)
        k += nin * nout
        b = w[k:k + nout]
        k += nout
        out.append((W, b))
    assert k == w.size
    return out


def forward(w, dims, x):
    acts = [x]
    layers = unpack(np.asarray(w, np.float64), dims)
    for l, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(z if l == len(layers) - 1 else np.tanh(z))
    return acts


def loss(w, dims, x, t, mask=None):
    y = forward(w, dims, x)[-1]
    m = np.ones_like(t) if mask is None else mask
    return float(np.sum(m * (y - t) ** 2) / max(np.sum(m), 1.0))


def gradient(w, dims, x, t, mask=None):
    """Backpropagation written out layer by layer."""
    w = np.asarray(w, np.float64)
    layers = unpack(w, dims)
    acts = forward(w, dims, x)
    m = np.ones_like(t) if mask is None else mask
    cnt = max(np.sum(m), 1.0)
    dz = 2.0 * m * (acts[-1] - t) / cnt
    grads = []
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        if l != len(layers) - 1:
            dz = dz * (1.0 - acts[l + 1] ** 2)
        grads.append((dz.T @ acts[l], dz.sum(0)))
        dz = dz @ W
    flat = []
    for gW, gb in reversed(grads):
        flat += [gW.ravel(), gb]
    return np.concatenate(flat)


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
