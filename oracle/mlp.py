"""Oracle float64 MLP for the fusion cost model.  Test infrastructure only.

Not from the paper (which has no learned component): a plain multilayer
perceptron with ReLU hidden layers and a linear scalar output, trained on
mean squared error with Adam (Kingma and Ba, arXiv:1412.6980, Algorithm 1).

Layout shared with the GPU kernels by convention only (no shared code):
weights W_l are row-major [fan_in, fan_out], biases b_l are [fan_out],
activations are row-major [batch, features].
"""
import numpy as np


def forward(params, X):
    """Returns (prediction [batch], cache).  params = [(W1, b1), ..., (WL, bL)]."""
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    a = acts[0]
    for li, (W, b) in enumerate(params):
        z = a @ W + b
        pre.append(z)
        a = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(a)
    return a[:, 0], (acts, pre)


def mse(pred, target):
    d = pred - target
    return float(np.mean(d * d))


def backward(params, cache, pred, target):
    """Gradients of mean((pred - target)^2) for every (W, b)."""
    acts, pre = cache
    B = pred.shape[0]
    dz = (2.0 / B) * (pred - target)[:, None]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        grads[li] = (acts[li].T @ dz, dz.sum(axis=0))
        if li > 0:
            da = dz @ W.T
            dz = da * (pre[li - 1] > 0)
    return grads


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of array p (returns new p, m, v); t counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
