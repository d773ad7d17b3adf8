"""FP64 NumPy oracle of the screening MLP (test infrastructure only).

The network (from the workload definition of the learned screen, not from the
paper): a_0 = x; z_l = a_{l-1} W_l + b_l and a_l = GELU(z_l) for the hidden
layers, with GELU(z) = z Phi(z) (Phi the standard normal CDF); the output
y = a_L W_out + b_out.  Loss: mean squared error over the batch.  Gradients
by hand-written backpropagation; Adam with the textbook bias correction.
"""
import numpy as np
from scipy.special import erf


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(params, x):
    """params: list of (W [fan_in, fan_out], b [fan_out]); returns y [n] and the
    pre-activations / activations needed by the backward pass."""
    a = np.asarray(x, dtype=np.float64)
    acts, zs = [a], []
    for l, (W, b) in enumerate(params):
        z = a @ np.asarray(W, np.float64) + np.asarray(b, np.float64)
        zs.append(z)
        a = gelu(z) if l < len(params) - 1 else z
        acts.append(a)
    return a[:, 0], (acts, zs)


def loss_and_grads(params, x, t):
    """MSE loss and its gradient with respect to every W and b."""
    y, (acts, zs) = forward(params, x)
    n = y.shape[0]
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    delta = (2.0 / n * r)[:, None]                     # dL/dz of the output layer
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W = np.asarray(params[l][0], np.float64)
        gW = acts[l].T @ delta
        gb = delta.sum(0)
        grads[l] = (gW, gb)
        if l > 0:
            delta = (delta @ W.T) * gelu_grad(zs[l - 1])
    return loss, grads


def flat(grads):
    return np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])


def adam_step(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (returns new params, m, v); step counts from 1."""
    out_p, out_m, out_v = [], [], []
    for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
        new = []
        for p, g, mm, vv in ((W, gW, mW, vW), (b, gb, mb, vb)):
            mm = b1 * mm + (1 - b1) * g
            vv = b2 * vv + (1 - b2) * g * g
            mh = mm / (1 - b1 ** step)
            vh = vv / (1 - b2 ** step)
            new.append((p - lr * mh / (np.sqrt(vh) + eps), mm, vv))
        out_p.append((new[0][0], new[1][0]))
        out_m.append((new[0][1], new[1][1]))
        out_v.append((new[0][2], new[1][2]))
    return out_p, out_m, out_v
