"""Seeded initial weights of the screening MLP (inputs shared by the oracle
and the GPU library; no network arithmetic here).

Layout of the flat parameter vector: for each layer l = 1..depth+1,
W_l [fan_in][fan_out] row-major, then b_l [fan_out].  Weights are normal with
standard deviation sqrt(2 / fan_in); biases start at zero.
"""
import numpy as np


def layer_sizes(nin, width, depth):
    return [nin] + [width] * depth + [1]


def init_params(nin, width=256, depth=3, seed=4):
    rng = np.random.default_rng(seed)
    sizes = layer_sizes(nin, width, depth)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        parts.append((rng.standard_normal((a, b)) * np.sqrt(2.0 / a)).ravel())
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def unflatten(flat, nin, width=256, depth=3):
    sizes = layer_sizes(nin, width, depth)
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        bias = flat[o:o + b]
        o += b
        out.append((W, bias))
    return out


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float32: the effective values of BF16 weights and inputs."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)
