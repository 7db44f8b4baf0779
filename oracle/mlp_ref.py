"""Plain numpy references for the learned seed -- test infrastructure only.

* ``features``: resample a trace to 128 points over its own duration (linear
  interpolation) as (position/16, velocity*4) pairs; velocity is the central
  difference of the trace (one-sided at the ends), interpolated the same way.
* ``forward`` / ``backward``: the MLP (ReLU hidden layers, linear output, mean
  squared error) in FP64 with explicit loops over layers, written from the
  chain rule; ``split_params`` maps the flat parameter vector (W0 [in][out],
  b0, W1, b1, ...) to layers.
* ``bf16``: round-to-nearest-even to bfloat16 (the operand format of the GPU
  GEMMs), used to hand the reference the same operands the GPU sees.
"""
import numpy as np

NPTS = 128


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def features(r, dt=1.0):
    r = np.asarray(r, np.float64)
    T = r.shape[0]
    vel = np.zeros(T)
    for q in range(T):
        if T < 2:
            break
        a, b = max(q - 1, 0), min(q + 1, T - 1)
        vel[q] = (r[b] - r[a]) / ((b - a) * dt)
    out = np.zeros(2 * NPTS)
    for j in range(NPTS):
        t = (T - 1) * j / (NPTS - 1)
        k = min(max(int(np.floor(t)), 0), max(T - 2, 0))
        f = t - k
        p1 = r[k + 1] if T > 1 else r[0]
        v1 = vel[k + 1] if T > 1 else vel[0]
        out[2 * j] = (r[k] + f * (p1 - r[k])) / 16.0
        out[2 * j + 1] = (vel[k] + f * (v1 - vel[k])) * 4.0
    return out


def split_params(w, widths):
    layers, off = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = np.asarray(w[off:off + n_in * n_out], np.float64).reshape(n_in, n_out)
        off += n_in * n_out
        b = np.asarray(w[off:off + n_out], np.float64)
        off += n_out
        layers.append((W, b))
    assert off == len(w)
    return layers


def forward(x, layers):
    """Returns the output and the list of layer inputs (post-ReLU activations)."""
    acts = [np.asarray(x, np.float64)]
    h = acts[0]
    for l, (W, b) in enumerate(layers):
        z = h @ W + b
        if l < len(layers) - 1:
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h, acts


def backward(x, target, layers):
    """Loss = mean over all outputs of (out - target)^2; returns loss and per-layer (dW, db)."""
    out, acts = forward(x, layers)
    n = out.size
    d = 2.0 * (out - target) / n
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (acts[l].T @ d, d.sum(axis=0))
        if l > 0:
            d = (d @ W.T) * (acts[l] > 0)
    return float(np.mean((out - target) ** 2)), grads


def flat(grads):
    return np.concatenate([np.concatenate([g[0].reshape(-1), g[1]]) for g in grads])
