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


# ---------------------------------------------------------------------------
# Optimiser: Adam (Kingma & Ba, "Adam: A Method for Stochastic Optimization",
# ICLR 2015, Algorithm 1), written out in FP64 with the paper's default
# constants.  Beside the state it carries a running bound on how far an FP32
# evaluation of the same step (each operation rounded once, unit roundoff
# 2^-24) can drift from it, so a test can compare an FP32 implementation
# element by element.

U32 = 2.0 ** -24          # FP32 unit roundoff
TINY32 = 2.0 ** -126      # smallest normal FP32 (a product below it may be flushed)


class Adam:
    def __init__(self, w, beta1=0.9, beta2=0.999, eps=1e-8):
        self.w = np.array(w, np.float64)
        self.m = np.zeros_like(self.w)
        self.v = np.zeros_like(self.w)
        self.b1, self.b2, self.eps = beta1, beta2, eps
        self.t = 0
        # error bounds of an FP32 evaluation, per element
        self.em = np.zeros_like(self.w)
        self.ev = np.zeros_like(self.w)
        self.ew = np.abs(self.w) * 0.0
        self.mag_m = np.zeros_like(self.w)   # same recursion as m on |g|: the scale m is made of

    def step(self, g, lr):
        g = np.asarray(g, np.float64)
        b1, b2, eps = self.b1, self.b2, self.eps
        self.t += 1
        t = self.t
        # moment estimates
        m_prev, v_prev = self.m, self.v
        self.m = b1 * m_prev + (1.0 - b1) * g
        self.v = b2 * v_prev + (1.0 - b2) * g * g
        # bias-corrected estimates and the parameter update
        mhat = self.m / (1.0 - b1 ** t)
        vhat = self.v / (1.0 - b2 ** t)
        den = np.sqrt(vhat) + eps
        r = mhat / den
        self.w = self.w - lr * r
        # FP32 drift: m -- two products, one sum, the two constants' representation (4u of its
        # terms); v -- the same plus the square (5u, all terms non-negative, so relative; a square
        # below the normal range may be flushed); ratio -- the drift of m through 1/den, the
        # relative drift of v halved by the root, and six more roundings (two corrections, two
        # products, root, sum, quotient); w -- lr x ratio drift, the product and the difference.
        self.mag_m = b1 * self.mag_m + (1.0 - b1) * np.abs(g)
        self.em = b1 * self.em + 4.0 * U32 * self.mag_m
        self.ev = b2 * self.ev + 5.0 * U32 * self.v + (1.0 - b2) * TINY32
        c1 = 1.0 / (1.0 - b1 ** t)
        rel_v = np.where(self.v > 0, self.ev / np.where(self.v > 0, self.v, 1.0), 0.0)
        er = c1 * self.em / den + np.abs(r) * (0.5 * rel_v + 8.0 * U32)
        self.ew = self.ew + lr * er + U32 * (np.abs(self.w) + lr * np.abs(r))
        return self.w


def cosine_lr(t, n, lr0, lr_min):
    """Cosine decay from lr0 (step 0) to lr_min (step n - 1): Loshchilov & Hutter, "SGDR", ICLR 2017,
    eq. (5) over a single period without restarts."""
    ph = t / (n - 1) if n > 1 else 1.0
    return lr_min + 0.5 * (lr0 - lr_min) * (1.0 + np.cos(np.pi * ph))


# ---------------------------------------------------------------------------
# Training data: one generated training sample, from the oracle's plant.
#
# The sample's draws come from the SplitMix64 stream (Steele, Lea & Flood 2014)
# keyed by (data seed, output 1 + (step << 40 | i << 8 | k)): draw k = 0 the
# amplitude A = 2 + 28 u deg, k = 1 the noise level sigma = sigma_max u, k =
# 2..19 the multipliers 1 + spread (2u - 1) of the Table 1 nominal OPC (PW
# nominal = D - 6 ms with the main-sequence duration D = 2.2 A + 21 ms), and
# from k = 32 on Box-Muller pairs of Gaussian noise, one pair per two samples.
# u = (output >> 40) 2^-24.  The draws and the interface values (A, D, the OPC,
# the target) are FP32, as the data format fixes them; the trajectory is the
# oracle's FP64 RK4 integration; the trace is rounded to FP32 once.

Z_SCALE = 0.3


def _u24(seed, step, i, k):
    from . import splitmix64
    z = splitmix64(seed, 1 + ((step << 40) | (i << 8) | k))
    return np.float32((z >> 40) * 2.0 ** -24)


def box_muller(seed, step, i, T):
    """T standard normal draws of sample i: pair k, k+1 from uniforms k + 32, k + 33 (Box & Muller 1958),
    the first uniform kept at or above 2^-25 so its logarithm is finite."""
    out = np.zeros(T)
    for k in range(0, T, 2):
        u1 = max(float(_u24(seed, step, i, 32 + k)), 2.0 ** -25)
        u2 = float(_u24(seed, step, i, 33 + k))
        rad = np.sqrt(-2.0 * np.log(u1))
        out[k] = rad * np.cos(2.0 * np.pi * u2)
        if k + 1 < T:
            out[k + 1] = rad * np.sin(2.0 * np.pi * u2)
    return out


def training_sample(seed, step, i, spread=0.3, sigma_max=0.1):
    """Returns (features [256] float64, target z [18] float32, trace [T] float32, opc [18] float32, amp)."""
    from . import nominal, simulate
    f32 = np.float32
    amp = f32(f32(2.0) + f32(f32(28.0) * _u24(seed, step, i, 0)))
    dur = f32(f32(f32(2.2) * amp) + f32(21.0))
    T = int(np.ceil(dur))
    sigma = f32(f32(sigma_max) * _u24(seed, step, i, 1))
    nom = nominal(float(dur)).astype(np.float32)
    mult = np.array([f32(1.0) + f32(f32(spread) * (f32(2.0) * _u24(seed, step, i, 2 + j) - f32(1.0)))
                     for j in range(18)], np.float32)
    opc = (nom * mult).astype(np.float32)
    z = ((mult - f32(1.0)) / f32(Z_SCALE)).astype(np.float32)
    theta = simulate(opc.astype(np.float64), float(amp), T)
    trace = (theta + float(sigma) * box_muller(seed, step, i, T)).astype(np.float32)
    return features(trace), z, trace, opc, float(amp)
