"""Pins for the numpy MLP / feature references (CPU)."""
import numpy as np

from oracle import mlp_ref


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    widths = (6, 5, 4, 3)
    n = sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(3))
    w = rng.normal(size=n) * 0.5
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=(7, 3))
    _, grads = mlp_ref.backward(x, t, mlp_ref.split_params(w, widths))
    g = mlp_ref.flat(grads)
    eps = 1e-6
    for i in range(n):
        wp, wm = w.copy(), w.copy()
        wp[i] += eps
        wm[i] -= eps
        lp, _ = mlp_ref.backward(x, t, mlp_ref.split_params(wp, widths))
        lm, _ = mlp_ref.backward(x, t, mlp_ref.split_params(wm, widths))
        assert abs((lp - lm) / (2 * eps) - g[i]) < 1e-6 * max(1.0, abs(g[i])), i


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159], np.float32)
    r = mlp_ref.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0   # tie -> even
    assert r[2] == 1.0 + 2 ** -7         # above the tie -> up
    assert r[3] == -2.5 and abs(r[4] - 3.140625) < 1e-12


def test_features_of_a_ramp():
    """A uniform ramp of slope s deg/ms: positions interpolate exactly, velocity is s everywhere."""
    T, s = 57, 0.3
    r = s * np.arange(T)
    f = mlp_ref.features(r)
    t = (T - 1) * np.arange(128) / 127
    assert np.allclose(f[0::2], s * t / 16.0, atol=1e-12)
    assert np.allclose(f[1::2], s * 4.0, atol=1e-12)
