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


def test_adam_first_step_and_constant_gradient():
    """Adam's bias corrections make m_hat = g and v_hat = g^2 whenever the gradient has been the same
    at every step so far (Kingma & Ba 2015, Section 3), so each step moves w by lr g / (|g| + eps),
    whatever beta1 and beta2 are.  A swapped correction, eps under the root or a wrong moment weight
    breaks this."""
    g = np.array([3.0, -2e-3, 1e-7, 0.0, -5e-9])
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        a = mlp_ref.Adam(np.ones(5), beta1=b1, beta2=b2, eps=1e-8)
        w = np.ones(5)
        for t in range(1, 30):
            lr = 1e-3 * t
            a.step(g, lr)
            w = w - lr * g / (np.abs(g) + 1e-8)
            assert np.allclose(a.w, w, rtol=1e-12, atol=1e-15), (b1, b2, t)


def test_adam_matches_torch_optimizer():
    """Against torch.optim.Adam (an independent implementation of the same algorithm) in FP64, with a
    varying gradient and learning rate."""
    torch = __import__("torch")
    rng = np.random.default_rng(3)
    w0 = rng.normal(size=50)
    a = mlp_ref.Adam(w0)
    p = torch.nn.Parameter(torch.tensor(w0, dtype=torch.float64))
    opt = torch.optim.Adam([p], lr=1.0, betas=(0.9, 0.999), eps=1e-8)
    for t in range(25):
        g = rng.normal(size=50) * 10.0 ** rng.uniform(-6, 1, size=50)
        lr = mlp_ref.cosine_lr(t, 25, 2e-3, 1e-4)
        for grp in opt.param_groups:
            grp["lr"] = lr
        p.grad = torch.tensor(g)
        opt.step()
        a.step(g, lr)
        assert np.allclose(a.w, p.detach().numpy(), rtol=1e-13, atol=1e-15), t
        st = opt.state[p]
        assert np.allclose(a.m, st["exp_avg"].numpy(), rtol=1e-13, atol=1e-300)
        assert np.allclose(a.v, st["exp_avg_sq"].numpy(), rtol=1e-13, atol=1e-300)


def test_adam_fp32_drift_bound_covers_an_fp32_evaluation():
    """The running bound holds for a plain numpy FP32 evaluation of the same steps, and is tight enough
    to flag a bias correction computed as 1 - beta^t in FP32 (cancellation, ~1e-5 relative) on the
    entries that start at zero, where the update is not hidden under the rounding of w."""
    rng = np.random.default_rng(5)
    n = 4000
    w0 = rng.normal(size=n).astype(np.float32)
    w0[::2] = 0.0
    a = mlp_ref.Adam(w0)
    f = np.float32
    w, m, v = w0.copy(), np.zeros(n, np.float32), np.zeros(n, np.float32)
    bad = w0.copy(); mb, vb = np.zeros(n, np.float32), np.zeros(n, np.float32)
    flagged = False
    for t in range(1, 13):
        g = (rng.normal(size=n) * 10.0 ** rng.uniform(-5, 0, size=n)).astype(np.float32)
        lr = f(mlp_ref.cosine_lr(t - 1, 12, 2e-3, 1e-4))
        c1, c2 = f(1.0 / (1.0 - 0.9 ** t)), f(1.0 / (1.0 - 0.999 ** t))
        m = f(0.9) * m + f(0.1) * g
        v = f(0.999) * v + f(0.001) * (g * g)
        w = w - lr * ((m * c1) / (np.sqrt(v * c2) + f(1e-8)))
        # the same with the corrections' 1 - beta^t taken in FP32
        cb1 = f(1.0) / (f(1.0) - f(0.9) ** f(t)); cb2 = f(1.0) / (f(1.0) - f(0.999) ** f(t))
        mb = f(0.9) * mb + (f(1.0) - f(0.9)) * g
        vb = f(0.999) * vb + (f(1.0) - f(0.999)) * (g * g)
        bad = bad - lr * ((mb * cb1) / (np.sqrt(vb * cb2) + f(1e-8)))
        a.step(g.astype(np.float64), float(lr))
        assert np.all(np.abs(m - a.m) <= a.em) and np.all(np.abs(v - a.v) <= a.ev)
        assert np.all(np.abs(w - a.w) <= a.ew), (t, np.max(np.abs(w - a.w) / a.ew))
        flagged |= bool(np.any(np.abs(bad - a.w) > a.ew))
    assert flagged


def test_cosine_schedule_matches_torch():
    torch = __import__("torch")
    p = torch.nn.Parameter(torch.zeros(1))
    opt = torch.optim.SGD([p], lr=2e-3)
    sch = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=19, eta_min=1e-4)
    for t in range(20):
        assert abs(opt.param_groups[0]["lr"] - mlp_ref.cosine_lr(t, 20, 2e-3, 1e-4)) <= 1e-15
        opt.step()
        sch.step()


def test_training_sample_reference():
    """The generated-sample reference: spread 0 gives the FP32 nominal OPC and z = 0; the noise-free trace
    is the oracle's trajectory rounded once, starts at rest and heads for the drawn amplitude; the
    duration is the main sequence; targets stay in [-1, 1]."""
    import oracle
    feat, z, tr, opc, amp = mlp_ref.training_sample(9, 4, 17, spread=0.0, sigma_max=0.0)
    dur = np.float32(np.float32(np.float32(2.2) * np.float32(amp)) + np.float32(21.0))
    assert len(tr) == int(np.ceil(dur)) and 2.0 <= amp < 30.0
    assert np.array_equal(opc, oracle.nominal(float(dur)).astype(np.float32)) and np.all(z == 0)
    assert np.array_equal(tr, oracle.simulate(opc.astype(np.float64), amp, len(tr)).astype(np.float32))
    assert tr[0] == 0.0 and 0.2 * amp < tr[-1] < amp   # on its way to the amplitude at t = D
    assert np.array_equal(feat, mlp_ref.features(tr))
    for i in range(40):
        _, z, _, opc, _ = mlp_ref.training_sample(9, 4, i, spread=0.3, sigma_max=0.0)
        assert np.all(np.abs(z) <= 1.0 + 1e-6)


def test_box_muller_draws_are_standard_normal():
    from scipy import stats
    x = np.concatenate([mlp_ref.box_muller(12, s, i, 100) for s in range(3) for i in range(40)])
    assert abs(x.mean()) < 0.04 and abs(x.var() - 1.0) < 0.05
    assert stats.kstest(x, "norm").pvalue > 1e-3
