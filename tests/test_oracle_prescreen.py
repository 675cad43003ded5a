"""Pins of the pre-screen network oracle (CPU, float64).

The gradient is pinned by central finite differences of the loss (an
independent check of every backward rule), the convolution by delta kernels
(identity and a known shift), the pooling by its tie rule, and the loss by its
value and slope at logit 0.
"""

import numpy as np

from oracle import prescreen as ps


def _theta(seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=ps.n_params())


def _block(seed):
    rng = np.random.default_rng(seed)
    p = rng.exponential(size=ps.BLOCK)
    p[1000:1010] += 40.0  # a bright feature
    return ps.features(p)


def test_parameter_count():
    assert ps.n_params() == (32 * 9 + 32) + 3 * (32 * 32 * 9 + 32) + 32 + 1


def test_conv_delta_kernels():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 50))
    W = np.zeros((3, 3, 9))
    for c in range(3):
        W[c, c, 4] = 1.0
    np.testing.assert_array_equal(ps.conv(x, W, np.zeros(3)), x)
    W = np.zeros((3, 3, 9))
    for c in range(3):
        W[c, c, 8] = 1.0  # y[t] = x[t + 4], zero past the end
    y = ps.conv(x, W, np.full(3, 0.5))
    np.testing.assert_array_equal(y[:, :46], x[:, 4:] + 0.5)
    np.testing.assert_array_equal(y[:, 46:], np.full((3, 4), 0.5))


def test_maxpool_first_maximum():
    y = np.array([[1.0, 3.0, 3.0, 0.0, 2.0, 2.0, 2.0, 2.0]])
    v, arg = ps.maxpool(y)
    np.testing.assert_array_equal(v, [[3.0, 2.0]])
    np.testing.assert_array_equal(arg, [[1, 0]])


def test_loss_is_finite_far_from_zero():
    for logit in (-800.0, 800.0):
        for lab in (0.0, 1.0):
            # the sigmoid's exp(-logit) overflows to inf at -800, which gives
            # the exact limit s = 0; the loss must stay finite regardless
            with np.errstate(over="ignore"):
                loss, d = ps.loss_and_dlogit(logit, lab, 2.0)
            assert np.isfinite(loss) and np.isfinite(d)
    loss, _ = ps.loss_and_dlogit(800.0, 0.0, 2.0)
    assert abs(loss - 800.0) < 1e-9


def test_loss_at_zero_logit():
    for w in (1.0, 5.0):
        l1, d1 = ps.loss_and_dlogit(0.0, 1.0, w)
        l0, d0 = ps.loss_and_dlogit(0.0, 0.0, w)
        assert abs(l1 - w * np.log(2)) < 1e-15 and abs(d1 + w / 2) < 1e-15
        assert abs(l0 - np.log(2)) < 1e-15 and abs(d0 - 0.5) < 1e-15


def test_gradient_matches_finite_differences():
    theta = _theta(3)
    X = np.stack([_block(10), _block(11)])
    y = np.array([1.0, 0.0])
    _, g = ps.batch_loss_grad(theta, X, y, 3.0)
    rng = np.random.default_rng(4)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in ps.param_shapes()])
    # a few indices in every parameter tensor
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], size=min(6, offs[i + 1] - offs[i]))
                          for i in range(len(offs) - 1)])
    eps = 1e-6
    checked = 0
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        lp, _ = ps.batch_loss_grad(tp, X, y, 3.0)
        lm, _ = ps.batch_loss_grad(tm, X, y, 3.0)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (int(i), fd, g[i])
        checked += 1
    assert checked == idx.size
    assert np.abs(g).max() > 0
