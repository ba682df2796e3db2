"""Pins of the FP64 surrogate-network oracle: gradients against central finite
differences of its own loss, SiLU derivative against a finite difference of
SiLU, Adam against its closed form for a constant gradient, and the flat
parameter layout's round trip."""
import numpy as np

from oracle import mlp as M

NIN, HID, NOUT = 5, 7, 4


def rand_problem(seed, N=9):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(M.nparams(NIN, HID, NOUT)) * 0.5
    X = rng.standard_normal((N, NIN))
    T = rng.standard_normal((N, NOUT))
    return theta, X, T


def test_parameter_count_of_the_surrogate():
    assert M.nparams(21, 128, 21) == 22037


def test_pack_unpack_round_trip():
    theta, _, _ = rand_problem(0)
    assert np.array_equal(M.pack(M.unpack(theta, NIN, HID, NOUT), NIN, HID, NOUT), theta)


def test_gradient_matches_central_differences():
    theta, X, T = rand_problem(1)
    L, g = M.loss_and_grad(theta, X, T, NIN, HID, NOUT)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (M.loss_and_grad(tp, X, T, NIN, HID, NOUT)[0]
                 - M.loss_and_grad(tm, X, T, NIN, HID, NOUT)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    # the loss is the mean of squares
    O, _ = M.forward(theta, X, NIN, HID, NOUT)
    assert abs(L - ((O - T) ** 2).mean()) < 1e-14


def test_silu_and_derivative():
    z = np.linspace(-30, 30, 241)
    assert np.allclose(M.silu(z), z * 0.5 * (1 + np.tanh(z / 2)), rtol=1e-12, atol=1e-14)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.abs(M.silu_grad(z) - fd).max() < 1e-8


def test_adam_closed_form_constant_gradient():
    """With a constant gradient g, m_t = g(1-b1^t), v_t = g^2(1-b2^t): every bias-corrected
    step moves theta by -lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    theta = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    for t in range(1, 6):
        theta, m, v = M.adam_step(theta, m, v, g, t, lr)
        np.testing.assert_allclose(theta, -lr * t * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, g * (1 - 0.9 ** 5), rtol=1e-12)
    np.testing.assert_allclose(v, g * g * (1 - 0.999 ** 5), rtol=1e-12)
