"""Pins of the oracle's Adam step (oracle/optim.py) by closed forms of the
published algorithm: the bias correction makes the first step, and every step
under a constant gradient, equal to -lr g / (|g| + eps) elementwise; a zero
gradient leaves theta unchanged; beta1 = beta2 = 0 reduces to that step for any
gradient sequence; and one hand-worked two-step case with changing gradients."""
import numpy as np
import pytest

from oracle import optim


def test_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    th, g = rng.normal(size=50), rng.normal(size=50)
    z = np.zeros(50)
    t1, m, v = optim.adam_step(th, g, z, z, 1, lr=1e-2, eps=1e-8)
    assert np.allclose(t1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_constant_gradient_gives_constant_step():
    g = np.array([0.5, -2.0, 3e-3, -7.0])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 40):
        th_new, m, v = optim.adam_step(th, g, m, v, t, lr=0.1, eps=1e-12)
        assert np.allclose(th_new - th, -0.1 * g / (np.abs(g) + 1e-12), rtol=1e-12, atol=0)
        th = th_new


def test_zero_gradient_is_a_fixed_point():
    th = np.array([1.0, -2.0, 3.0])
    z = np.zeros(3)
    t1, m, v = optim.adam_step(th, z, z, z, 5)
    assert np.array_equal(t1, th) and not m.any() and not v.any()


def test_no_memory_reduces_to_normalised_step():
    rng = np.random.default_rng(1)
    th = rng.normal(size=8)
    m = v = np.zeros(8)
    for t in range(1, 6):
        g = rng.normal(size=8)
        th_new, m, v = optim.adam_step(th, g, m, v, t, lr=0.3, beta1=0.0, beta2=0.0, eps=1e-9)
        assert np.allclose(th_new - th, -0.3 * g / (np.abs(g) + 1e-9), rtol=1e-13, atol=0)
        th = th_new


def test_two_steps_by_hand():
    # beta1 = 0.5, beta2 = 0.75, lr = 1, eps = 0, scalar gradients 2 then 4
    th, m, v = np.array([0.0]), np.array([0.0]), np.array([0.0])
    th, m, v = optim.adam_step(th, np.array([2.0]), m, v, 1, lr=1.0, beta1=0.5, beta2=0.75, eps=1e-300)
    assert m[0] == 1.0 and v[0] == 1.0 and th[0] == pytest.approx(-1.0, abs=1e-15)   # m^ = 2, v^ = 4
    th, m, v = optim.adam_step(th, np.array([4.0]), m, v, 2, lr=1.0, beta1=0.5, beta2=0.75, eps=1e-300)
    # m = 0.5 + 2 = 2.5, m^ = 2.5 / 0.75; v = 0.75 + 4 = 4.75, v^ = 4.75 / 0.4375
    assert m[0] == 2.5 and v[0] == 4.75
    assert th[0] == pytest.approx(-1.0 - (2.5 / 0.75) / np.sqrt(4.75 / 0.4375), rel=1e-15)


def test_step_count_must_start_at_one():
    with pytest.raises(ValueError):
        optim.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 0)
