"""Pins of the oracle's adaptive parameter setting (oracle/ita.py:
normalized_step, kth_largest_magnitude, ita_adaptive; Section IV.B) against
what does not depend on its own formulas: the exact line search of the data
term, a dense brute-force operator on a tiny grid, the orthonormal (full
mask) closed form, the fixed-lambda oracle at the first iteration, and exact
recovery of a noiseless sparse scene."""

import numpy as np
import pytest

import inputs
from oracle import csa, ita

STRIP = inputs.RADAR_STRIPMAP
STRESS = inputs.RADAR_LBAND_STRESS


def _scene(params, shape, k, rate, seed, noisy=True):
    g = csa.Geometry(params, shape)
    rows, cols, sig = inputs.point_targets(shape, k, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, rate, seed=seed + 1)
    y = mask * csa.G(xt, g)
    if noisy:
        n = inputs.circular_noise(shape, seed + 2)
        y = y + mask * 0.05 * np.sqrt(np.mean(np.abs(y[mask]) ** 2)) * n
    return g, xt, mask, y


def test_kth_largest_magnitude_special_cases():
    v = np.array([3.0, -5.0, 1j, 4.0 + 0j, 0.0])
    assert ita.kth_largest_magnitude(v, 1) == 5.0
    assert ita.kth_largest_magnitude(v, 2) == 4.0
    assert ita.kth_largest_magnitude(v, 5) == 0.0
    assert ita.kth_largest_magnitude(v, 6) == 0.0  # fewer entries than r
    assert ita.kth_largest_magnitude(np.array([2.0, 2.0, 1.0]), 2) == 2.0  # ties


@pytest.mark.parametrize("params", [STRIP, STRESS])
def test_step_is_the_exact_line_search(params):
    # mu minimises phi(t) = 1/2 ||m o (y - G(X + t dX_G))||^2: phi'(mu) = 0
    # and phi is larger on both sides (checked on phi itself, not on the
    # ratio).  A transposed ratio, or a numerator taken over the whole
    # image, fails this.
    shape = (16, 32)
    g, xt, mask, y = _scene(params, shape, 6, 0.5, seed=31)
    x, *_ = ita.ita_adaptive(y, mask, 6, 2, g)
    assert np.count_nonzero(x) == 6
    m = mask.astype(float)
    dx = csa.M(m * (y - csa.G(x, g)), g)
    mu = ita.normalized_step(dx, x != 0, mask, g)
    d = np.where(x != 0, dx, 0)

    def phi(t):
        r = m * (y - csa.G(x + t * d, g))
        return 0.5 * float(np.vdot(r, r).real)

    h = 1e-4 * mu
    assert abs((phi(mu + h) - phi(mu - h)) / (2 * h)) <= 1e-8 * phi(0.0) / mu
    assert phi(mu) < phi(0.99 * mu) and phi(mu) < phi(1.01 * mu)
    # the step exceeds 1 with a thinned mask (||m o G z|| <= ||z||)
    assert mu > 1.0


def test_step_of_a_single_pixel_support_by_brute_force():
    # Support {p}: mu = 1 / sum_q m_q |G_qp|^2, with column p of G built by
    # applying G to the unit vector (brute force over the dense operator).
    shape = (8, 16)
    g = csa.Geometry(STRESS, shape)
    mask = inputs.random_mask(shape, 0.4, seed=5)
    dx = inputs.random_complex(shape, seed=6)
    for p in [(0, 0), (3, 7), (7, 15)]:
        e = np.zeros(shape, complex)
        e[p] = 1.0
        col = csa.G(e, g)
        want = 1.0 / float(np.sum(mask * np.abs(col) ** 2))
        sup = np.zeros(shape, bool)
        sup[p] = True
        got = ita.normalized_step(dx, sup, mask, g)
        assert abs(got - want) <= 1e-12 * want


@pytest.mark.parametrize("rate", [1.0, 0.5])
def test_step_over_the_whole_image_is_one(rate):
    # Support = every pixel and dX = M(m o R): ||m o G dX|| = ||m o R|| = ||dX||
    # (Theorem 1 with G M = I), so mu = 1 exactly; the empty support gives 1 too.
    shape = (16, 16)
    g = csa.Geometry(STRIP, shape)
    mask = inputs.random_mask(shape, rate, seed=9)
    r = mask * inputs.random_complex(shape, seed=10)
    dx = csa.M(r, g)
    assert abs(ita.normalized_step(dx, np.ones(shape, bool), mask, g) - 1.0) <= 1e-12
    assert ita.normalized_step(dx, np.zeros(shape, bool), mask, g) == 1.0


def test_full_mask_closed_form():
    # m = 1: mu = 1 at every iteration (G unitary) and X + dX = M y, so every
    # iterate is the k-term soft threshold of M y at its (k+1)-th magnitude.
    shape = (16, 32)
    g = csa.Geometry(STRESS, shape)
    y = inputs.random_complex(shape, seed=12)
    ones = np.ones(shape, bool)
    my = csa.M(y, g)
    s = ita.kth_largest_magnitude(my, 11)
    want = ita.soft_threshold(my, s)
    for iters in (1, 4):
        x, res, mus, lams = ita.ita_adaptive(y, ones, 10, iters, g)
        assert np.allclose(mus, 1.0, rtol=0, atol=1e-12)
        assert np.allclose(lams, s, rtol=1e-12, atol=0)
        assert np.abs(x - want).max() <= 1e-12 * np.abs(my).max()


def test_first_iteration_equals_fixed_lambda_rule():
    # X(1) with the adaptive rule is the fixed-lambda iteration with lambda
    # set once from the sparsity at X(0) = 0 (mu_0 = 1).
    shape = (32, 32)
    g, xt, mask, y = _scene(STRIP, shape, 12, 0.5, seed=41)
    lam = ita.lambda_from_sparsity(y, mask, 12, g)
    x1, _ = ita.ita(y, mask, lam, 1, g)
    xa, _, mus, lams = ita.ita_adaptive(y, mask, 12, 1, g)
    assert mus == [1.0]
    assert abs(lams[0] - lam) <= 1e-12 * lam
    assert np.abs(xa - x1).max() <= 1e-12 * np.abs(x1).max()


def test_every_iterate_keeps_exactly_k():
    # lambda_i mu_i is the (k+1)-th magnitude of V = X + mu dX, so exactly k
    # entries of V lie above it and survive the threshold.
    shape = (32, 32)
    k = 15
    g, xt, mask, y = _scene(STRESS, shape, 20, 0.5, seed=51)
    m = mask.astype(float)
    x = np.zeros(shape, complex)
    for it in range(1, 6):
        xn, _, mus, lams = ita.ita_adaptive(y, mask, k, it, g)
        dx = csa.M(m * (y - csa.G(x, g)), g)
        v = x + mus[-1] * dx
        sigma = lams[-1] * mus[-1]  # (rounded once by the division and product)
        a = np.abs(v)
        assert np.count_nonzero(a > sigma * (1 + 1e-12)) == k
        assert np.count_nonzero(a >= sigma * (1 - 1e-12)) == k + 1
        assert np.count_nonzero(xn) == k
        x = xn


@pytest.mark.parametrize("params", [STRIP, STRESS])
def test_exact_recovery_of_a_noiseless_sparse_scene(params):
    # y = m o G x* with k nonzeros and 60 % sampling: the iteration with the
    # true k converges to x* itself (the threshold tends to 0 with the residual).
    shape = (32, 32)
    g, xt, mask, y = _scene(params, shape, 4, 0.6, seed=3, noisy=False)
    x, res, mus, lams = ita.ita_adaptive(y, mask, 4, 60, g)
    assert np.linalg.norm(x - xt) <= 1e-9 * np.linalg.norm(xt)
    assert (x != 0).sum() == 4 and np.all((x != 0) == (xt != 0))
    assert all(mu >= 1.0 for mu in mus)
