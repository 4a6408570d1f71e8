"""Pins of the oracle's support-change safeguard (oracle/ita.py:
safeguard_bound, ita_adaptive_safeguarded), the step bound of the
normalized iterative hard thresholding that Section IV.B cites for its step
mu_i, applied to the paper's soft-threshold step.  They hold independently of
the oracle's loop: the special case without shrinks, the orthonormal (full
mask) closed form, the bound on a dense brute-force operator, and the descent
the bound guarantees (a quadratic data term majorised by the step's own
proximal surrogate)."""

import numpy as np
import pytest

import inputs
from oracle import csa, ita

STRIP = inputs.RADAR_STRIPMAP


def _scene(shape, k_true, rate, seed):
    g = csa.Geometry(STRIP, shape)
    rows, cols, sig = inputs.point_targets(shape, k_true, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, rate, seed=seed + 1)
    clean = csa.G(xt, g)
    n = inputs.circular_noise(shape, seed + 2)
    y = mask * (clean + 0.1 * np.sqrt(np.mean(np.abs(clean) ** 2)) * n)
    return g, mask, y


def test_without_shrinks_it_is_the_adaptive_iteration():
    g, mask, y = _scene((32, 64), 10, 0.4, seed=41)
    a = ita.ita_adaptive(y, mask, 40, 6, g)
    b = ita.ita_adaptive_safeguarded(y, mask, 40, 6, g, c=0.5, kappa=4.0, max_shrinks=0)
    assert np.array_equal(a[0], b[0])
    assert a[1] == b[1] and a[2] == b[2] and a[3] == b[3]
    assert b[4] == [0] * 6 and b[5] == []


def test_full_mask_closed_form():
    # With every sample kept, G is unitary: ||m o G d|| = ||d|| for every d,
    # so omega = 1 - c whenever the support changes, and the normalized step
    # is 1.  The first step leaves the empty support, mu = 1 > 1 - c, one
    # shrink to mu = 1 / (kappa (1 - c)) <= 1 - c ends the loop, and
    # X(1) = S_sigma(mu M y) = mu S_{|My|_(k+1)}(M y).
    shape, k, c, kappa = (32, 32), 25, 0.02, 3.0
    g = csa.Geometry(STRIP, shape)
    y = inputs.random_complex(shape, seed=43)
    mask = np.ones(shape, dtype=bool)
    x, _, mus, lams, shrinks, ratios = ita.ita_adaptive_safeguarded(y, mask, k, 1, g, c=c, kappa=kappa)
    my = csa.M(y, g)
    s = np.sort(np.abs(my).ravel())[::-1][k]
    a = np.abs(my)
    ref = np.where(a > s, my / np.where(a > 0, a, 1) * (a - s), 0) / (kappa * (1 - c))
    assert shrinks == [1]
    assert ratios[0] == pytest.approx(1.0 / (1.0 - c), rel=1e-12)
    assert mus[0] == pytest.approx(1.0 / (kappa * (1.0 - c)), rel=1e-15)
    assert np.max(np.abs(x - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert lams[0] == pytest.approx(s, rel=1e-12)  # lambda = sigma / mu is unchanged


def test_bound_against_a_dense_operator():
    # omega from G built column by column from unit vectors (brute force)
    shape, c = (16, 16), 0.1
    g = csa.Geometry(STRIP, shape)
    n = shape[0] * shape[1]
    dense = np.empty((n, n), dtype=np.complex128)
    for j in range(n):
        e = np.zeros(n, dtype=np.complex128)
        e[j] = 1.0
        dense[:, j] = csa.G(e.reshape(shape), g).ravel()
    mask = inputs.random_mask(shape, 0.3, seed=44)
    x = inputs.random_complex(shape, seed=45)
    x_new = inputs.random_complex(shape, seed=46)
    d = (x_new - x).ravel()
    gd = mask.ravel() * (dense @ d)
    want = (1 - c) * np.vdot(d, d).real / np.vdot(gd, gd).real
    assert ita.safeguard_bound(x_new, x, mask, g, c) == pytest.approx(want, rel=1e-10)
    assert ita.safeguard_bound(x, x, mask, g, c) == np.inf  # no change: no bound


@pytest.mark.parametrize("shape,k,k_true,rate,seed,c,kappa,bound", [
    ((32, 64), 120, 10, 0.3, 47, 0.5, 2.5, 3),
    ((64, 32), 150, 15, 0.4, 50, 0.5, 4.0, 2),
])
def test_accepted_steps_descend(shape, k, k_true, rate, seed, c, kappa, bound):
    # An accepted step (mu <= omega after a support change) decreases
    # F(X) = 1/2 ||m o (y - G X)||^2 + lambda ||X||_1, lambda = sigma / mu of
    # that step, by at least c ||X+ - X||^2 / (2 mu): the data term is
    # quadratic, so it equals its expansion at X, which the bound caps by the
    # proximal surrogate that the soft threshold minimises.  A bound with the
    # wrong operator, mask or constant, or a shrink in the wrong direction,
    # accepts steps that break it.  Steps one at a time from the previous
    # iterate; the cases also take shrinks.
    g, mask, y = _scene(shape, k_true, rate, seed)
    x = np.zeros(shape, dtype=np.complex128)
    tested = shrunk = 0
    for t in range(8):
        x_new, _, mus, lams, shrinks, ratios = ita.ita_adaptive_safeguarded(
            y, mask, k, 1, g, c=c, kappa=kappa, max_shrinks=bound, x0=x if t else None)
        shrunk += shrinks[0]
        if ratios and ratios[-1] <= 1.0:
            lam, mu = lams[0], mus[0]
            d = x_new - x
            drop = ita.objective(x, y, mask, lam, g) - ita.objective(x_new, y, mask, lam, g)
            assert drop >= c * np.vdot(d, d).real / (2 * mu) * (1 - 1e-9)
            tested += 1
        x = x_new
    assert tested >= 3 and shrunk >= 2


def test_parameters_are_checked():
    g, mask, y = _scene((16, 16), 3, 0.5, seed=49)
    for c, kappa in ((0.0, 2.0), (1.0, 2.0), (0.5, 2.0), (0.1, 1.0)):
        with pytest.raises(ValueError):
            ita.ita_adaptive_safeguarded(y, mask, 3, 1, g, c=c, kappa=kappa)
