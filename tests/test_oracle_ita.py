"""Pins for the oracle's thresholding and iteration (eqs. (L12), (th2d),
Algorithm 1, Section IV.B)."""

import numpy as np
import pytest

import inputs
from oracle import csa, ita

P = inputs.RADAR_STRIPMAP


def test_soft_threshold_special_cases():
    sig = 0.5
    v = np.array([0.0, 0.5, -0.5, 0.3j, 2.0, -3.0j, 3 + 4j, 0.4 - 0.3j])
    out = ita.soft_threshold(v, sig)
    assert out[0] == 0                      # x = 0 -> 0
    assert out[1] == 0 and out[2] == 0      # |x| = sigma -> 0 (either branch)
    assert out[3] == 0                      # below threshold
    assert out[7] == 0                      # |x| = 0.5 exactly
    np.testing.assert_allclose(out[4], 1.5)
    np.testing.assert_allclose(out[5], -2.5j)
    np.testing.assert_allclose(out[6], (3 + 4j) / 5 * 4.5)   # phase kept


def test_soft_threshold_real_line_is_textbook():
    # Restricted to reals, e_{1,sigma} is sgn(x) max(|x| - sigma, 0).
    x = np.linspace(-3, 3, 601)
    want = np.sign(x) * np.maximum(np.abs(x) - 0.7, 0.0)
    np.testing.assert_allclose(ita.soft_threshold(x, 0.7).real, want, atol=1e-15)


def test_soft_threshold_is_prox_of_l1():
    # prox property: S(v) minimises 1/2|u - v|^2 + sigma |u| (brute force
    # over a fine grid of complex u near the answer).
    g = inputs.rng(3)
    for _ in range(20):
        v = complex(*g.normal(size=2))
        s = 0.6
        u0 = ita.soft_threshold(np.array([v]), s)[0]
        f = lambda u: 0.5 * abs(u - v) ** 2 + s * abs(u)
        grid = u0 + (np.linspace(-0.05, 0.05, 41)[:, None]
                     + 1j * np.linspace(-0.05, 0.05, 41)[None, :])
        assert f(u0) <= np.min(f(grid)) + 1e-12


def _problem(shape, k, rate, seed, noise_snr=None):
    g = csa.Geometry(P, shape)
    rows, cols, sig = inputs.point_targets(shape, k, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    m = inputs.random_mask(shape, rate, seed=seed + 100)
    y = m * csa.G(xt, g)
    if noise_snr is not None:
        from oracle import sim
        y = sim.add_noise(csa.G(xt, g), m, noise_snr,
                          inputs.circular_noise(shape, seed + 200))
    return g, xt, m, y


def test_first_iteration_from_zero():
    # Algorithm 1 with X^(0) = 0: R^(0) = m o y, so X^(1) = E(mu M(m o y)).
    g, xt, m, y = _problem((32, 48), 5, 0.5, 1, noise_snr=20)
    lam = 0.05
    x1, hist = ita.ita(y, m, lam, 1, g)
    want = ita.soft_threshold(csa.M(m * y, g), lam)
    np.testing.assert_allclose(x1, want, atol=1e-14)
    np.testing.assert_allclose(hist[0], np.vdot(m * y, m * y).real)


def test_full_mask_is_one_step_lasso():
    # mask = 1 and mu = 1: G is unitary, so X^(t) = S_lambda(M y) for every
    # t >= 1 (the LASSO solution of an orthonormal design).  A wrong residual
    # sign or a G that is not M^{-1} breaks the fixed point.
    shape = (32, 32)
    g = csa.Geometry(P, shape)
    y = inputs.random_complex(shape, seed=5)
    lam = 0.8
    want = ita.soft_threshold(csa.M(y, g), lam)
    for iters in (1, 2, 5):
        x, _ = ita.ita(y, np.ones(shape, bool), lam, iters, g)
        np.testing.assert_allclose(x, want, atol=1e-12)


@pytest.mark.parametrize("mu", [1.0, 0.6])
def test_objective_decreases(mu):
    # ISTA with step mu <= 1/||m G||^2 = 1 is a majorise-minimise scheme for
    # 1/2||m o (y - G x)||^2 + lambda ||x||_1: the objective never increases.
    g, xt, m, y = _problem((32, 32), 6, 0.4, 2, noise_snr=20)
    lam = 0.03
    x = np.zeros_like(y)
    prev = ita.objective(x, y, m, lam, g)
    for _ in range(15):
        x, _ = ita.ita(y, m, lam, 1, g, mu=mu, x0=x)
        cur = ita.objective(x, y, m, lam, g)
        assert cur <= prev + 1e-12
        prev = cur


def test_kkt_at_convergence():
    # Optimality of the LASSO: c = M(m o (y - G x*)) satisfies |c_p| <= lambda
    # off the support and c_p = lambda x*_p / |x*_p| on it.
    g, xt, m, y = _problem((32, 32), 5, 0.5, 3, noise_snr=25)
    lam = 0.02
    x, _ = ita.ita(y, m, lam, 3000, g)
    c = csa.M(m * (y - csa.G(x, g)), g)
    on = np.abs(x) > 0
    assert on.any()
    assert np.max(np.abs(c[~on])) <= lam * (1 + 1e-6)
    np.testing.assert_allclose(c[on], lam * x[on] / np.abs(x[on]), atol=1e-7)


def test_exact_recovery_noiseless_sparse():
    # Noiseless y = m o G x_true with k << (rate * n): decreasing lambda by
    # continuation recovers the exact support and x_true to 1e-6.
    g, xt, m, y = _problem((64, 64), 8, 0.5, 3)
    lam = ita.lambda_from_sparsity(y, m, 8, g)
    x = None
    for _ in range(12):
        x, _ = ita.ita(y, m, lam, 60, g, x0=x)
        lam *= 0.3
    assert set(np.flatnonzero(x)) == set(np.flatnonzero(xt))
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) < 1e-6


def test_lambda_rule_keeps_k_largest():
    # Section IV.B: with lambda = |b(0)|_(k+1) / mu, the first iterate keeps
    # exactly the k largest entries of b(0) = mu M(m o y).
    g, xt, m, y = _problem((32, 32), 7, 0.5, 4, noise_snr=20)
    k = 7
    lam = ita.lambda_from_sparsity(y, m, k, g)
    x1, _ = ita.ita(y, m, lam, 1, g)
    assert np.count_nonzero(x1) == k


def test_residual_history_decreases_for_exact_data():
    g, xt, m, y = _problem((32, 32), 4, 0.6, 6)
    _, hist = ita.ita(y, m, 1e-3, 30, g)
    assert hist[-1] < 1e-2 * hist[0]


def test_entries_outside_the_mask_are_ignored():
    # Theta selects the measured samples (eq. (model)); what y holds at an
    # unsampled position is not data: a NaN or a large value there changes
    # nothing, for the fixed and the adaptive iteration and for lambda.
    shape = (32, 48)
    g = csa.Geometry(P, shape)
    y = inputs.random_complex(shape, seed=21)
    mask = inputs.random_mask(shape, 0.5, seed=22)
    clean = np.where(mask, y, 0)
    dirty = clean.copy()
    off = np.argwhere(~mask)
    dirty[tuple(off[0])] = np.nan
    dirty[tuple(off[1])] = 1e30 + 1e30j
    x1, h1 = ita.ita(clean, mask, 0.05, 4, g)
    x2, h2 = ita.ita(dirty, mask, 0.05, 4, g)
    assert np.array_equal(x1, x2) and h1 == h2
    assert ita.lambda_from_sparsity(dirty, mask, 10, g) == ita.lambda_from_sparsity(clean, mask, 10, g)
    a1 = ita.ita_adaptive(clean, mask, 10, 3, g)
    a2 = ita.ita_adaptive(dirty, mask, 10, 3, g)
    assert np.array_equal(a1[0], a2[0]) and a1[1:] == a2[1:]
    # a NaN at a sampled position does propagate (it is data)
    bad = clean.copy()
    bad[tuple(np.argwhere(mask)[0])] = np.nan
    assert not np.all(np.isfinite(ita.ita(bad, mask, 0.05, 1, g)[1]))


def test_warm_start_splits_the_iteration():
    # Algorithm 1 is a fixed-point iteration of X alone: n1 iterations, then
    # n2 more from X^(n1), are the same arithmetic as n1 + n2 iterations
    # (bit for bit in the oracle), residual norms included.
    shape = (32, 64)
    g = csa.Geometry(P, shape)
    rng = np.random.default_rng(17)
    x = np.zeros(shape, dtype=np.complex128)
    idx = rng.choice(x.size, 40, replace=False)
    x.flat[idx] = rng.normal(size=40) + 1j * rng.normal(size=40)
    mask = inputs.random_mask(shape, 0.5, seed=18)
    y = np.where(mask, csa.G(x, g), 0)
    lam = 0.05
    x7, h7 = ita.ita(y, mask, lam, 7, g)
    x3, h3 = ita.ita(y, mask, lam, 3, g)
    x34, h34 = ita.ita(y, mask, lam, 4, g, x0=x3)
    assert np.array_equal(x34, x7) and h3 + h34 == h7
    # the warm start really starts there: from X^(0) = 0 it differs
    x4, _ = ita.ita(y, mask, lam, 4, g)
    assert not np.allclose(x4, x7)


def test_trace_records_the_iterates_norms():
    # trace["l1"][t] and trace["nnz"][t] are ||X^(t+1)||_1 and the nonzero
    # count of X^(t+1), the iterate a solve of t + 1 iterations returns.
    shape = (32, 32)
    g = csa.Geometry(P, shape)
    mask = inputs.random_mask(shape, 0.6, seed=21)
    y = np.where(mask, inputs.random_complex(shape, seed=22), 0)
    tr = {}
    ita.ita(y, mask, 0.4, 5, g, trace=tr)
    assert len(tr["l1"]) == len(tr["nnz"]) == 5
    for t in range(5):
        xt, _ = ita.ita(y, mask, 0.4, t + 1, g)
        assert tr["l1"][t] == float(np.sum(np.abs(xt)))
        assert tr["nnz"][t] == int(np.count_nonzero(xt))
        assert 0 < tr["nnz"][t] < xt.size  # the threshold is active
    # full mask: X^(t) = S(M y) for every t (M G = I), so the trace is flat
    ones = np.ones(shape, dtype=bool)
    tr = {}
    ita.ita(inputs.random_complex(shape, seed=23), ones, 0.4, 3, g, trace=tr)
    assert abs(tr["l1"][0] - tr["l1"][2]) <= 1e-12 * tr["l1"][0]
    assert tr["nnz"][0] == tr["nnz"][2]
