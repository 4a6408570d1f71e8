"""Pins of the oracle gradient (oracle/grad.py): the analytic screen
derivatives and the product-rule tangents of M and G against FP64 central
differences, the reverse-mode ITA gradient against central differences of
the loss, and closed forms of special cases."""

import numpy as np
import pytest

import inputs
from oracle import csa, grad, ita, sim

STRIP = inputs.RADAR_STRIPMAP
STRESS = inputs.RADAR_LBAND_STRESS  # wide Doppler band: D far from 1, large SRC


def _fd_params(params, name, rel):
    th = grad.ka_of(params) if name == "Ka" else params["Kr"]
    h = rel * th
    kw = lambda t: {name: t}
    return grad.with_theta(params, **kw(th + h)), grad.with_theta(params, **kw(th - h)), h


def _richardson(f, h):
    """Central difference of f at 0 with the O(h^2) term cancelled:
    (4 D(h/2) - D(h)) / 3, D(s) = (f(s) - f(-s)) / 2s."""
    d1 = (f(h) - f(-h)) / (2.0 * h)
    d2 = (f(h / 2) - f(-h / 2)) / h
    return (4.0 * d2 - d1) / 3.0


def _theta_fn(params, name, fn):
    """s -> fn(params with theta (1 + s))."""
    th = grad.ka_of(params) if name == "Ka" else params["Kr"]
    return lambda s: fn(grad.with_theta(params, **{name: th * (1.0 + s)})), th


@pytest.mark.parametrize("params", [STRIP, STRESS, inputs.params_with(STRESS, src=0)])
@pytest.mark.parametrize("name", ["Ka", "Kr"])
def test_arg_derivatives_match_central_differences(params, name):
    shape = (32, 64)
    g = csa.Geometry(params, shape)
    d = grad.arg_derivatives(g)[name]
    # relative step 1e-4: truncation O(1e-8), while 1/D - 1 for D near 1
    # loses digits to cancellation in the arguments themselves
    pp, pm, h = _fd_params(params, name, 1e-4)
    gp, gm = csa.Geometry(pp, shape), csa.Geometry(pm, shape)
    for k, (fa, fb) in enumerate(((gp.arg1, gm.arg1), (gp.arg2, gm.arg2), (gp.arg3, gm.arg3))):
        a, b = fa(), fb()
        fd = (a - b) / (2.0 * h)
        # plus the rounding of the arguments themselves (up to 1.9e8 rad)
        tol = 1e-6 * np.abs(fd).max() + 8 * np.finfo(float).eps * np.abs(a).max() / h
        assert np.abs(d[k] - fd).max() <= tol, (name, k)


def test_with_theta_round_trips():
    ka = grad.ka_of(STRIP)
    p = grad.with_theta(STRIP, Ka=ka)
    assert abs(p["v"] - STRIP["v"]) <= 1e-9 * STRIP["v"]
    # K_a = 2 V^2 / (lambda r_ref) at the stripmap parameters (about 2097 Hz/s)
    assert 2000.0 < ka < 2200.0


@pytest.mark.parametrize("name", ["Ka", "Kr"])
def test_tangents_match_central_differences(name):
    shape = (16, 32)
    params = STRESS
    g = csa.Geometry(params, shape)
    d = grad.arg_derivatives(g)[name]
    r = inputs.random_complex(shape, seed=3)
    mr, dmr = grad.M_tangent(r, g, d)
    gr, dgr = grad.G_tangent(r, g, d)
    assert np.allclose(mr, csa.M(r, g)) and np.allclose(gr, csa.G(r, g))
    fm, th = _theta_fn(params, name, lambda p: csa.M(r, csa.Geometry(p, shape)))
    fg, _ = _theta_fn(params, name, lambda p: csa.G(r, csa.Geometry(p, shape)))
    fd_m = _richardson(fm, 1e-6) / th
    fd_g = _richardson(fg, 1e-6) / th
    assert np.linalg.norm(dmr - fd_m) <= 1e-6 * np.linalg.norm(fd_m)
    assert np.linalg.norm(dgr - fd_g) <= 1e-6 * np.linalg.norm(fd_g)
    # G = M^-1 for every theta, so dG M + G dM = 0
    _, dg_of_m = grad.G_tangent(csa.M(r, g), g, d)
    assert np.linalg.norm(dg_of_m + csa.G(dmr, g)) <= 1e-9 * np.linalg.norm(dmr)


def _problem(params, shape, seed, k=12, rate=0.6):
    g = csa.Geometry(params, shape)
    rows, cols, sig = inputs.point_targets(shape, k, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, rate, seed=seed + 1)
    y = sim.add_noise(csa.G(xt, g), mask, 20.0, inputs.circular_noise(shape, seed + 2))
    lam = 0.5 * ita.lambda_from_sparsity(y, mask, k, g)
    return xt, y, mask, lam


@pytest.mark.parametrize("params", [STRIP, STRESS])
def test_gradient_matches_central_differences_smooth(params):
    # lambda = 0 with a partial mask: the unrolled iteration is smooth (no
    # threshold kinks), so central differences pin every component tightly.
    shape = (32, 32)
    K = 5
    xt, y, mask, _ = _problem(params, shape, seed=7)
    L, (ybar, lbar, kabar, krbar) = grad.loss_and_grad(y, mask, 0.0, K, params, shape, xt)
    f = lambda p=params, yy=y: grad.loss(yy, mask, 0.0, K, p, shape, xt)
    for name, got in (("Ka", kabar), ("Kr", krbar)):
        # step 1e-5: the stripmap Phi3 argument (1.9e8 rad) rounds at 3e-8 rad
        fl, th = _theta_fn(params, name, lambda p: f(p=p))
        fd = _richardson(fl, 1e-5) / th
        assert abs(got - fd) <= 1e-5 * abs(fd), (name, got, fd)
    dirn = mask * inputs.random_complex(shape, seed=11)
    dirn *= np.linalg.norm(y) / np.linalg.norm(dirn)
    fd = _richardson(lambda s: f(yy=y + s * dirn), 1e-6)
    got = float(np.sum(ybar.real * dirn.real + ybar.imag * dirn.imag))
    assert abs(got - fd) <= 1e-6 * abs(fd)
    assert np.abs(ybar[~mask]).max() == 0.0


def _tangent_of_loss(y, mask, lam, K, params, shape, xt, dy, dlam, dargs):
    """Forward-mode derivative of L = ||X(K) - x*||^2 along (dy, dlam, dtheta):
    (X, dX) carried through every iteration with the threshold's Jacobian
    applied to the tangent (no transposition anywhere)."""
    g = csa.Geometry(params, shape)
    m = mask.astype(float)
    x = np.zeros(shape, complex)
    dx = np.zeros(shape, complex)
    for _ in range(K):
        gx, dgx = grad.G_tangent(x, g, dargs)
        r = m * (y - gx)
        dr = m * (dy - csa.G(dx, g) - dgx)
        mr, dmr = grad.M_tangent(r, g, dargs)
        v = x + mr
        dv = dx + csa.M(dr, g) + dmr
        a = np.abs(v)
        on = a > lam
        xn = np.zeros_like(v)
        dxn = np.zeros_like(v)
        xn[on] = v[on] * (1.0 - lam / a[on])
        # d[v (1 - lam/|v|)] = dv (1 - lam/|v|) + v lam Re(conj(v) dv)/|v|^3 - v/|v| dlam
        vv, dd, aa = v[on], dv[on], a[on]
        dxn[on] = (dd * (1.0 - lam / aa) + vv * lam * (np.conj(vv) * dd).real / aa ** 3
                   - vv / aa * dlam)
        x, dx = xn, dxn
    return 2.0 * float(np.sum(((x - xt).conj() * dx).real))


@pytest.mark.parametrize("params", [STRIP, STRESS])
def test_reverse_mode_equals_forward_mode(params):
    # With the threshold active (lambda > 0) finite differences meet its
    # kinks; the reverse-mode gradient is pinned instead by the forward-mode
    # tangent of the same map along each direction (the two must agree to
    # rounding), and lambda and y by central differences.
    shape = (32, 32)
    K = 5
    xt, y, mask, lam = _problem(params, shape, seed=7)
    L, (ybar, lbar, kabar, krbar) = grad.loss_and_grad(y, mask, lam, K, params, shape, xt)
    g = csa.Geometry(params, shape)
    zero = np.zeros(shape)
    zargs = (zero, zero, zero)
    dd = grad.arg_derivatives(g)
    for name, got in (("Ka", kabar), ("Kr", krbar)):
        want = _tangent_of_loss(y, mask, lam, K, params, shape, xt, 0 * y, 0.0, dd[name])
        assert abs(got - want) <= 1e-9 * abs(want), name
    want = _tangent_of_loss(y, mask, lam, K, params, shape, xt, 0 * y, 1.0, zargs)
    assert abs(lbar - want) <= 1e-9 * abs(want)
    dirn = mask * inputs.random_complex(shape, seed=11)
    want = _tangent_of_loss(y, mask, lam, K, params, shape, xt, dirn, 0.0, zargs)
    got = float(np.sum(ybar.real * dirn.real + ybar.imag * dirn.imag))
    assert abs(got - want) <= 1e-9 * abs(want)
    # lambda and y by central differences (kinks are rare at these steps)
    f = lambda yy=y, ll=lam: grad.loss(yy, mask, ll, K, params, shape, xt)
    fd = _richardson(lambda s: f(ll=lam * (1.0 + s)), 1e-6) / lam
    assert abs(lbar - fd) <= 1e-5 * abs(fd)
    fd = _richardson(lambda s: f(yy=y + s * dirn), 1e-6)
    assert abs(got - fd) <= 1e-5 * abs(fd)


def test_closed_forms_full_mask_lambda_zero():
    # mask = 1 and lambda = 0: X(t) = M y for t >= 1, so L = ||M y - x*||^2,
    # ybar = 2 G(M y - x*) and thetabar = 2 Re<M y - x*, dM y>.
    shape = (16, 32)
    params = STRESS
    g = csa.Geometry(params, shape)
    y = inputs.random_complex(shape, seed=21)
    xt = inputs.random_complex(shape, seed=22)
    ones = np.ones(shape, dtype=bool)
    for K in (1, 3):
        L, (ybar, lbar, kabar, krbar) = grad.loss_and_grad(y, ones, 0.0, K, params, shape, xt)
        e = csa.M(y, g) - xt
        assert np.allclose(ybar, 2.0 * csa.G(e, g), rtol=1e-10, atol=1e-10)
        for name, got in (("Ka", kabar), ("Kr", krbar)):
            _, dmy = grad.M_tangent(y, g, grad.arg_derivatives(g)[name])
            want = 2.0 * float(np.sum(e.real * dmy.real + e.imag * dmy.imag))
            assert abs(got - want) <= 1e-9 * abs(want), (K, name)
        # lambda = 0: dS/dsigma = -v/|v| on every nonzero pixel (only the last
        # iteration contributes, earlier adjoints vanish for a unitary G)
        v = csa.M(y, g)
        want = -float(np.sum((2 * e * np.conj(v)).real / np.abs(v)))
        assert abs(lbar - want) <= 1e-9 * abs(want)


def test_threshold_vjp_matches_finite_differences():
    rng = np.random.default_rng(5)
    v = rng.normal(size=50) + 1j * rng.normal(size=50)
    xb = rng.normal(size=50) + 1j * rng.normal(size=50)
    sigma = 0.8
    vbar, dsig = grad.threshold_vjp(v, xb, sigma)
    h = 1e-7
    for part in (1.0, 1j):
        fd = (ita.soft_threshold(v + h * part, sigma) - ita.soft_threshold(v - h * part, sigma)) / (2 * h)
        # <xb, dS> along the direction equals <vbar, direction>
        lhs = (np.conj(xb) * fd).real
        rhs = (np.conj(vbar) * part).real
        assert np.allclose(lhs, rhs, atol=1e-6)
    fd = (ita.soft_threshold(v, sigma + h) - ita.soft_threshold(v, sigma - h)) / (2 * h)
    assert abs(float(np.sum((np.conj(xb) * fd).real)) - dsig) <= 1e-6 * max(1.0, abs(dsig))
