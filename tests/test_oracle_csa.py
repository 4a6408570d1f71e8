"""Pins for the oracle's focusing chain M and approximated observation G.

Theorem 1 (Section III.C): G is linear with G^H = M; rules i)-ii) of
Section III.C make every step of M invertible, so G = M^{-1}.  The phase
screens are pinned against the paper's frequency-domain matched filters of
eq. (amf) in their parabolic limit, and against the matrix (Kronecker) form
of the proof of Theorem 1 built with an independent DFT.
"""

import numpy as np
import pytest

import inputs
from oracle import csa

P = inputs.RADAR_STRIPMAP
SHAPES = [(16, 16), (24, 32), (64, 48)]


def _vdot(a, b):
    return np.vdot(a.ravel(), b.ravel())


@pytest.mark.parametrize("shape", SHAPES)
def test_adjoint_identity(shape):
    # <G x, y> = <x, M y>  (Theorem 1), FP64 to 1e-12.
    g = csa.Geometry(P, shape)
    x = inputs.random_complex(shape, seed=11)
    y = inputs.random_complex(shape, seed=12)
    lhs = _vdot(csa.G(x, g), y)
    rhs = _vdot(x, csa.M(y, g))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y)


@pytest.mark.parametrize("shape", SHAPES)
def test_inverse_and_unitarity(shape):
    g = csa.Geometry(P, shape)
    y = inputs.random_complex(shape, seed=21)
    my = csa.M(y, g)
    assert abs(np.linalg.norm(my) - np.linalg.norm(y)) <= 1e-12 * np.linalg.norm(y)
    np.testing.assert_allclose(csa.G(my, g), y, atol=1e-12)
    np.testing.assert_allclose(csa.M(csa.G(y, g), g), y, atol=1e-12)


def test_linearity():
    shape = (16, 24)
    g = csa.Geometry(P, shape)
    a = inputs.random_complex(shape, seed=1)
    b = inputs.random_complex(shape, seed=2)
    s, t = 0.3 - 1.2j, 2.0 + 0.5j
    np.testing.assert_allclose(csa.G(s * a + t * b, g),
                               s * csa.G(a, g) + t * csa.G(b, g), atol=1e-12)


def test_kronecker_matrix_form():
    # Proof of Theorem 1: vec(G(X)) = F_eta^H P1* F_tau^H P2* F_tau P3* F_eta vec(X)
    # with F_eta acting on columns and F_tau on rows of X.  Built here with
    # numpy's FFT of the identity (an independent DFT), row-major vec.
    na, nr = 8, 12
    g = csa.Geometry(P, (na, nr))
    fa = np.fft.fft(np.eye(na), norm="ortho")
    fr = np.fft.fft(np.eye(nr), norm="ortho")
    Fa = np.kron(fa, np.eye(nr))       # acts along axis 0 of a row-major vec
    Fr = np.kron(np.eye(na), fr)       # acts along axis 1
    p1, p2, p3 = (np.diag(s.ravel()) for s in g.screens())
    Gm = Fa.conj().T @ p1.conj() @ Fr.conj().T @ p2.conj() @ Fr @ p3.conj() @ Fa
    Mm = Fa.conj().T @ p3 @ Fr.conj().T @ p2 @ Fr @ p1 @ Fa
    x = inputs.random_complex((na, nr), seed=5)
    np.testing.assert_allclose(csa.G(x, g).ravel(), Gm @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(csa.M(x, g).ravel(), Mm @ x.ravel(), atol=1e-12)
    np.testing.assert_allclose(Gm.conj().T, Mm, atol=1e-12)


def test_screens_are_unimodular():
    g = csa.Geometry(P, (32, 64))
    for s in g.screens():
        np.testing.assert_allclose(np.abs(s), 1.0, atol=1e-13)


def test_zero_doppler_row_reduces_to_range_matched_filter():
    # At f_eta = 0: D = 1, Km = Kr, so Phi1 = 1 and Phi2 = exp(+i pi f^2/Kr),
    # the matched filter of an up-chirp (eq. (amf) P_tau, sign reading).
    g = csa.Geometry(P, (32, 128))
    p1, p2, _ = g.screens()
    np.testing.assert_allclose(p1[0], 1.0, atol=1e-14)
    want = np.exp(1j * np.pi * g.f_tau ** 2 / P["Kr"])
    np.testing.assert_allclose(p2[0], want, atol=1e-12)


def test_azimuth_filter_parabolic_limit():
    # At the reference range (no residual phase) and small Doppler, Phi3 is
    # exp(i 4 pi R0/lambda) times eq. (amf)'s P_eta = exp(-i pi f^2 / Ka),
    # Ka = 2 V^2 / (lambda R0); the next term is O(f^4) (< 2e-3 rad here).
    na, nr = 256, 64
    g = csa.Geometry(P, (na, nr))
    _, _, p3 = g.screens()
    j = nr // 2
    r0 = g.r0[j]
    assert abs(r0 - P["r_ref"]) < 1e-6
    ka = 2 * P["v"] ** 2 / (g.lam * r0)
    f = g.f_eta
    band = np.abs(f) <= P["ba"] / 2
    got = p3[band, j] * np.exp(-4j * np.pi * r0 / g.lam)
    want = np.exp(-1j * np.pi * f[band] ** 2 / ka)
    assert np.max(np.abs(np.angle(got / want))) < 2e-3
    # and the quartic term is really there (not a pure parabola)
    assert np.max(np.abs(np.angle(got / want))) > 1e-5


def test_km_reduces_without_src():
    g0 = csa.Geometry(inputs.params_with(P, src=0), (64, 16))
    np.testing.assert_array_equal(g0.Km, P["Kr"])
    g1 = csa.Geometry(P, (64, 16))
    assert g1.Km[0] == P["Kr"]
    assert np.all(g1.Km[1:] != P["Kr"])


@pytest.mark.parametrize("shape", [(16, 32), (48, 24)])
def test_column_restricted_operators(shape):
    g = csa.Geometry(P, shape)
    x = inputs.random_complex(shape, seed=9)
    cols = [0, 3, shape[1] - 1]
    np.testing.assert_allclose(csa.M_cols(x, g, cols), csa.M(x, g)[:, cols], atol=1e-12)
    np.testing.assert_allclose(csa.G_cols(x, g, cols), csa.G(x, g)[:, cols], atol=1e-12)


def test_nonzero_doppler_centroid_rejected():
    with pytest.raises(ValueError):
        csa.Geometry(inputs.params_with(P, f_dc=10.0), (8, 8))
