"""Physics pins for the oracle: focusing of exact point-target echoes.

These fix the phase screens (signs, SRC, bulk RCMC, residual phase) by
what the paper and SAR theory say a matched-filter focusing chain must do:
Section III.B (M H ~ I), the error model eq. (apobs) x~ = p_eps o x + s_eps,
and the matched-filter point response printed in Section V.A.2 for the
Table 2 simulation parameters.
"""

import os

import numpy as np
import pytest

import inputs
from oracle import csa, metrics, sim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def _focus(params, shape, targets):
    rows, cols, sig = zip(*targets)
    y = sim.echo(params, shape, rows, cols, sig)
    return csa.M(y, csa.Geometry(params, shape))


def test_table2_matched_filter_point_response():
    # Section V.A.2: RDA (matched filter, full samples): PSLR -13.32 dB and
    # IRW 15 samples (x16) in both directions.  The CSA chain is a matched
    # filter too, so it must give the same point response.
    gold = _golden("mf_point_response_table2.txt")
    p = inputs.RADAR_TABLE2_SIM
    x = _focus(p, (128, 256), [(64, 128, 1.0)])
    pk = np.unravel_index(int(np.argmax(np.abs(x))), x.shape)
    assert pk == (64, 128)
    r = metrics.point_response(x, pk, chip=int(gold["chip"]), factor=int(gold["upsample"]))
    assert abs(r["pslr_r"] - gold["pslr_range_db"]) < 0.3
    assert abs(r["pslr_a"] - gold["pslr_azimuth_db"]) < 0.3
    assert abs(r["irw_r"] - gold["irw_range_samples"]) <= 1
    assert abs(r["irw_a"] - gold["irw_azimuth_samples"]) <= 1


def test_stripmap_point_target_resolution_and_phase():
    # Focused peak at the true pixel; IRW = 0.886 * (sampling rate /
    # bandwidth) samples in each axis (rect spectra), PSLR of a sinc
    # (-13.26 dB); the two stationary-phase constants cancel, so the peak
    # carries the target's phase; a unit-norm echo with spectral fill
    # beta_r * beta_a focuses to a peak of sqrt(beta_r beta_a) |sigma|.
    p = inputs.RADAR_STRIPMAP
    sigma = 0.8 * np.exp(0.7j)
    x = _focus(p, (256, 256), [(100, 140, sigma)])
    pk = np.unravel_index(int(np.argmax(np.abs(x))), x.shape)
    assert pk == (100, 140)
    beta_r = p["Kr"] * p["Tp"] / p["fs"]
    beta_a = p["ba"] / p["prf"]
    assert abs(abs(x[pk]) - abs(sigma) * np.sqrt(beta_r * beta_a)) < 0.01
    assert abs(np.angle(x[pk] / sigma)) < 0.01
    r = metrics.point_response(x, pk)
    assert abs(r["irw_r_frac"] - 16 * 0.886 / beta_r) < 0.5
    assert abs(r["irw_a_frac"] - 16 * 0.886 / beta_a) < 0.5
    assert abs(r["pslr_r"] + 13.26) < 0.3
    assert abs(r["pslr_a"] + 13.26) < 0.3


@pytest.mark.parametrize("col", [40, 512, 980])
def test_range_variant_focusing_stress_geometry(col):
    # Large, range-variant migration (about 31 range cells at the band edge):
    # chirp scaling, bulk RCMC and the residual phase must all be right for a
    # target at the near edge, centre and far edge of a wide swath to focus
    # at its pixel with its phase.  A sign error in any of the three, or a
    # missing chirp-scaling step, moves or smears the peak (amplitude < 0.2).
    p = inputs.RADAR_LBAND_STRESS
    sigma = np.exp(0.3j)
    x = _focus(p, (256, 1024), [(128, col, sigma)])
    pk = np.unravel_index(int(np.argmax(np.abs(x))), x.shape)
    assert pk == (128, col)
    assert abs(x[pk]) > 0.65
    assert abs(np.angle(x[pk] / sigma)) < (0.025 if col == 512 else 0.06)
    r = metrics.point_response(x, pk)
    assert 14 <= r["irw_r"] <= 16
    assert 16 <= r["irw_a"] <= 20


def test_brute_force_exact_observation_vs_G():
    # Dense exact observation H (eq. (ob2d), exact slant range) against the
    # dense approximated observation G on a 32 x 32 grid.  Eq. (apobs):
    # M H e_k = p_eps o e_k + s_eps, i.e. every pixel focuses back to
    # itself with a small phase error, and the focused response agrees with
    # the exact matched filter H^H H e_k up to side-lobe differences.
    # Bounds measured once on this grid and frozen (parity-approximate).
    p = inputs.RADAR_TABLE2_SIM
    shape = (32, 32)
    n = shape[0] * shape[1]
    H = sim.dense_H(p, shape)
    g = csa.Geometry(p, shape)
    Gd = np.empty((n, n), complex)
    for k in range(n):
        e = np.zeros(n, complex)
        e[k] = 1.0
        Gd[:, k] = csa.G(e.reshape(shape), g).ravel()
    MH = Gd.conj().T @ H
    HH = H.conj().T @ H
    assert np.all(np.argmax(np.abs(MH), axis=0) == np.arange(n))
    d = np.diag(MH)
    assert np.max(np.abs(np.angle(d))) < 0.01           # p_eps: phase error
    assert 0.93 < np.min(np.abs(d)) and np.max(np.abs(d)) < 0.97
    a = MH / np.linalg.norm(MH, axis=0)
    b = HH / np.linalg.norm(HH, axis=0)
    corr = np.abs(np.sum(b.conj() * a, axis=0))
    assert corr.min() > 0.96                              # s_eps small


def test_echo_columns_have_unit_norm_before_wrapping():
    p = inputs.RADAR_STRIPMAP
    r, c, v = sim.target_echo_samples(p, (4096, 4096), 2000, 2048)
    assert abs(np.linalg.norm(v) - 1.0) < 1e-12
    # window sizes: Tp*fs range samples, ba/Ka*prf pulses
    assert abs(len(set(c.tolist())) - p["Tp"] * p["fs"]) <= 2


def test_add_noise_follows_its_snr_definition():
    # The measurement model of eq. (model): y = m o (G x + n), the noise scaled
    # so that the mean signal power over the sampled pixels is snr_db above
    # the noise power.  With unit-modulus "noise" the added power is exactly
    # s^2 on every sampled pixel, which pins the scale; unsampled pixels are 0.
    rng = np.random.default_rng(3)
    shape = (16, 24)
    clean = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    mask = rng.random(shape) < 0.4
    phase = np.exp(2j * np.pi * rng.random(shape))
    for snr in (0.0, 10.0, 20.0, 35.0):
        y = sim.add_noise(clean, mask, snr, phase)
        assert np.all(y[~mask] == 0)
        added = np.abs(y[mask] - clean[mask]) ** 2
        p_sig = np.mean(np.abs(clean[mask]) ** 2)
        np.testing.assert_allclose(added, p_sig / 10 ** (snr / 10), rtol=1e-12)
        assert 10 * np.log10(p_sig / np.mean(added)) == pytest.approx(snr, abs=1e-9)
    # Gaussian noise of unit variance: the realised SNR is within sampling error
    n = inputs.circular_noise((256, 256), 7)
    big = rng.standard_normal((256, 256)) + 1j * rng.standard_normal((256, 256))
    m = np.ones((256, 256), dtype=bool)
    y = sim.add_noise(big, m, 20.0, n)
    snr = 10 * np.log10(np.mean(np.abs(big) ** 2) / np.mean(np.abs(y - big) ** 2))
    assert snr == pytest.approx(20.0, abs=0.05)
    # no sampled pixel: nothing to scale against, all zeros
    assert np.all(sim.add_noise(clean, np.zeros(shape, dtype=bool), 20.0, phase) == 0)
