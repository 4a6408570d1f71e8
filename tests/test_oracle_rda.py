"""Pins of the oracle's range-Doppler chain (oracle/rda.py; eqs. (RDA),
(RCMCs), (CD), (apob), Theorem 1): adjointness with the gather and the
scatter written separately, the interpolation matrices by brute force,
exact special cases of the interpolation, the point response the paper
prints for its matched filter (Section V.A.2, which is this chain), the
stripmap resolution and phase, and the direction of the migration
correction where it matters."""

import os

import numpy as np
import pytest

import inputs
from oracle import ita, metrics, rda, sim

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
STRIP = inputs.RADAR_STRIPMAP
STRESS = inputs.RADAR_LBAND_STRESS


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


@pytest.mark.parametrize("params,shape,taps", [
    (STRIP, (32, 64), 8), (STRIP, (48, 24), 4), (STRESS, (64, 128), 8), (STRESS, (32, 256), 16),
])
def test_theorem1_G_is_the_adjoint_of_M(params, shape, taps):
    # <G x, y> = <x, M y>: C (a gather) and D (a scatter) are written
    # separately, so this checks D = C^T and the reversed order of eq. (apob).
    # The stress geometry migrates by tens of samples and wraps.
    rg = rda.RdaGeometry(params, shape, taps)
    x = inputs.random_complex(shape, seed=1)
    y = inputs.random_complex(shape, seed=2)
    lhs = np.vdot(rda.G(x, rg), y)
    rhs = np.vdot(x, rda.M(y, rg))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_interpolation_matrices_by_brute_force():
    # Row by row, the matrix of D (built from unit vectors) is the transpose of
    # that of C, and each row of C holds exactly K nonzero sinc weights at
    # K consecutive (cyclic) positions.
    shape = (8, 40)
    rg = rda.RdaGeometry(STRESS, shape, 6)
    n = shape[1]
    for i in (0, 3, 5):
        cm = np.zeros((n, n))
        dm = np.zeros((n, n))
        for j in range(n):
            e = np.zeros((1, n), complex)
            e[0, j] = 1.0
            cm[:, j] = rda.rcmc(e, rg.delta[i:i + 1], 6)[0].real
            dm[:, j] = rda.rcmc_transpose(e, rg.delta[i:i + 1], 6)[0].real
        assert np.allclose(dm, cm.T, rtol=0, atol=1e-15)
        pos = np.arange(n) + rg.delta[i]
        for j in range(n):
            nz = np.flatnonzero(np.abs(cm[j]) > 0)
            p = int(np.floor(pos[j]))
            want = sorted((p + np.arange(-2, 4)) % n)
            if pos[j] != p:  # (an integer position puts zeros on the other taps)
                assert sorted(nz) == want
            assert abs(cm[j, (p + 0) % n] - np.sinc(pos[j] - p)) < 1e-15


def test_interpolation_special_cases():
    n = 64
    v = inputs.random_complex((1, n), seed=3)
    # no migration: the identity (sinc at the other integers is 0 to rounding)
    assert np.allclose(rda.rcmc(v, np.zeros((1, n)), 8), v, rtol=0, atol=1e-15)
    # an integer migration m: the cyclic shift U[j] = V[j + m]
    for m in (1, 5, -3, 70):
        u = rda.rcmc(v, np.full((1, n), float(m)), 8)
        assert np.allclose(u, np.roll(v, -m, axis=1), rtol=0, atol=1e-15)
    # the zero-Doppler row of a real geometry has D = 1: no migration
    rg = rda.RdaGeometry(STRIP, (16, 32))
    assert np.all(rg.delta[0] == 0.0)


def test_fractional_shift_of_a_tone():
    # Truncated sinc interpolation of a periodic tone e^(2 pi i nu n) at
    # n + s approximates e^(2 pi i nu (n + s)); the error falls as taps are
    # added (measured: <= 0.07 with 8 taps, <= 0.011 with 64, |nu| <= 0.3).
    n = 256
    for taps, bound in ((8, 0.07), (64, 0.012)):
        for m in (13, 26, 51, 77):
            nu, s = m / n, 0.37
            v = np.exp(2j * np.pi * nu * np.arange(n))[None, :]
            u = rda.rcmc(v, np.full((1, n), s), taps)
            want = np.exp(2j * np.pi * nu * (np.arange(n) + s))
            assert np.abs(u[0] - want).max() <= bound, (taps, m)
            # a shift in the wrong direction is far off
            bad = np.exp(2j * np.pi * nu * (np.arange(n) - s))
            assert np.abs(u[0] - bad).max() > 0.2


def test_table2_point_response_printed_by_the_paper():
    # Section V.A.2: the matched filter (RDA) response on the Table 2
    # simulation parameters: PSLR -13.32 dB and IRW 15 samples (x16) in
    # both directions.
    gold = _golden("mf_point_response_table2.txt")
    p = inputs.RADAR_TABLE2_SIM
    shape = (128, 256)
    y = sim.echo(p, shape, [64], [128], [1.0])
    x = rda.M(y, rda.RdaGeometry(p, shape))
    pk = np.unravel_index(int(np.argmax(np.abs(x))), shape)
    assert pk == (64, 128)
    r = metrics.point_response(x, pk, chip=int(gold["chip"]), factor=int(gold["upsample"]))
    assert abs(r["pslr_r"] - gold["pslr_range_db"]) < 0.3
    assert abs(r["pslr_a"] - gold["pslr_azimuth_db"]) < 0.3
    assert abs(r["irw_r"] - gold["irw_range_samples"]) <= 1
    assert abs(r["irw_a"] - gold["irw_azimuth_samples"]) <= 1


def test_stripmap_point_target_resolution_and_phase():
    # Peak at the true pixel, phase arg(sigma) - 4 pi R0 / lambda_w (P_eta
    # carries no constant phase), IRW 0.886 x sampling rate / bandwidth in
    # each axis and a sinc PSLR (-13.26 dB) within the interpolation error.
    p = STRIP
    shape = (256, 256)
    sigma = 0.8 * np.exp(0.7j)
    rg = rda.RdaGeometry(p, shape)
    x = rda.M(sim.echo(p, shape, [100], [140], [sigma]), rg)
    pk = np.unravel_index(int(np.argmax(np.abs(x))), shape)
    assert pk == (100, 140)
    ph = np.angle(x[pk] / sigma * np.exp(4j * np.pi * rg.g.r0[140] / rg.g.lam))
    assert abs(ph) < 0.02
    beta_r = p["Kr"] * p["Tp"] / p["fs"]
    beta_a = p["ba"] / p["prf"]
    r = metrics.point_response(x, pk)
    assert abs(r["irw_r_frac"] - 16 * 0.886 / beta_r) < 0.5
    assert abs(r["irw_a_frac"] - 16 * 0.886 / beta_a) < 0.5
    assert abs(r["pslr_r"] + 13.26) < 0.4
    assert abs(r["pslr_a"] + 13.26) < 0.4


@pytest.mark.parametrize("col", [40, 512, 980])
def test_migration_correction_direction(col):
    # Stress geometry (up to about 48 samples of migration, varying along
    # range): the correction as defined peaks at the true pixel and higher
    # than with no correction or with the migration reversed.
    shape = (256, 1024)
    y = sim.echo(STRESS, shape, [128], [col], [1.0])
    peaks = []
    for sgn in (1.0, 0.0, -1.0):
        rg = rda.RdaGeometry(STRESS, shape)
        rg.delta = sgn * rg.delta
        x = rda.M(y, rg)
        peaks.append((np.abs(x).max(), np.unravel_index(int(np.argmax(np.abs(x))), shape)))
    assert peaks[0][1] == (128, col)
    assert peaks[0][0] > 1.3 * peaks[1][0] and peaks[0][0] > 1.3 * peaks[2][0]


def test_G_inverts_M_up_to_the_interpolation_error():
    # G = M^H is only close to M^-1: on a band-limited echo, G(M y) returns y
    # within the interpolation error (measured 0.12 for the stripmap echo;
    # frozen at 0.15), and more taps bring it closer.
    shape = (128, 128)
    y = sim.echo(STRIP, shape, [40, 90], [30, 100], [1.0, 0.5j])
    errs = []
    for taps in (8, 32):
        rg = rda.RdaGeometry(STRIP, shape, taps)
        errs.append(np.linalg.norm(rda.G(rda.M(y, rg), rg) - y) / np.linalg.norm(y))
    assert errs[0] <= 0.15 and errs[1] < errs[0]


def test_iteration_runs_on_the_range_doppler_chain():
    # The solver oracle takes either chain: on y = m o G(x*) built with the
    # range-Doppler G, the adaptive iteration recovers x* itself (the
    # iteration only needs G and its adjoint M), and X(1) = S(M(m o y)).
    from oracle import ita
    shape = (32, 32)
    rg = rda.RdaGeometry(STRIP, shape)
    rows, cols, sig = inputs.point_targets(shape, 4, seed=3)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, 0.6, seed=4)
    y = mask * rda.G(xt, rg)
    x1, _ = ita.ita(y, mask, 0.3, 1, rg)
    assert np.abs(x1 - ita.soft_threshold(rda.M(y, rg), 0.3)).max() <= 1e-12
    x, *_ = ita.ita_adaptive(y, mask, 4, 80, rg)
    assert np.linalg.norm(x - xt) <= 1e-8 * np.linalg.norm(xt)


def test_bilinear_upsampling_closed_forms():
    # The second reading of the 16-fold interpolation of Section V.A.2
    # (bilinear interpolation of the chip's magnitude).  A single nonzero
    # pixel becomes the triangle 1 - |i| / f; its 3 dB width counts the
    # samples with (1 - |i| / f)^2 >= 1/2, i.e. |i| <= f (1 - 2^-1/2): 9 at
    # f = 16, and it has no side lobe.
    chip = np.zeros((16, 16), dtype=np.complex128)
    chip[8, 8] = 2.0j
    up = metrics.upsample_linear_magnitude(chip, 16)
    assert up.shape == (241, 241)
    cut = up[8 * 16, :]
    i = np.arange(cut.size) - 8 * 16
    np.testing.assert_allclose(cut, 2.0 * np.clip(1.0 - np.abs(i) / 16.0, 0.0, None), atol=1e-15)
    assert metrics.irw_samples(cut) == 2 * int(np.floor(16 * (1.0 - 2.0 ** -0.5))) + 1 == 9
    r = metrics.point_response_linear(np.pad(chip, 40), (48, 48))
    assert r["irw_r"] == r["irw_a"] == 9 and r["pslr_r"] == r["pslr_a"] == -np.inf
    # a positive plane is reproduced exactly (bilinear is exact on it) ...
    a, b = np.meshgrid(np.arange(16.0), np.arange(16.0), indexing="ij")
    up = metrics.upsample_linear_magnitude(1.0 + 0.5 * a + 0.25 * b, 4)
    ta = np.arange(up.shape[0]) / 4.0
    tb = np.arange(up.shape[1]) / 4.0
    np.testing.assert_allclose(up, 1.0 + 0.5 * ta[:, None] + 0.25 * tb[None, :], rtol=1e-14)
    # ... and the axes are not swapped: a ramp along axis 0 only
    up = metrics.upsample_linear_magnitude(np.repeat(np.arange(4.0)[:, None], 3, axis=1), 2)
    np.testing.assert_allclose(up[:, 0], np.arange(7) / 2.0)
    np.testing.assert_allclose(up[3, :], np.full(5, 1.5))


def test_super_resolution_three_targets_oracle():
    # Section V.A.2 (resolving ability): the adaptive ITA on the range-Doppler
    # operator (CSRDA) separates three unit targets 12 samples apart in
    # azimuth and in range from 10 % of the samples, with k = 600: the three
    # largest pixels are the targets and the image between them is low.
    p = inputs.RADAR_TABLE2_SIM
    shape = (128, 128)
    c = (64, 64)
    rows, cols = [c[0], c[0] + 12, c[0]], [c[1], c[1], c[1] + 12]
    y = sim.echo(p, shape, rows, cols, np.exp(1j * np.array([0.7, 2.1, -1.3])))
    mask = inputs.random_mask(shape, 0.10, seed=43)
    x, _, _, _ = ita.ita_adaptive(np.where(mask, y, 0), mask, 600, 100, rda.RdaGeometry(p, shape))
    a = np.abs(x)
    top = np.argsort(a.ravel())[::-1][:3]
    got = sorted(tuple(int(t) for t in np.unravel_index(i, shape)) for i in top)
    assert got == sorted(zip(rows, cols))
    assert a[c[0] + 6, c[1]] < 0.1 * a[c] and a[c[0], c[1] + 6] < 0.1 * a[c]
    # the matched filter on the same samples does not: its side lobes and
    # aliasing leave pixels away from the targets above 10 % of the peak
    mf = np.abs(rda.M(np.where(mask, y, 0), rda.RdaGeometry(p, shape)))
    far = mf.copy()
    far[c[0] - 8:c[0] + 21, c[1] - 8:c[1] + 21] = 0
    assert far.max() > 0.1 * mf.max()
