"""Radar parameter sets, as plain SI numbers.

Field names follow the stripmap model of the paper (Section II.A): carrier
``fc`` (the paper's f0), range chirp rate ``Kr``, pulse duration ``Tp`` (t_s),
range sampling rate ``fs`` (F_r), pulse repetition frequency ``prf`` (F_a),
effective radar velocity ``v`` (V), reference slant range ``r_ref`` (R_c, the
scene-centre range), processed Doppler bandwidth ``ba`` and Doppler centroid
``f_dc``.  ``src`` selects secondary range compression in the chirp-scaling
chain (1 = on).
"""

# Stripmap C-band parameters of the synthetic workloads: fc 5.3 GHz,
# bandwidth 30 MHz over a 10 us pulse, fs 36 MHz, PRF 1700 Hz, v 7100 m/s,
# R0 850 km.  The paper's Table 2 gives no azimuth bandwidth; 0.8 * PRF is
# used (about a 9.25 m antenna).
RADAR_STRIPMAP = dict(
    fc=5.3e9,
    Kr=30e6 / 10e-6,
    Tp=10e-6,
    fs=36e6,
    prf=1700.0,
    v=7100.0,
    r_ref=850e3,
    ba=0.8 * 1700.0,
    f_dc=0.0,
    src=1,
)

# Simulation column of the paper's Table 2 (Section V): R_c 20 km,
# V 350 m/s, squint 0, f0 5000 MHz, PRF 175 Hz, Kr 37.5 MHz/us, Tr 2 us,
# Fr 75 MHz.  The table has no Doppler bandwidth; the printed matched-filter
# azimuth IRW (15 samples at x16) corresponds to about 0.95 * PRF.
RADAR_TABLE2_SIM = dict(
    fc=5000e6,
    Kr=37.5e12,
    Tp=2e-6,
    fs=75e6,
    prf=175.0,
    v=350.0,
    r_ref=20e3,
    ba=0.95 * 175.0,
    f_dc=0.0,
    src=1,
)

# A low-frequency, slow-platform geometry with large, strongly range-variant
# range cell migration.  Not from the paper: used only to make the
# chirp-scaling and residual-phase terms of the focusing chain matter in the
# oracle's focusing checks (with the C-band sets above their effect is well
# below one resolution cell).
RADAR_LBAND_STRESS = dict(
    fc=1.25e9,
    Kr=20e6 / 4e-6,
    Tp=4e-6,
    fs=24e6,
    prf=500.0,
    v=120.0,
    r_ref=6e3,
    ba=0.8 * 500.0,
    f_dc=0.0,
    src=1,
)


def params_with(base, **changes):
    """A copy of a parameter dict with some fields replaced."""
    out = dict(base)
    for k, val in changes.items():
        if k not in out:
            raise KeyError(f"unknown radar parameter {k!r}")
        out[k] = val
    return out
