"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars (floating point): relative L2 <= 1e-5 per operator application and
<= 1e-4 on the final ITA image.  Inputs are seeded and synthetic.
"""

import numpy as np
import pytest

import inputs
from oracle import csa, ita
from tests.helpers import point_problem, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OP_TOL = 1e-5
IMG_TOL = 1e-4
P = inputs.RADAR_STRIPMAP


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _op(shape, params=P):
    import paper_1302_3120_amd as pk
    return pk.make_operator(params, shape)


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _h(t):
    return t.cpu().numpy().astype(np.complex128)


# Shapes spanning several row groups and column tiles, non-square, mixed radix.
OP_SHAPES = [(64, 64), (128, 256), (256, 512), (512, 256), (768, 1024), (1536, 768),
             (1024, 1536), (256, 3072), (3072, 256), (2048, 2048), (8192, 64), (64, 8192)]


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_apply_G_and_GH_match_oracle(dev, shape):
    say(f"[gpu] apply_G/apply_GH {shape}")
    g = csa.Geometry(P, shape)
    op = _op(shape)
    x = inputs.random_complex(shape, seed=shape[0] + 3 * shape[1])
    y = inputs.random_complex(shape, seed=shape[0] + 5 * shape[1] + 1)
    gx = _h(op.apply_G(_d(x, dev)))
    my = _h(op.apply_GH(_d(y, dev)))
    torch.cuda.synchronize()
    e1 = rel_l2(gx, csa.G(x, g))
    e2 = rel_l2(my, csa.M(y, g))
    say(f"    rel L2  G {e1:.2e}  G^H {e2:.2e}")
    assert e1 <= OP_TOL and e2 <= OP_TOL


@pytest.mark.parametrize("shape", [(256, 256), (1024, 2048)])
def test_point_target_focuses_on_gpu(dev, shape):
    # Exact echo of one target, focused by the GPU chain: peak at the target
    # pixel with its phase (the oracle pins the physics; this checks that the
    # GPU chain reproduces it element by element too).
    say(f"[gpu] point target focus {shape}")
    from oracle import sim
    i0, j0 = shape[0] // 3, shape[1] // 2 + 7
    sig = 0.9 * np.exp(1.1j)
    y = sim.echo(P, shape, [i0], [j0], [sig])
    x = _h(_op(shape).apply_GH(_d(y, dev)))
    pk = np.unravel_index(int(np.argmax(np.abs(x))), shape)
    assert pk == (i0, j0)
    assert abs(np.angle(x[pk] / sig)) < 0.02
    assert rel_l2(x, csa.M(y, csa.Geometry(P, shape))) <= OP_TOL


def test_adjoint_and_inverse_on_gpu(dev):
    shape = (1024, 1024)
    say(f"[gpu] adjoint identity / inverse {shape}")
    op = _op(shape)
    x = _d(inputs.random_complex(shape, seed=1), dev)
    y = _d(inputs.random_complex(shape, seed=2), dev)
    gx = op.apply_G(x)
    my = op.apply_GH(y)
    lhs = torch.vdot(gx.flatten().to(torch.complex128), y.flatten().to(torch.complex128))
    rhs = torch.vdot(x.flatten().to(torch.complex128), my.flatten().to(torch.complex128))
    n = float(x.abs().pow(2).sum().sqrt() * y.abs().pow(2).sum().sqrt())
    assert abs(complex(lhs) - complex(rhs)) <= 1e-5 * n
    back = op.apply_G(op.apply_GH(y))
    assert rel_l2(_h(back), _h(y)) <= 2 * OP_TOL


def test_bitwise_deterministic(dev):
    shape = (512, 1024)
    say(f"[gpu] determinism {shape}")
    op = _op(shape)
    y = _d(inputs.random_complex(shape, seed=7), dev)
    mask = torch.from_numpy(inputs.random_mask(shape, 0.5, seed=8)).to(dev)
    bits = op.pack_mask(mask)
    a, ha = op.ita_solve(y, bits, 0.05, 12, resid=True)
    b, hb = op.ita_solve(y, bits, 0.05, 12, resid=True)
    assert torch.equal(a, b) and torch.equal(ha, hb)
    assert torch.equal(op.apply_G(y), op.apply_G(y))


def test_ita_stripmap_256_full_run(dev):
    # 256 x 256 stripmap scene: 20 point targets, exact echoes, 50 % mask,
    # 20 dB, lambda from the sparsity rule, 100 iterations.
    shape = (256, 256)
    say(f"[gpu] ITA stripmap {shape} x100")
    xt, y, mask, lam = point_problem(P, shape, 20, 0.5, 20.0, seed=1)
    g = csa.Geometry(P, shape)
    xr, hr = ita.ita(y, mask, lam, 100, g)
    op = _op(shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    xg, hg = op.ita_solve(_d(y, dev), bits, lam, 100, resid=True)
    op.sync_status()
    e = rel_l2(_h(xg), xr)
    say(f"    final image rel L2 {e:.2e}; nnz gpu {int((xg != 0).sum())} oracle {np.count_nonzero(xr)}")
    assert e <= IMG_TOL
    np.testing.assert_allclose(hg.cpu().numpy(), np.array(hr), rtol=1e-4)


@pytest.mark.parametrize("shape,iters,rate,k", [((1024, 1024), 20, 0.5, 100),
                                                 ((768, 1536), 30, 0.3, 60),
                                                 ((2048, 2048), 6, 0.3, 200)])
def test_ita_matches_oracle(dev, shape, iters, rate, k):
    say(f"[gpu] ITA {shape} x{iters} rate {rate}")
    xt, y, mask, lam = point_problem(P, shape, k, rate, 20.0, seed=5, echo="operator")
    xr, hr = ita.ita(y, mask, lam, iters, csa.Geometry(P, shape))
    op = _op(shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    xg, hg = op.ita_solve(_d(y, dev), bits, lam, iters, resid=True)
    e = rel_l2(_h(xg), xr)
    say(f"    final image rel L2 {e:.2e}")
    assert e <= IMG_TOL
    np.testing.assert_allclose(hg.cpu().numpy(), np.array(hr), rtol=1e-4)


def test_ita_first_iteration_and_full_mask_at_4096(dev):
    # Full-size (4096 x 4096) checks on sampled columns the oracle computes
    # one by one: X(1) = S(M(m o y)) with a 50 % mask, and, with mask = 1,
    # X(100) = S(M y) (fixed point of the orthonormal case).
    shape = (4096, 4096)
    cols = [0, 1, 3, 777, 2048, 4095]
    g = csa.Geometry(P, shape)
    y = inputs.random_complex(shape, seed=61)
    mask = inputs.random_mask(shape, 0.5, seed=62)
    op = _op(shape)
    lam = 0.8
    say(f"[gpu] ITA 4096^2 first iteration, 50% mask")
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    ym = np.where(mask, y, 0)
    x1 = _h(op.ita_solve(_d(ym, dev), bits, lam, 1))[:, cols]
    want1 = ita.soft_threshold(csa.M_cols(ym, g, cols), lam)
    e1 = rel_l2(x1, want1)
    say(f"    X(1) sampled columns rel L2 {e1:.2e}")
    assert e1 <= OP_TOL
    say(f"[gpu] ITA 4096^2 full mask x100")
    ones = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    x100 = _h(op.ita_solve(_d(y, dev), ones, lam, 100))[:, cols]
    want = ita.soft_threshold(csa.M_cols(y, g, cols), lam)
    e2 = rel_l2(x100, want)
    say(f"    X(100) sampled columns rel L2 {e2:.2e}")
    assert e2 <= IMG_TOL


def test_operators_at_4096_full_size(dev):
    shape = (4096, 4096)
    say(f"[gpu] apply_G/apply_GH {shape} sampled columns")
    g = csa.Geometry(P, shape)
    cols = [0, 2, 1000, 2047, 2048, 4095]
    op = _op(shape)
    x = inputs.random_complex(shape, seed=41)
    gx = _h(op.apply_G(_d(x, dev)))[:, cols]
    my = _h(op.apply_GH(_d(x, dev)))[:, cols]
    e1 = rel_l2(gx, csa.G_cols(x, g, cols))
    e2 = rel_l2(my, csa.M_cols(x, g, cols))
    say(f"    rel L2 G {e1:.2e} G^H {e2:.2e}")
    assert e1 <= OP_TOL and e2 <= OP_TOL


def test_edge_cases(dev):
    shape = (256, 512)
    say(f"[gpu] edge cases {shape}")
    g = csa.Geometry(P, shape)
    op = _op(shape)
    y = inputs.random_complex(shape, seed=9)
    yd = _d(y, dev)
    # empty mask: residual 0, image 0
    zero = op.pack_mask(torch.zeros(shape, dtype=torch.bool, device=dev))
    x, h = op.ita_solve(yd, zero, 0.1, 3, resid=True)
    assert float(x.abs().max()) == 0.0 and float(h.abs().max()) == 0.0
    # huge threshold: everything thresholded away
    ones = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    x = op.ita_solve(yd, ones, 1e6, 2)
    assert float(x.abs().max()) == 0.0
    # lambda = 0, full mask: X(t) = M y exactly (Landweber on a unitary G)
    x = _h(op.ita_solve(yd, ones, 0.0, 3))
    assert rel_l2(x, csa.M(y, g)) <= 3 * OP_TOL
    # zero input
    z = op.apply_G(torch.zeros(shape, dtype=torch.complex64, device=dev))
    assert float(z.abs().max()) == 0.0
    # in-place / aliasing is refused
    import paper_1302_3120_amd as pk
    with pytest.raises(pk.CssarError):
        op.apply_G(yd, out=yd)
    op.sync_status()


def test_nonfinite_input_is_reported(dev):
    shape = (256, 256)
    say(f"[gpu] non-finite input {shape}")
    import paper_1302_3120_amd as pk
    op = _op(shape)
    y = inputs.random_complex(shape, seed=3)
    y[10, 10] = np.nan
    ones = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    op.ita_solve(_d(y, dev), ones, 0.1, 2)
    with pytest.raises(pk.CssarError) as ei:
        op.sync_status()
    assert ei.value.code == pk.cssar.ENONFINITE
    op.sync_status()  # cleared


def test_nonfinite_outside_the_mask_is_ignored(dev):
    # Only m o y enters the method (eq. (th2d)): NaN and Inf at unsampled
    # entries are not read, on the GPU as in the oracle.  The image equals
    # the one with zeros there, bit for bit, matches the oracle's, and no
    # non-finite status is raised.
    shape = (256, 512)
    say(f"[gpu] non-finite values outside the mask {shape}")
    op = _op(shape)
    mask = inputs.random_mask(shape, 0.4, seed=5)
    y = np.where(mask, inputs.random_complex(shape, seed=4), 0)
    un = np.argwhere(~mask)
    yb = y.copy()
    yb[tuple(un[7])] = np.nan
    yb[tuple(un[100])] = np.inf
    yb[tuple(un[200])] = complex(-np.inf, np.nan)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    lam = 0.05
    xa, ha = op.ita_solve(_d(y, dev), bits, lam, 5, resid=True)
    xb, hb = op.ita_solve(_d(yb, dev), bits, lam, 5, resid=True)
    op.sync_status()
    assert torch.equal(xa, xb) and torch.equal(ha, hb)
    xo, ho = ita.ita(yb, mask, lam, 5, csa.Geometry(P, shape))
    e = rel_l2(_h(xb), xo)
    say(f"    image rel L2 vs oracle {e:.2e}")
    assert e <= 1e-4
    np.testing.assert_allclose(hb.cpu().numpy(), ho, rtol=1e-4)


def test_wide_swath_8192_sampled_columns(dev):
    # The 8192 x 8192 wide-swath configuration (all state resident): G, G^H
    # and the first ITA iterate on sampled columns the oracle computes one by
    # one (its azimuth DFTs are full 8192-point matrix products).
    shape = (8192, 8192)
    cols = [0, 1, 4095, 4096, 8191]
    say(f"[gpu] {shape} operators and X(1), sampled columns")
    g = csa.Geometry(P, shape)
    op = _op(shape)
    x = inputs.random_complex(shape, seed=81)
    gx = _h(op.apply_G(_d(x, dev)))[:, cols]
    e1 = rel_l2(gx, csa.G_cols(x, g, cols))
    del gx
    mask = inputs.random_mask(shape, 0.5, seed=82)
    xm = np.where(mask, x, 0)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    lam = 0.9
    x1 = _h(op.ita_solve(_d(xm, dev), bits, lam, 1))[:, cols]
    e2 = rel_l2(x1, ita.soft_threshold(csa.M_cols(xm, g, cols), lam))
    say(f"    rel L2 G {e1:.2e}  X(1) {e2:.2e}")
    assert e1 <= OP_TOL and e2 <= OP_TOL


def test_ita_config_2048_points_and_patches(dev):
    # The 2048 x 2048 single-scene configuration: 200 point targets plus
    # extended complex-Gaussian patches over 2 % of the pixels (echo through
    # the oracle's G), 30 % mask, 15 dB, lambda by the sparsity rule; the
    # first 10 of its iterations against the oracle on the whole image.
    from oracle import sim
    wl = inputs.workload("stripmap_2048")
    shape = wl["shape"]
    say(f"[gpu] ITA {shape} points + patches, 10 of {wl['iters']} iterations")
    g = csa.Geometry(P, shape)
    rows, cols, sig = inputs.point_targets(shape, wl["targets"], seed=wl["seed"])
    x = inputs.targets_to_image(shape, rows, cols, sig)
    x = x + inputs.extended_patches(shape, wl["patch_coverage"], seed=wl["seed"] + 1)
    mask = inputs.random_mask(shape, wl["mask_rate"], seed=wl["seed"] + 2)
    y = sim.add_noise(csa.G(x, g), mask, wl["snr_db"], inputs.circular_noise(shape, wl["seed"] + 3))
    lam = ita.lambda_from_sparsity(y, mask, int(np.count_nonzero(x)), g)
    xr, hr = ita.ita(y, mask, lam, 10, g)
    op = _op(shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    xg, hg = op.ita_solve(_d(y, dev), bits, lam, 10, resid=True)
    e = rel_l2(_h(xg), xr)
    say(f"    final image rel L2 {e:.2e}")
    assert e <= IMG_TOL
    np.testing.assert_allclose(hg.cpu().numpy(), np.array(hr), rtol=1e-4)
    # the full run stays finite and its residual settles
    xg, hg = op.ita_solve(_d(y, dev), bits, lam, wl["iters"], resid=True)
    op.sync_status()
    h = hg.cpu().numpy()
    assert np.all(np.isfinite(h)) and h[-1] <= h[0]
