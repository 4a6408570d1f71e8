"""GPU parity of the support-change safeguard of the adaptive step
(cssar_ita_solve_safeguarded) against the FP64 oracle
(oracle.ita.ita_adaptive_safeguarded, pinned on the CPU by the full-mask
closed form, a dense brute-force bound and the descent the bound
guarantees).

Bars as for the adaptive solver: relative L2 <= 1e-4 on the final image and
the residual norms, relative 1e-5 on every accepted step mu_t and 1e-4 on
every lambda_t; the shrink counts equal.  Whether to shrink is a decision
taken on GPU-summed norms; the cases here keep every bound test at least
1e-3 away from a tie (checked on the oracle's ratios)."""

import numpy as np
import pytest

import inputs
from oracle import csa, ita, rda
from tests.helpers import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

IMG_TOL = 1e-4
MU_TOL = 1e-5
P = inputs.RADAR_STRIPMAP
STRESS = inputs.RADAR_LBAND_STRESS


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _h(t):
    return t.cpu().numpy().astype(np.complex128)


def _problem(params, shape, k_true, rate, seed, chain="csa"):
    g = csa.Geometry(params, shape) if chain == "csa" else rda.RdaGeometry(params, shape)
    rows, cols, sig = inputs.point_targets(shape, k_true, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    mask = inputs.random_mask(shape, rate, seed=seed + 1)
    clean = ita._G(xt, g)
    n = inputs.circular_noise(shape, seed + 2)
    y = mask * (clean + 0.1 * np.sqrt(np.mean(np.abs(clean) ** 2)) * n)
    return g, y, mask


def _run(op, y, mask, k, iters, dev, **kw):
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    x, mu, lam, res, s = op.ita_solve_safeguarded(_d(y, dev), bits, k, iters, **kw)
    op.sync_status()
    return _h(x), mu.cpu().numpy(), lam.cpu().numpy(), res.cpu().numpy(), s.cpu().numpy()


@pytest.mark.parametrize("params,shape,k_true,k,rate,c,kappa,bound,iters,chain", [
    (P, (256, 256), 20, 200, 0.5, 0.5, 4.0, 2, 6, "csa"),      # one shrink per iteration
    (STRESS, (128, 512), 40, 400, 0.3, 0.5, 2.5, 3, 6, "csa"),  # at the bound every iteration
    (P, (512, 256), 60, 600, 0.5, 0.4, 2.0, 2, 5, "csa"),
    (P, (256, 256), 20, 100, 0.5, 0.01, 2.0, 2, 6, "csa"),     # default constants: no shrink
    (P, (256, 256), 20, 200, 0.4, 0.5, 3.0, 2, 6, "rda"),      # range-Doppler chain
    (P, (8192, 64), 40, 300, 0.5, 0.5, 2.5, 2, 4, "csa"),      # 8192-point columns
])
def test_safeguarded_matches_oracle(dev, params, shape, k_true, k, rate, c, kappa, bound, iters, chain):
    import paper_1302_3120_amd as pk
    say(f"[gpu] safeguarded solve {shape} {chain} k={k} c={c} kappa={kappa} bound={bound}")
    g, y, mask = _problem(params, shape, k_true, rate, shape[0] + shape[1] + k_true, chain)
    wx, wres, wmu, wlam, ws, wr = ita.ita_adaptive_safeguarded(y, mask, k, iters, g, c=c, kappa=kappa,
                                                               max_shrinks=bound)
    assert not wr or np.min(np.abs(np.array(wr) - 1.0)) > 1e-3  # no near-tie in the decisions
    op = pk.make_operator(params, shape, chain=chain)
    x, mu, lam, res, s = _run(op, y, mask, k, iters, dev, c=c, kappa=kappa, max_shrinks=bound)
    e_x = rel_l2(x, wx)
    e_mu = np.max(np.abs(mu - wmu) / np.abs(wmu))
    e_lam = np.max(np.abs(lam - wlam) / np.abs(wlam))
    e_res = rel_l2(res, wres)
    say(f"    shrinks {list(s)} (oracle {ws}); rel err X {e_x:.2e} mu {e_mu:.2e} "
        f"lambda {e_lam:.2e} resid {e_res:.2e}")
    assert list(s) == list(ws)
    assert e_x <= IMG_TOL and e_mu <= MU_TOL and e_lam <= IMG_TOL and e_res <= IMG_TOL
    assert np.count_nonzero(x) == min(k, x.size)


def test_full_mask_shrinks_once_at_the_start(dev):
    # Every sample kept: omega = 1 - c after the first step, so mu_0 = 1 shrinks
    # once to 1 / (kappa (1 - c)) and X(1) = mu_0 S_sigma(M y) (closed form
    # pinned on the CPU).
    import paper_1302_3120_amd as pk
    shape, k, c, kappa = (256, 512), 300, 0.02, 3.0
    say(f"[gpu] safeguarded solve, full mask {shape} k={k}")
    g = csa.Geometry(P, shape)
    y = inputs.random_complex(shape, seed=71)
    mask = np.ones(shape, dtype=bool)
    op = pk.make_operator(P, shape)
    x, mu, lam, _, s = _run(op, y, mask, k, 1, dev, c=c, kappa=kappa)
    my = csa.M(y, g)
    a = np.abs(my)
    sg = np.sort(a.ravel())[::-1][k]
    ref = np.where(a > sg, my / np.where(a > 0, a, 1) * (a - sg), 0) / (kappa * (1 - c))
    e = rel_l2(x, ref)
    say(f"    shrinks {list(s)} mu {mu[0]:.6f} rel err X {e:.2e}")
    assert list(s) == [1]
    assert abs(mu[0] * kappa * (1 - c) - 1.0) <= 1e-6
    assert e <= IMG_TOL


def test_no_shrinks_reproduce_the_adaptive_solver(dev):
    # With the loop bound 0 the safeguarded solver takes the adaptive solver's
    # steps: the same passes on the same inputs, so mu, lambda, the residuals
    # and the image agree bit for bit.
    import paper_1302_3120_amd as pk
    shape, k, iters = (1024, 2048), 3000, 4
    say(f"[gpu] safeguarded (bound 0) against adaptive {shape} k={k}")
    g, y, mask = _problem(P, shape, 300, 0.5, seed=72)
    op = pk.make_operator(P, shape)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    yd = _d(y, dev)
    xa, mua, lama, resa = op.ita_solve_adaptive(yd, bits, k, iters)
    xs, mus, lams, ress, s = op.ita_solve_safeguarded(yd, bits, k, iters, max_shrinks=0)
    op.sync_status()
    say(f"    equal X {torch.equal(xa, xs)} mu {torch.equal(mua, mus)} lambda {torch.equal(lama, lams)} "
        f"resid {torch.equal(resa, ress)}")
    assert torch.equal(mua, mus) and torch.equal(lama, lams) and torch.equal(resa, ress)
    assert torch.equal(xa, xs) and int(s.abs().sum()) == 0


def test_at_4096_full_size(dev):
    # The headline grid: the first iteration against the oracle, then five
    # iterations with the default constants, whose properties hold at any size.
    import paper_1302_3120_amd as pk
    shape, k = (4096, 4096), 2000
    say(f"[gpu] safeguarded solve {shape} k={k}: first iteration against the oracle")
    g, y, mask = _problem(P, shape, 200, 0.5, seed=73)
    op = pk.make_operator(P, shape)
    x1, mu1, lam1, _, s1 = _run(op, y, mask, k, 1, dev)
    wx, _, wmu, wlam, ws, _ = ita.ita_adaptive_safeguarded(y, mask, k, 1, g)
    e = rel_l2(x1, wx)
    say(f"    shrinks {list(s1)} (oracle {ws}); rel err X {e:.2e}")
    assert list(s1) == list(ws) and e <= IMG_TOL
    assert abs(lam1[0] - wlam[0]) <= 1e-4 * wlam[0]
    x, mu, lam, res, s = _run(op, y, mask, k, 5, dev)
    say(f"    5 iterations: shrinks {list(s)} mu {np.round(mu, 4)} resid {np.round(res, 2)}")
    assert np.count_nonzero(x) == k
    assert np.all((s >= 0) & (s <= 2)) and np.all(np.isfinite(mu)) and np.all(mu > 0)
    assert np.all(np.isfinite(res)) and res[-1] < res[0]
    assert mu[0] == mu1[0] and lam[0] == lam1[0] and s[0] == s1[0]  # same first iteration


def test_edge_cases_and_arguments(dev):
    import paper_1302_3120_amd as pk
    shape = (128, 128)
    say(f"[gpu] safeguarded solve edge cases {shape}")
    g, y, mask = _problem(P, shape, 10, 0.5, seed=74)
    op = pk.make_operator(P, shape)
    x, mu, lam, _, s = _run(op, y, mask, 0, 3, dev)  # k = 0: nothing kept
    assert not np.any(x) and list(s) == [0, 0, 0]
    x, *_ = _run(op, np.zeros(shape), mask, 10, 3, dev)  # y = 0
    assert not np.any(x)
    n = shape[0] * shape[1]
    x, _, lam, _, _ = _run(op, y, mask, n + 5, 2, dev)  # k >= n: threshold 0, X+ = V
    wx, *_ = ita.ita_adaptive_safeguarded(y, mask, n + 5, 2, g)
    assert rel_l2(x, wx) <= IMG_TOL and np.all(lam == 0)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    yd = _d(y, dev)
    for kw in (dict(c=0.0), dict(c=1.0), dict(c=0.5, kappa=2.0), dict(max_shrinks=-1),
               dict(max_shrinks=17)):
        with pytest.raises(pk.CssarError):
            op.ita_solve_safeguarded(yd, bits, 10, 2, **kw)
    with pytest.raises(pk.CssarError):
        op.ita_solve_safeguarded(yd, bits, -1, 2)
    # the same workspace twice: the state is set up again by each call
    ws = op.workspace(3, dev)
    a = op.ita_solve_safeguarded(yd, bits, 40, 4, c=0.5, kappa=4.0, ws=ws)
    b = op.ita_solve_safeguarded(yd, bits, 40, 4, c=0.5, kappa=4.0, ws=ws)
    op.sync_status()
    assert all(torch.equal(u, v) for u, v in zip(a, b))
