"""GPU tests of the gradient through the unrolled iteration (checkpointed
forward, reverse pass, torch.autograd binding) against the FP64 oracle
gradient (oracle/grad.py, pinned by finite differences and forward-mode
tangents on the CPU).

Bar: relative error <= 1e-3 for every gradient component (the GPU runs in
FP32; supports decided in FP32 and FP64 can differ at pixels within
rounding of the threshold)."""

import numpy as np
import pytest

import inputs
from oracle import csa, grad, ita, sim
from tests.helpers import rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = inputs.RADAR_STRIPMAP
GRAD_TOL = 1e-3


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _h(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _problem(params, shape, k, rate, seed, echo):
    g = csa.Geometry(params, shape)
    rows, cols, sig = inputs.point_targets(shape, k, seed=seed)
    xt = inputs.targets_to_image(shape, rows, cols, sig)
    clean = sim.echo(params, shape, rows, cols, sig) if echo == "exact" else csa.G(xt, g)
    mask = inputs.random_mask(shape, rate, seed=seed + 1)
    y = sim.add_noise(clean, mask, 20.0, inputs.circular_noise(shape, seed + 2))
    lam = ita.lambda_from_sparsity(y, mask, k, g)
    return xt, y, mask, lam


def _gpu_grad(params, shape, xt, y, mask, lam, K, every, dev):
    """Loss ||X(K) - x*||^2 through the autograd binding; returns the loss and
    (ybar, lambdabar, Kabar, Krbar) as numpy / floats."""
    import paper_1302_3120_amd as pk
    yd = _d(y, dev).requires_grad_(True)
    lt = torch.tensor(float(lam), dtype=torch.float64, requires_grad=True)
    ka = torch.tensor(pk.ka_of(params), dtype=torch.float64, requires_grad=True)
    kr = torch.tensor(float(params["Kr"]), dtype=torch.float64, requires_grad=True)
    m = torch.from_numpy(mask).to(dev)
    x = pk.ITAUnrolled.apply(yd, lt, ka, kr, m, K, every, params)
    loss = (x - _d(xt, dev)).abs().pow(2).sum()
    loss.backward()
    return (float(loss.detach()), yd.grad.cpu().numpy().astype(np.complex128), float(lt.grad),
            float(ka.grad), float(kr.grad))


def _compare(tag, got, want):
    L, ybar, lbar, kabar, krbar = got
    wybar, wlbar, wka, wkr = want
    e_y = rel_l2(ybar, wybar)
    e_l = abs(lbar - wlbar) / abs(wlbar)
    e_a = abs(kabar - wka) / abs(wka)
    e_r = abs(krbar - wkr) / abs(wkr)
    say(f"    {tag}: rel err ybar {e_y:.2e} lambda {e_l:.2e} Ka {e_a:.2e} Kr {e_r:.2e}")
    assert e_y <= GRAD_TOL and e_l <= GRAD_TOL and e_a <= GRAD_TOL and e_r <= GRAD_TOL


def test_checkpointed_forward_equals_solve(dev):
    import paper_1302_3120_amd as pk
    shape = (256, 512)
    say(f"[gpu] checkpointed forward vs solve {shape}")
    op = pk.make_operator(P, shape)
    y = _d(inputs.random_complex(shape, seed=3), dev)
    bits = op.pack_mask(torch.from_numpy(inputs.random_mask(shape, 0.5, seed=4)).to(dev))
    ref = op.ita_solve(y, bits, 0.4, 7)
    first = None
    for every in (1, 3, 7, 10):
        x, _ = op.ita_forward(y, bits, 0.4, 7, every)
        # the checkpoint interval does not change the iterates
        if first is None:
            first = x
        assert torch.equal(x, first), every
        # the solver keeps its iterate spatially, the gradient's forward pass
        # as its azimuth spectrum (for the checkpoints): the same iteration,
        # rounded differently
        e = rel_l2(_h(x), _h(ref))
        assert e <= 1e-6, (every, e)


@pytest.mark.parametrize("params,shape,K,every", [
    (P, (128, 256), 6, 2),
    (inputs.RADAR_LBAND_STRESS, (256, 128), 5, 5),
    (P, (2048, 128), 3, 2),  # 2048-point columns: the update pass and its adjoint on variant 1
])
def test_gradient_matches_oracle(dev, params, shape, K, every):
    say(f"[gpu] gradient vs oracle {shape} K={K} every={every} fc={params['fc']:.3g}")
    xt, y, mask, lam = _problem(params, shape, 30, 0.5, seed=40, echo="operator")
    got = _gpu_grad(params, shape, xt, y, mask, lam, K, every, dev)
    _, want = grad.loss_and_grad(y, mask, lam, K, params, shape, xt)
    _compare(str(shape), got, want)


def test_gradient_independent_of_checkpoint_interval(dev):
    import paper_1302_3120_amd as pk
    shape = (256, 256)
    say(f"[gpu] gradient vs checkpoint interval {shape}")
    op = pk.make_operator(P, shape)
    xt, y, mask, lam = _problem(P, shape, 20, 0.5, seed=50, echo="operator")
    yd = _d(y, dev)
    bits = op.pack_mask(torch.from_numpy(mask).to(dev))
    gx = _d(inputs.random_complex(shape, seed=51), dev)
    res = []
    for every in (1, 4, 9):
        _, ck = op.ita_forward(yd, bits, lam, 9, every)
        res.append(op.ita_backward(yd, bits, lam, 9, every, ck, gx))
    for gy, gs in res[1:]:
        assert torch.equal(gy, res[0][0]) and torch.equal(gs, res[0][1])


def test_gradient_config_1024_k20(dev):
    # Full differentiated workload: 1024 x 1024, 100 point targets (exact
    # echoes), 50 % mask, 20 dB, K = 20, checkpoint every 5.
    wl = inputs.workload("grad_1024")
    shape = wl["shape"]
    say(f"[gpu] gradient {shape} K={wl['iters']} every={wl['every']} (oracle runs on the host)")
    xt, y, mask, lam = _problem(P, shape, wl["targets"], wl["mask_rate"], seed=wl["seed"], echo="exact")
    got = _gpu_grad(P, shape, xt, y, mask, lam, wl["iters"], wl["every"], dev)
    _, want = grad.loss_and_grad(y, mask, lam, wl["iters"], P, shape, xt)
    _compare(str(shape), got, want)


def test_backward_rejects_bad_arguments(dev):
    import paper_1302_3120_amd as pk
    shape = (128, 128)
    op = pk.make_operator(P, shape)
    y = _d(inputs.random_complex(shape, seed=1), dev)
    bits = op.pack_mask(torch.ones(shape, dtype=torch.bool, device=dev))
    with pytest.raises(pk.CssarError):
        op.ita_forward(y, bits, 0.1, 4, 0)
    with pytest.raises(pk.CssarError):
        op.ita_forward(y, bits, -0.1, 4, 2)
    x, ck = op.ita_forward(y, bits, 0.1, 4, 2)
    with pytest.raises(pk.CssarError):
        op.ita_backward(y, bits, 0.1, 0, 2, ck, x)
