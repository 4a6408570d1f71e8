"""GPU tests of the batched solver (grouped pass kernels over many scenes,
HIP-graph replay, autotuner) through the C ABI.

Bars: bit-for-bit equality with per-scene cssar_ita_solve when both use the
default plans (the grouped kernels run the same per-line code); relative L2
<= 1e-5 against per-scene solves with autotuned plans (other FFT schedules
round differently); <= 1e-4 on the final image against the FP64 oracle.
"""

import numpy as np
import pytest

import inputs
from oracle import csa, ita
from tests.helpers import point_problem, rel_l2, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

P = inputs.RADAR_STRIPMAP


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _d(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a).astype(np.complex64)).to(dev)


def _h(t):
    return t.cpu().numpy().astype(np.complex128)


def _random_batch(shapes, seed, dev):
    """Seeded raw data and masks on the GPU (torch's generator), mask rate
    U(0.3, 0.7) per scene, lambda per scene."""
    import paper_1302_3120_amd as pk
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    ops, ys, bits, masks = [], [], [], []
    rates = np.random.default_rng(seed).uniform(0.3, 0.7, size=len(shapes))
    for (na, nr), rate in zip(shapes, rates):
        op = pk.make_operator(P, (na, nr))
        y = torch.randn(na, nr, dtype=torch.complex64, device=dev, generator=g)
        m = torch.rand(na, nr, device=dev, generator=g) < float(rate)
        ops.append(op)
        ys.append(torch.where(m, y, torch.zeros_like(y)))
        masks.append(m)
        bits.append(op.pack_mask(m))
    lams = [0.9 + 0.01 * s for s in range(len(shapes))]
    return ops, ys, masks, bits, lams


def _check_gate(desc):
    """Every plan variant of every tuned pass was run through the parity
    gate (a distance, not "-"), and the chosen one is within 1e-5 of the
    default plan's output."""
    lines = [l for l in desc.splitlines() if " gate=" in l]
    assert lines
    for l in lines:
        chosen = int(l.split(" variant=")[1].split()[0])
        gates = dict(g.split(":") for g in l.split(" gate=")[1].split(","))
        assert all(v != "-" for v in gates.values()), l
        assert float(gates[str(chosen)]) <= 1e-5, l
        say(f"    gate {l.split(' scenes=')[0]}: {gates}")


# (2048 and 4096 columns run plan variant 1 for the update / residual pass by default)
SMALL = [(256, 512), (512, 256), (768, 1024), (1024, 768), (512, 512), (256, 256), (1536, 512),
         (2048, 256), (4096, 64)]


def test_batched_equals_per_scene_bitwise(dev):
    import paper_1302_3120_amd as pk
    say(f"[gpu] batched vs per-scene, {len(SMALL)} scenes, default plans, direct launches")
    ops, ys, masks, bits, lams = _random_batch(SMALL, 11, dev)
    b = pk.make_batch(ops)
    say("    " + b.describe().replace("\n", "; "))
    for iters in (1, 2, 7):
        outs = b.ita_solve(ys, bits, lams, iters)
        for s, op in enumerate(ops):
            ref = op.ita_solve(ys[s], bits[s], lams[s], iters)
            assert torch.equal(outs[s], ref), (iters, s, SMALL[s])


def test_graph_replay_matches_direct_launches(dev):
    import paper_1302_3120_amd as pk
    say(f"[gpu] batched graph replay vs direct launches")
    ops, ys, masks, bits, lams = _random_batch(SMALL, 12, dev)
    b = pk.make_batch(ops)
    direct = b.ita_solve(ys, bits, lams, 9)
    b.set_graph(True)
    for rep in range(3):
        got = b.ita_solve(ys, bits, lams, 9)
        torch.cuda.synchronize()
        for s in range(len(SMALL)):
            assert torch.equal(got[s], direct[s]), (rep, s)
        # eager work between replays, on the same stream
        junk = torch.randn(1 << 20, device=dev).cumsum(0)
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
    # new inputs through the same graph (the argument tables are re-uploaded)
    ys2 = [y.flip(0).contiguous() for y in ys]
    b.set_graph(False)
    want = b.ita_solve(ys2, bits, lams, 6)
    b.set_graph(True)
    got = b.ita_solve(ys2, bits, lams, 6)
    for s in range(len(SMALL)):
        assert torch.equal(got[s], want[s]), s


def test_autotuned_batch_matches_oracle(dev, tmp_path):
    import paper_1302_3120_amd as pk
    shapes = [(512, 512), (512, 1024), (1024, 512)]
    say(f"[gpu] autotuned batch vs oracle {shapes}")
    probs = [point_problem(P, sh, 40, 0.5, 20.0, seed=30 + i, echo="operator")
             for i, sh in enumerate(shapes)]
    ops = [pk.make_operator(P, sh) for sh in shapes]
    b = pk.make_batch(ops)
    cache = str(tmp_path / "tune.txt")
    b.autotune(cache_path=cache)
    say("    " + b.describe().replace("\n", "; "))
    _check_gate(b.describe())
    ys = [_d(p[1], dev) for p in probs]
    bits = [op.pack_mask(torch.from_numpy(p[2]).to(dev)) for op, p in zip(ops, probs)]
    lams = [p[3] for p in probs]
    iters = 8
    outs = b.ita_solve(ys, bits, lams, iters)
    for s, (sh, p) in enumerate(zip(shapes, probs)):
        xr, _ = ita.ita(p[1], p[2], p[3], iters, csa.Geometry(P, sh))
        e = rel_l2(_h(outs[s]), xr)
        say(f"    {sh}: final image rel L2 vs oracle {e:.2e}")
        assert e <= 1e-4
    # the cache file now answers the same question without measuring
    lines = open(cache).read().splitlines()
    assert any(l.startswith("cssar-tune ") for l in lines)
    assert any(l.startswith("cssar-graph ") for l in lines)
    b2 = pk.make_batch(ops)
    b2.autotune(cache_path=cache)
    assert b2.describe() == b.describe()
    assert open(cache).read().splitlines() == lines


def test_batched_64_scene_workload(dev):
    # The 64-scene workload: each dimension from {512, 1024, 1536, 2048},
    # 100 iterations, autotuned plans and graph replay.  Checked against
    # per-scene solves (which the single-scene tests pin to the oracle), and
    # the first iterate of three scenes against the oracle on sampled columns.
    import paper_1302_3120_amd as pk
    wl = inputs.workload("batched_64")
    shapes = inputs.batched_shapes(wl["count"], wl["seed"], wl["sizes"])
    say(f"[gpu] batched_64: {len(shapes)} scenes, {sum(a * b for a, b in shapes) / 1e6:.1f} Mpx")
    ops, ys, masks, bits, lams = _random_batch(shapes, wl["seed"], dev)
    b = pk.make_batch(ops)
    b.autotune()
    say("    " + b.describe().replace("\n", "; "))
    _check_gate(b.describe())
    outs = b.ita_solve(ys, bits, lams, wl["iters"])
    b.sync_status()
    worst = 0.0
    for s, op in enumerate(ops):
        ref = op.ita_solve(ys[s], bits[s], lams[s], wl["iters"])
        num = float((outs[s] - ref).abs().pow(2).sum().sqrt())
        den = float(ref.abs().pow(2).sum().sqrt())
        worst = max(worst, num / max(den, 1e-30))
    say(f"    worst rel L2 batched vs per-scene over 64 scenes: {worst:.2e}")
    assert worst <= 1e-5
    x1 = b.ita_solve(ys, bits, lams, 1)
    for s in (0, 17, 63):
        sh = shapes[s]
        cols = [0, 3, sh[1] // 2, sh[1] - 1]
        y = _h(ys[s])
        want = ita.soft_threshold(csa.M_cols(y, csa.Geometry(P, sh), cols), lams[s])
        e = rel_l2(_h(x1[s])[:, cols], want)
        say(f"    scene {s} {sh}: X(1) sampled columns rel L2 vs oracle {e:.2e}")
        assert e <= 1e-5


def test_batch_rejects_bad_arguments(dev):
    import paper_1302_3120_amd as pk
    ops = [pk.make_operator(P, (256, 256)), pk.make_operator(P, (512, 256))]
    b = pk.make_batch(ops)
    ys = [torch.zeros(256, 256, dtype=torch.complex64, device=dev),
          torch.zeros(512, 256, dtype=torch.complex64, device=dev)]
    bits = [op.pack_mask(torch.ones(op.shape, dtype=torch.bool, device=dev)) for op in ops]
    with pytest.raises(pk.CssarError):
        b.ita_solve(ys, bits, [0.1, -1.0], 3)
    with pytest.raises(pk.CssarError):
        b.ita_solve(ys, bits, [0.1, 0.1], 0)
    with pytest.raises(pk.CssarError):
        b.ita_solve(ys, bits, [0.1, 0.1], 3, outs=ys)
    out = b.ita_solve(ys, bits, [0.1, 0.1], 3)
    assert all(float(o.abs().max()) == 0.0 for o in out)


def test_batched_nonfinite_scene_is_reported(dev):
    # A NaN at a sampled entry of one scene's y spreads through that scene's
    # iteration; the call's check of every X^(iters) reports that scene (the
    # others stay finite and equal their per-scene solves), and the flag is
    # cleared by the report.  A NaN outside the mask is ignored.
    import paper_1302_3120_amd as pk
    shapes = [(256, 256), (512, 256), (256, 512)]
    say(f"[gpu] batched non-finite check {shapes}")
    ops, ys, masks, bits, lams = _random_batch(shapes, 21, dev)
    b = pk.make_batch(ops)
    bad = ys[1].clone()
    i, j = (int(t) for t in torch.nonzero(masks[1])[5])
    bad[i, j] = float("nan")
    outs = b.ita_solve([ys[0], bad, ys[2]], bits, lams, 4)
    with pytest.raises(pk.CssarError) as e:
        b.sync_status()
    assert e.value.code == pk.cssar.ENONFINITE and "scene 1" in str(e.value)
    for s in (0, 2):
        assert torch.equal(outs[s], ops[s].ita_solve(ys[s], bits[s], lams[s], 4))
    b.sync_status()  # cleared
    # NaN outside the mask: not read
    un = ys[2].clone()
    i, j = (int(t) for t in torch.nonzero(~masks[2])[3])
    un[i, j] = float("nan")
    outs = b.ita_solve([ys[0], ys[1], un], bits, lams, 4)
    b.sync_status()
    assert torch.equal(outs[2], ops[2].ita_solve(ys[2], bits[2], lams[2], 4))
