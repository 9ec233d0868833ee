"""The fused MD sub-cycle (off by default; blocks of K sub-steps per
launch, each workgroup
recomputing the chain neighbours and close partners that can reach its
segment) against one launch per sub-step, through the C ABI: bit for bit on
every population and bead field, with the bead noise and bending on (both
paths run on the GPU, so no last-bit difference of libm can hide one of
arithmetic).  Cases: a short chain (one segment), long chains over several
segments with their per-step lists, an ensemble of uneven replicas replayed
from the captured graph, block lengths 10, 5 and 2, and a drifting chain
fast enough to leave the cell table's margin inside the cycle, so that
blocks fail their check and the replica is redone from the failed block by
one workgroup."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C0, initial_chain, scaled

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _state(ctx, r=0):
    torch = ctx.torch
    torch.cuda.synchronize()
    b = {k: t.cpu().numpy().copy() for k, t in ctx.beads(r).items()}
    return ctx.pops(r).double().cpu().numpy(), b


def _same(a, b, tag):
    pa, ba = a
    pb, bb = b
    diff = {k: int((ba[k] != bb[k]).sum()) for k in ("r", "v", "up", "J")}
    print(f"{tag}: pops differing {int((pa != pb).sum())}, beads {diff}", flush=True)
    assert np.array_equal(pa, pb), tag
    for k in ("r", "v", "up", "J"):
        assert np.array_equal(ba[k], bb[k]), (tag, k)


def _pair(cfg, precision, relax=300):
    from paper_0711_2665_amd import lbmd
    r, v = initial_chain(cfg)
    sims = []
    for K in (10, None):
        s = lbmd.Simulation(cfg, r, v, precision=precision)
        s.relax(relax, 1.0)
        if K is not None:
            s.md_fused(K)
        sims.append(s)
    return sims


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_fused_equals_per_substep_c0(prec):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    p = lbmd.LB_FP64 if prec == "fp64" else lbmd.LB_FP32_DEV
    fused, plain = _pair(C0, p)
    for n in (1, 5, 30):
        fused.couple_step(n)
        plain.couple_step(n)
        _same(_state(fused), _state(plain), f"c0 {prec} +{n}")
    d = fused.diagnostics()
    print("fused diagnostics", d, flush=True)
    assert d["fused_blocks"] > 0
    fused.check()
    plain.check()


@pytest.mark.parametrize("K", [10, 5, 2])
def test_fused_long_chain_block_lengths(K):
    """1100 beads (nine segments), kT and bending on, every block length."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=1100, init_seed=9)
    fused, plain = _pair(cfg, lbmd.LB_FP64)
    fused.md_fused(K)
    fused.couple_step(4)
    plain.couple_step(4)
    _same(_state(fused), _state(plain), f"1100 beads K={K}")
    d = fused.diagnostics()
    print("diagnostics", d, flush=True)


def test_fused_drifting_chain_redoes_failed_blocks():
    """A uniform drift of 2 per LB step along the wall takes every bead more
    than the fused keep radius (half the skin less the block displacement
    bound, 0.5) from where the step's lists were built, inside the cycle:
    blocks of 2 sub-steps fail their check, one workgroup redoes the cycle
    from the failed block (pairs from the cell table, or from all beads once
    the table is unusable), and the result is still bit for bit that of one
    launch per sub-step (whose lists are rebuilt inside the cycle)."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=(40, 40, 40), wall_pos=20, nb=1100, init_seed=9)
    r, v = initial_chain(cfg)
    sims = []
    for K in (2, None):
        s = lbmd.Simulation(cfg, r, v, precision=lbmd.LB_FP64)
        s.relax(300, 1.0)
        vv = np.zeros((cfg["nb"], 3))
        vv[:, 1] = 2.0
        s.beads()["v"].copy_(torch.as_tensor(vv, device=s.device))
        if K is not None:
            s.md_fused(K)
        sims.append(s)
    fused, plain = sims
    fused.couple_step(3)
    plain.couple_step(3)
    _same(_state(fused), _state(plain), "drifting 1100 beads")
    d = fused.diagnostics()
    print("diagnostics", d, flush=True)
    assert d["fused_redos"] >= 1 and d["why_moved"] >= 1


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_fused_ensemble_graph_replay(prec):
    """Uneven replicas (chains of 0 to 700 beads, one without a wall) in one
    context, replayed from the captured graph with the fused cycle, against
    the same context stepped with one launch per sub-step."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    p = lbmd.LB_FP64 if prec == "fp64" else lbmd.LB_FP32_DEV
    cfgs = [scaled(C0, shape=(32, 32, 32), nb=20, seed=3, replica=0),
            scaled(C0, shape=(40, 36, 44), wall_pos=22, nb=700, seed=4, replica=1, init_seed=4),
            scaled(C0, shape=(24, 24, 24), wall_axis=-1, wall_pos=0, pore_h=0, nb=0, replica=2),
            scaled(C0, shape=(36, 36, 36), wall_pos=18, nb=260, seed=5, replica=3, init_seed=6)]
    r0s = [initial_chain(c)[0] if c["nb"] > 0 else None for c in cfgs]
    ens = []
    for K in (10, None):
        e = lbmd.Ensemble(cfgs, r0s, precision=p)
        e.relax(300, 1.0)
        if K is not None:
            e.md_fused(K)
        ens.append(e)
    fused, plain = ens
    fused.run(6, graph=True)
    plain.run(6, graph=False)
    for k in range(len(cfgs)):
        _same(_state(fused, k), _state(plain, k), f"ensemble {prec} replica {k}")
    print("diagnostics", fused.diagnostics(), flush=True)


def test_fused_switch_is_validated():
    _torch()
    from paper_0711_2665_amd import lbmd
    s = lbmd.Simulation(C0, initial_chain(C0)[0])
    assert s.diagnostics()["fused_blocks"] == 0
    for bad in (-1, 1, 3, 20):
        with pytest.raises(lbmd.LbError):
            s.md_fused(bad)
    s.md_fused(5)
    s.md_fused(0)
    mts = scaled(C0, mts_outer=5)
    m = lbmd.Simulation(mts, initial_chain(mts)[0])
    with pytest.raises(lbmd.LbError) as e:
        m.md_fused(10)
    assert e.value.code == lbmd.LB_ERR_UNSUPPORTED
    m.md_fused(0)
