"""lb_observables_static, the entry point for callers that cannot allocate:
through the C ABI it gives what lb_observables gives (the same kernels, the
same summation order, so bit for bit), on two calls in a row, the second on
a smaller context, and after the static array held a larger lattice's
partial sums."""
import numpy as np
import pytest

from paper_0711_2665_amd.workloads import C0, initial_chain, scaled

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx(shape, wall_pos, nb, steps, precision):
    from paper_0711_2665_amd import lbmd
    cfg = scaled(C0, shape=shape, wall_pos=wall_pos, nb=nb)
    r, v = initial_chain(cfg)
    s = lbmd.Simulation(cfg, r, v, precision=precision)
    s.relax(200, 1.0)
    s.couple_step(steps)
    return s


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_static_observables_equal_the_allocating_entry_point(prec):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    p = lbmd.LB_FP64 if prec == "fp64" else lbmd.LB_FP32_DEV
    big = _ctx((48, 40, 36), 18, 30, 4, p)        # 17 reduction tiles
    small = _ctx((20, 18, 16), 8, 10, 3, p)       # 2 reduction tiles
    for s in (big, small):                         # the second call: a smaller input
        want = s.observables(lbmd.LB_OBS_ALL).cpu().numpy().copy()
        out = torch.full((lbmd.LB_NOBS,), float("nan"), dtype=torch.float64, device="cuda:0")
        got = s.observables_static(out, lbmd.LB_OBS_ALL).cpu().numpy()
        torch.cuda.synchronize()
        print(prec, s.shape, "max |diff|", float(np.nanmax(np.abs(got - want))), flush=True)
        assert np.array_equal(got, want), (s.shape, got, want)
        # one group: the others stay as the caller left them
        out.fill_(-7.0)
        got = s.observables_static(out, lbmd.LB_OBS_FLUID).cpu().numpy()
        assert np.array_equal(got[:4], want[:4]) and (got[4:] == -7.0).all()
    # and once more on the large one after the small one used the array
    want = big.observables().cpu().numpy().copy()
    out = torch.empty(lbmd.LB_NOBS, dtype=torch.float64, device="cuda:0")
    assert np.array_equal(big.observables_static(out).cpu().numpy(), want)


def test_static_observables_reject_bad_masks():
    _torch()
    from paper_0711_2665_amd import lbmd
    s = _ctx((20, 18, 16), 8, 10, 1, lbmd.LB_FP64)
    import torch
    out = torch.empty(lbmd.LB_NOBS, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lbmd.LbError):
        s.observables_static(out, 32)


def test_static_observables_reject_lattices_beyond_the_limit():
    """A 512 x 256 x 514 lattice (67,371,008 nodes, 16448 reduction tiles)
    exceeds the static array: the fluid group is refused with LB_ERR_ARG,
    the groups that need no partial sums still work."""
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = dict(shape=(512, 256, 514), wall_axis=-1, wall_pos=0, pore_h=0, nb=0, tau=1.0)
    s = lbmd.Simulation(cfg, precision=lbmd.LB_FP32_DEV)
    out = torch.full((lbmd.LB_NOBS,), float("nan"), dtype=torch.float64, device="cuda:0")
    with pytest.raises(lbmd.LbError) as e:
        s.observables_static(out, lbmd.LB_OBS_FLUID)
    assert e.value.code == lbmd.LB_ERR_ARG
    got = s.observables_static(out, lbmd.LB_OBS_STEP).cpu().numpy()
    assert got[22] == 0.0 and np.isnan(got[:22]).all()
    del s
    torch.cuda.empty_cache()
