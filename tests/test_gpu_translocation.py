"""Translocation campaigns on the GPU (Sec. 4): the translocation step of a
replica equals the oracle's (no noise, no bending: bitwise dynamics), every
replica of a campaign ensemble equals the same system run alone, and the
campaign driver returns its statistics."""
import numpy as np
import pytest

from paper_0711_2665_amd import translocation as tl
from paper_0711_2665_amd.workloads import initial_chain

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_translocation_step_matches_oracle(orc):
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    cfg = tl.replica_configs(12, 1, shape=(16, 16, 16), tau=1.0, kT=0.0, kappa=0.0)[0]
    r, v = initial_chain(cfg)
    o = orc.Oracle(cfg, r, v)
    o.relax(cfg["relax_substeps"], cfg["gamma_relax"])
    rr = o.beads()["r"]
    o = orc.Oracle(cfg, rr, np.zeros_like(rr))
    tx = -1
    for k in range(1, 3001):
        o.couple_step(1)
        if o.observables()[9] == 1.0:
            tx = k
            break
    assert tx > 0
    s = lbmd.Simulation(cfg, rr, None)
    s.couple_step(tx + 10)
    torch.cuda.synchronize()
    s.check()
    print(f"12 beads: oracle t_X {tx}, gpu {s.translocation_steps()[0]}", flush=True)
    assert s.translocation_steps()[0] == tx


def test_campaign_replicas_equal_runs_alone():
    torch = _torch()
    from paper_0711_2665_amd import lbmd
    res = tl.run_length(10, 4, max_steps=1500, sample_every=25, shape=(16, 16, 16), tau=1.0)
    total = int(res["steps"][-1])
    print("campaign t_X", res["tX"], "steps run", total, flush=True)
    assert res["obs"].shape == (len(res["steps"]), 4, lbmd.LB_NOBS)
    assert sum(t >= 0 for t in res["tX"]) >= 2
    for k, cfg in enumerate(res["cfgs"]):
        s = lbmd.Simulation(cfg, initial_chain(cfg)[0], precision=lbmd.LB_FP32_DEV)
        s.relax(cfg["relax_substeps"], cfg["gamma_relax"])
        s0 = s.step_count()
        s.couple_step(total)
        torch.cuda.synchronize()
        t = s.translocation_steps()[0]
        assert (t - s0 if t >= 0 else -1) == res["tX"][k], (k, t, res["tX"][k])
        s.close()
    summ = tl.summarize(res)
    assert summ["events"] == sum(t >= 0 for t in res["tX"]) and summ["censored"] == 4 - summ["events"]
    assert np.isfinite(summ["most_probable"]) and summ["mean_N_r"] >= 0.0


def test_campaign_driver_over_two_lengths():
    _torch()
    out = tl.run_campaign([8, 14], 3, max_steps=1500, sample_every=50, shape=(16, 16, 16), tau=1.0)
    print({k: v for k, v in out.items() if k != "lengths"},
          [(s["length"], s["events"], s["most_probable"]) for s in out["lengths"]], flush=True)
    assert [s["length"] for s in out["lengths"]] == [8, 14]
    assert all(s["events"] >= 1 for s in out["lengths"])
    assert np.isfinite(out["alpha"])
