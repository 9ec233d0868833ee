"""Host-side statistics of the translocation campaigns (Sec. 4): the most
probable time of a skewed duration histogram, the scaling exponent of
tau(N_0), replica set-up, and the per-length summary.  CPU only."""
import math

import numpy as np

from paper_0711_2665_amd import translocation as tl
from paper_0711_2665_amd.workloads import initial_chain


def test_most_probable_time_finds_the_mode_of_a_skewed_distribution():
    # lognormal durations: mode exp(mu - s^2), well below the mean exp(mu + s^2/2)
    rng = np.random.default_rng(1)
    mu, s = math.log(1000.0), 0.4
    t = rng.lognormal(mu, s, 20000)
    mode, mean = math.exp(mu - s * s), math.exp(mu + s * s / 2)
    mp, counts, edges = tl.most_probable_time(t)
    assert abs(mp - mode) < 0.08 * mode, (mp, mode)
    assert abs(t.mean() - mean) < 0.02 * mean and mean - mp > 0.15 * mode
    assert counts.sum() == t.size and edges[0] <= t.min() and edges[-1] > t.max()


def test_most_probable_time_with_given_bins_and_integer_steps():
    t = [10, 11, 11, 12, 12, 12, 30]
    mp, counts, _ = tl.most_probable_time(t, bins=np.arange(9.5, 31.5, 1.0))
    assert mp == 12.0 and counts.max() == 3
    assert math.isnan(tl.most_probable_time([])[0])


def test_scaling_exponent_recovers_a_power_law():
    N = np.array([50, 100, 200, 300, 400])
    tau = 3.7 * N ** 1.28
    a, se = tl.scaling_exponent(N, tau)
    assert abs(a - 1.28) < 1e-12 and se < 1e-10
    rng = np.random.default_rng(2)
    a2, se2 = tl.scaling_exponent(N, tau * np.exp(0.05 * rng.standard_normal(N.size)))
    assert abs(a2 - 1.28) < 4 * se2 + 1e-3 and se2 > 0


def test_replica_configs_follow_the_paper_geometry():
    # Sec. 4, Numerical Set-up: N_x x N_x/2 x N_x/2 with N_x = 80 up to 400
    # beads and 100 beyond, the wall normal to x at N_x/2 with a 3 x 3 hole,
    # kinematic viscosity 0.1, kT = 1e-4, F_drive = 0.02, gamma = 0.1
    cfgs = tl.replica_configs(50, 6)
    assert len(cfgs) == 6 and len({c["seed"] for c in cfgs}) == 6 and len({c["init_seed"] for c in cfgs}) == 6
    for k, c in enumerate(cfgs):
        assert c["shape"] == (80, 40, 40)
        assert c["wall_axis"] == 0 and c["wall_pos"] == 40 and c["pore_h"] == 3
        assert abs((c["tau"] - 0.5) / 3.0 - 0.1) < 1e-15
        assert c["kT"] == 1e-4 and c["f_drive"] == 0.02 and c["gamma"] == 0.1
        assert c["nb"] == 50 and c["replica"] == k
    assert tl.replica_configs(400, 1)[0]["shape"] == (80, 40, 40)
    assert tl.replica_configs(500, 1)[0]["shape"] == (100, 50, 50)
    # the chain starts on one side of the wall with its first bead at the pore
    c = cfgs[0]
    r, _ = initial_chain(c)
    assert (r[:, 0] < c["wall_pos"]).all()
    assert abs(r[0, 0] - (c["wall_pos"] - 1.0)) < 1e-12
    assert abs(r[0, 1] - 20.0) < 1e-12 and abs(r[0, 2] - 20.0) < 1e-12


def test_lambda_r_and_drive_of_synthetic_events():
    nobs = 25
    steps = np.array([0, 10, 20, 30])
    obs = np.zeros((steps.size, 2, nobs))
    obs[0, :, tl.OBS["R_U"]] = [4.0, 5.0]
    obs[:, :, tl.OBS["R_T"]] = [[0.0, 0.0], [1.0, 1.5], [2.0, 2.5], [3.0, 3.5]]
    obs[:, :, tl.OBS["N_r"]] = 3.0
    obs[:, :, tl.OBS["drag_U"]] = -0.01
    obs[:, :, tl.OBS["drag_T"]] = -0.02
    s = tl.summarize(dict(length=10, tX=[20, 30], obs=obs, steps=steps, f_drive=0.02))
    assert abs(s["lambda_R"] - 0.5 * (2.0 / 4.0 + 3.5 / 5.0)) < 1e-15
    assert abs(s["mean_drive"] - 0.06) < 1e-15 and abs(s["mean_drag_total"] + 0.03) < 1e-15
    # without a start sample lambda_R is not defined
    s = tl.summarize(dict(length=10, tX=[20, 30], obs=obs[1:], steps=steps[1:], f_drive=0.02))
    assert np.isnan(s["lambda_R"])


def test_summary_of_synthetic_events():
    nobs = 25
    steps = np.arange(10, 110, 10)
    obs = np.zeros((steps.size, 3, nobs))
    obs[:, :, tl.OBS["N_r"]] = 4.0
    obs[:, 1, tl.OBS["drag_U"]] = np.linspace(-1, 1, steps.size)
    obs[:, :, tl.OBS["R_T"]] = 2.5
    res = dict(length=20, tX=[55, 80, -1], obs=obs, steps=steps)
    s = tl.summarize(res)
    assert s["events"] == 2 and s["censored"] == 1 and s["mean"] == 67.5
    assert s["mean_N_r"] == 4.0 and abs(s["R_T_at_tX"] - 2.5) < 1e-15
    # replica 1's drag averaged over its samples up to t_X = 80 (steps 10..80)
    want = np.mean([np.mean(obs[steps <= 55, 0, tl.OBS["drag_U"]]), np.mean(obs[steps <= 80, 1, tl.OBS["drag_U"]]),
                    np.mean(obs[:, 2, tl.OBS["drag_U"]])])
    assert abs(s["mean_drag_U"] - want) < 1e-15
