"""Translocation campaigns (Sec. 4): many replicas of each chain length driven
through the pore, run as batched ensembles on the GPU library until every
chain has crossed the wall or a step limit is reached.

For each length the campaign records every replica's translocation step
t_X (the first step after which the whole chain is past the wall plane; the
library keeps it on the device) and, every `sample_every` steps, the
ensemble's observables: the radii R_U, R_T, R_eff of the two parts, the
number of beads in the pore channel N_r, the viscous drag on the
untranslocated and translocated parts, and the hydrodynamic and electric
work rates.  From the events it forms the duration histogram, its most
probable time (the position of the histogram's maximum, which the paper
uses instead of the mean because the distributions are skewed), and the
scaling exponent alpha of tau(N_0) ~ N_0^alpha by a least-squares fit of
log tau against log N_0.  Replicas that do not translocate within the limit
are reported as censored and left out of the histograms.

The statistics functions are plain numpy and run on the host; the stepping
runs only in the library (`lbmd.Ensemble`).
"""
import math

import numpy as np

from .workloads import BASE, initial_chain

# observable indices (lb_observables)
OBS = dict(R_U=11, R_T=12, R_eff=13, dWH_dt=14, dWE_dt=15, N_r=10, translocated=9, drag_U=23, drag_T=24)


def paper_box(length):
    """The box of Sec. 4's numerical set-up: N_x x N_x/2 x N_x/2 with
    N_x = 80 for chains of up to 400 beads and 100 for longer ones."""
    nx = 80 if length <= 400 else 100
    return (nx, nx // 2, nx // 2)


def replica_configs(length, replicas, seed=2007, shape=None, **kw):
    """Replicas of one chain length on the set-up of Sec. 4: the box of
    paper_box (unless `shape` is given), the wall normal to x at
    x = N_x / 2 with a 3 x 3 pore at its centre, kinematic viscosity 0.1
    (tau = 0.8), kT = 1e-4, gamma = 0.1 and F_drive = 0.02 on the beads in
    the pore channel; one noise key and one initial walk per replica, the
    walk entirely on one side of the wall with its first bead at the pore."""
    if shape is None:
        shape = paper_box(length)
    rng = np.random.default_rng(seed + 7919 * length)
    out = []
    for k in range(replicas):
        c = dict(BASE)
        c.update(name=f"N{length}_r{k}", shape=tuple(shape), wall_axis=0, wall_pos=shape[0] // 2, pore_h=3,
                 tau=0.5 + 3.0 * 0.1, kT=1e-4, gamma=0.1, f_drive=0.02,
                 nb=length, seed=int(rng.integers(1, 2 ** 31)), replica=k, init_seed=int(rng.integers(1, 2 ** 31)))
        c.update(kw)
        out.append(c)
    return out


def most_probable_time(times, bins=None):
    """Centre of the fullest bin of the duration histogram.  Without `bins`
    the bin width follows the Freedman-Diaconis rule, 2 IQR n^(-1/3)
    (at least one step)."""
    t = np.asarray(times, dtype=np.float64)
    if t.size == 0:
        return float("nan"), None, None
    if bins is None:
        q75, q25 = np.percentile(t, [75, 25])
        width = max(1.0, 2.0 * (q75 - q25) * t.size ** (-1.0 / 3.0))
        nbins = max(1, int(math.ceil((t.max() - t.min()) / width)))
        edges = t.min() + width * np.arange(nbins + 1)
        if edges[-1] <= t.max():
            edges = np.append(edges, edges[-1] + width)
    else:
        edges = np.asarray(bins, dtype=np.float64)
    counts, edges = np.histogram(t, bins=edges)
    k = int(np.argmax(counts))
    return float(0.5 * (edges[k] + edges[k + 1])), counts, edges


def scaling_exponent(lengths, taus):
    """alpha and its standard error from the least-squares line through
    (log N_0, log tau)."""
    x = np.log(np.asarray(lengths, dtype=np.float64))
    y = np.log(np.asarray(taus, dtype=np.float64))
    if x.size < 2:
        return float("nan"), float("nan")
    A = np.vstack([x, np.ones_like(x)]).T
    coef, res, _, _ = np.linalg.lstsq(A, y, rcond=None)
    alpha = float(coef[0])
    if x.size > 2:
        s2 = float(((y - A @ coef) ** 2).sum()) / (x.size - 2)
        se = math.sqrt(s2 / float(((x - x.mean()) ** 2).sum()))
    else:
        se = float("nan")
    return alpha, se


def run_length(length, replicas, max_steps, sample_every=50, precision=None, relax=None, device="cuda:0",
               graph=True, progress=None, **kw):
    """One ensemble of `replicas` chains of `length` beads, relaxed, then
    stepped in chunks of `sample_every` until every replica has translocated
    or `max_steps` are done.  Returns the translocation steps (-1: censored),
    the sampled observables [samples, replicas, LB_NOBS] and their steps."""
    import torch
    from . import lbmd
    prec = lbmd.LB_FP32_DEV if precision is None else precision
    cfgs = replica_configs(length, replicas, **kw)
    r0s = [initial_chain(c)[0] for c in cfgs]
    ens = lbmd.Ensemble(cfgs, r0s, precision=prec, device=device)
    ens.relax(cfgs[0]["relax_substeps"] if relax is None else relax, cfgs[0]["gamma_relax"])
    step0 = ens.step_count()
    # the relaxed start is the first sample (R_U(0) of lambda_R)
    samples, when = [ens.observables().clone()], [0]
    done = 0
    while done < max_steps:
        n = min(sample_every, max_steps - done)
        ens.run(n, graph=graph)
        done += n
        samples.append(ens.observables().clone())
        when.append(ens.step_count() - step0)
        tx_now = ens.translocation_steps()
        if progress is not None and len(samples) % progress == 0:
            import sys
            print(f"N_0 = {length}: {done} steps, {sum(t >= 0 for t in tx_now)} of {replicas} translocated",
                  file=sys.stderr, flush=True)
        if all(t >= 0 for t in tx_now):
            break
    torch.cuda.synchronize()
    ens.check()
    tx = [t - step0 if t >= 0 else -1 for t in ens.translocation_steps()]
    obs = torch.stack(samples).cpu().numpy() if samples else np.zeros((0, replicas, lbmd.LB_NOBS))
    ens.close()
    return dict(length=length, cfgs=cfgs, tX=tx, obs=obs, steps=np.asarray(when), f_drive=cfgs[0]["f_drive"])


def summarize(result):
    """Statistics of one length: events, censored count, most probable and
    mean translocation time, and per-replica averages of N_r, the drags and
    the work rates while the chain was still crossing (samples up to t_X).
    lambda_R = R_T(t_X) / R_U(0) (Sec. 4.1) is averaged over the replicas
    that translocated, when the first sample is the start (step 0); the
    drive is F_drive times the mean number of beads in the channel, beside
    the mean drag on both parts."""
    tx = np.asarray(result["tX"])
    ev = tx[tx >= 0]
    mp, counts, edges = most_probable_time(ev) if ev.size else (float("nan"), None, None)
    obs, steps = result["obs"], result["steps"]
    means = {}
    for name in ("N_r", "drag_U", "drag_T", "dWH_dt", "dWE_dt", "R_eff"):
        vals = []
        for r in range(len(tx)):
            end = tx[r] if tx[r] >= 0 else np.inf
            sel = steps <= end
            if sel.any():
                vals.append(float(obs[sel, r, OBS[name]].mean()))
        means[name] = float(np.mean(vals)) if vals else float("nan")
    lam, lam_r = [], []
    start = obs.shape[0] > 0 and steps[0] == 0
    for r in range(len(tx)):
        if tx[r] >= 0 and obs.shape[0] > 0:
            k = int(np.searchsorted(steps, tx[r]))
            k = min(k, obs.shape[0] - 1)
            lam.append(obs[k, r, OBS["R_T"]])
            if start and obs[0, r, OBS["R_U"]] > 0:
                lam_r.append(obs[k, r, OBS["R_T"]] / obs[0, r, OBS["R_U"]])
    fd = result.get("f_drive", float("nan"))
    return dict(length=result["length"], events=int(ev.size), censored=int((tx < 0).sum()),
                most_probable=mp, mean=float(ev.mean()) if ev.size else float("nan"),
                histogram=(counts.tolist() if counts is not None else []),
                bin_edges=(edges.tolist() if edges is not None else []),
                R_T_at_tX=float(np.mean(lam)) if lam else float("nan"),
                lambda_R=float(np.mean(lam_r)) if lam_r else float("nan"),
                mean_drag_total=means["drag_U"] + means["drag_T"], mean_drive=fd * means["N_r"],
                **{f"mean_{k}": v for k, v in means.items()})


def run_campaign(lengths, replicas, max_steps, sample_every=50, **kw):
    """Every length in turn; returns the per-length summaries and the
    scaling exponent of the most probable times."""
    out = []
    for L in lengths:
        out.append(summarize(run_length(L, replicas, max_steps, sample_every=sample_every, **kw)))
        if kw.get("progress") is not None:
            import sys
            print(f"N_0 = {L} done: {out[-1]['events']} events", file=sys.stderr, flush=True)
    ok = [s for s in out if s["events"] > 0 and np.isfinite(s["most_probable"])]
    alpha, se = scaling_exponent([s["length"] for s in ok], [s["most_probable"] for s in ok]) if len(ok) >= 2 \
        else (float("nan"), float("nan"))
    return dict(lengths=out, alpha=alpha, alpha_stderr=se)


def campaign_markdown(out, argv, seconds):
    """A short text record of a campaign: the command, and per length the
    events, the most probable and mean t_X, the histogram, lambda_R, <N_r>,
    and the mean drag on both parts beside the drive."""
    box = paper_box(max(s["length"] for s in out["lengths"]))
    lines = ["# Translocation campaign on the set-up of Sec. 4",
             "",
             f"Box {box[0]}x{box[1]}x{box[2]} (N_x x N_x/2 x N_x/2), wall normal to x at N_x/2 with a 3x3 pore, "
             "nu = 0.1 (tau = 0.8), kT = 1e-4, gamma = 0.1, F_drive = 0.02, FP32 deviation storage, "
             f"{out['replicas']} replicas per length, at most {out['max_steps']} LB steps; {seconds:.0f} s on one GPU.",
             "",
             "Command (from the repository root):",
             "",
             "```",
             "python -m paper_0711_2665_amd.translocation " + " ".join(argv),
             "```",
             "",
             "| N_0 | events | censored | most probable t_X | mean t_X | lambda_R | <N_r> | drag U+T | drive F N_r |",
             "|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for s in out["lengths"]:
        lines.append(f"| {s['length']} | {s['events']} | {s['censored']} | {s['most_probable']:.0f} | "
                     f"{s['mean']:.0f} | {s['lambda_R']:.3f} | {s['mean_N_r']:.3f} | "
                     f"{s['mean_drag_total']:.3e} | {s['mean_drive']:.3e} |")
    lines += ["", "Histograms of t_X (counts over bin edges):", ""]
    for s in out["lengths"]:
        edges = ", ".join(f"{e:.0f}" for e in s["bin_edges"])
        lines.append(f"- N_0 = {s['length']}: counts {s['histogram']}, edges [{edges}]")
    lines += ["", f"alpha from the most probable times: {out['alpha']:.3f} +- {out['alpha_stderr']:.3f} "
              "(reported, not a target)", ""]
    return "\n".join(lines)


def main():
    import argparse
    import json
    import sys
    import time
    ap = argparse.ArgumentParser(description="translocation campaign over chain lengths (GPU)")
    ap.add_argument("--lengths", type=int, nargs="+", default=[50, 100, 200])
    ap.add_argument("--replicas", type=int, default=32)
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--json", help="write the full result here")
    ap.add_argument("--md", help="write the text record here")
    a = ap.parse_args()
    t0 = time.perf_counter()
    out = run_campaign(a.lengths, a.replicas, a.max_steps, sample_every=a.sample_every, progress=20)
    out.update(replicas=a.replicas, max_steps=a.max_steps)
    sec = time.perf_counter() - t0
    text = json.dumps(out)
    if a.json:
        with open(a.json, "w") as f:
            f.write(text)
    if a.md:
        with open(a.md, "w") as f:
            f.write(campaign_markdown(out, sys.argv[1:], sec))
    print(text)


if __name__ == "__main__":
    main()


__all__ = ["OBS", "paper_box", "replica_configs", "most_probable_time", "scaling_exponent", "run_length", "summarize",
           "run_campaign"]
