"""BF16 + incremental sampling vs FP32 + the paper's n-pass full recompute, at equal cut.

Every form trains the same MADE (same initial weights, Adam settings and, per training
seed, the same Philox seed) on the same Max-Cut instance.  The best cut found so far is
tracked after every update and the wall time to first reach a target cut is measured
without evaluation time (the hitting-time protocol of Table 5: evaluate after each update,
exclude evaluation time).  Training runs over several seeds; the target is the lowest final
best cut over all forms and seeds, so that every run reaches it.

The n-pass sampler computes the same conditionals as the incremental one in exact
arithmetic, but not the same FP32 roundings: a draw whose uniform lies within rounding of
its probability can come out differently, and from the first differing draw on the two
trajectories diverge.  The two forms are therefore statistically equivalent, not
trajectory-identical (``agreement`` reports, step by step, the measured fraction of equal
strings of the two forms over the first ``--plain-steps`` steps).

Two ways to give the n-pass form's time to the target:
  * ``--direct``: run it for every step, like the other forms, and measure its hitting time
    (affordable at n = 500: ``--workload maxcut500 --steps 100 --direct``);
  * otherwise (n = 10^4, seconds per n-pass step): an estimate, the FP32 incremental form's
    steps to the target for each seed times the measured n-pass step time, reported with its
    spread over the seeds and marked ``derived``.

    python -m paper_2106_13308_amd.equal_cut --workload maxcut10k_h2000 --steps 500 --seeds 0 1 2
    python -m paper_2106_13308_amd.equal_cut --workload maxcut500 --steps 100 --seeds 0 1 2 --direct

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

import torch

from . import binding as B
from . import inputs
from .vqmc import Trainer

FORMS = {"bf16_incremental": (B.BF16, 0), "fp32_incremental": (B.F32, 0), "fp32_plain": (B.F32, 1)}


def build(workload: str, wdtype: int, algo: int, lr: float, seed: int):
    w = inputs.WORKLOADS[workload]
    inst = inputs.make_instance(w)
    made = B.Made.from_dense(inst["W1"], inst["b1"], inst["W2"], inst["b2"], inst["degrees"], wdtype=wdtype)
    H = B.Hamiltonian.from_edges(w.n, inst["edges"], inst["weights"])
    return w, Trainer(made, H, w.B, seed=seed, lr=lr, algo=algo)


def run(trainer: Trainer, steps: int, log_every: int = 0, tag: str = ""):
    """Train; return the per-step trajectory (wall time excludes the stats readback)."""
    traj = []
    wall = 0.0
    best = None
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trainer.step(log=False)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        st = B.stats_to_dict(trainer.bufs.stats)            # evaluation: not timed
        best = st["min"] if best is None else min(best, st["min"])
        rec = {"step": i + 1, "wall_s": wall, "mean_E": st["mean"], "min_E": st["min"], "best_E": best,
               "best_cut": (trainer.H.W_tot - best) / 2, "mean_cut": (trainer.H.W_tot - st["mean"]) / 2}
        traj.append(rec)
        if log_every and (i + 1) % log_every == 0:
            print(f"[equal_cut] {tag} step {i + 1}: best cut {rec['best_cut']:.0f} mean cut "
                  f"{rec['mean_cut']:.1f} wall {wall:.2f}s", file=sys.stderr, flush=True)
    return traj


def first_reach(traj, target):
    for r in traj:
        if r["best_cut"] >= target:
            return r
    return None


def spread(xs):
    xs = [float(x) for x in xs]
    return {"mean": statistics.fmean(xs), "min": min(xs), "max": max(xs), "values": xs}


def agreement(workload: str, lr: float, seed: int, steps: int):
    """Step both FP32 forms side by side from the same state; measured fraction of equal strings
    and whether the energies agree, and the n-pass step times."""
    _, ti = build(workload, B.F32, 0, lr, seed)
    _, tp = build(workload, B.F32, 1, lr, seed)
    times, rows = [], []
    for i in range(steps):
        ti.step(log=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tp.step(log=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rows.append({"step": i + 1,
                     "strings_equal_fraction": float((ti.bufs.S == tp.bufs.S).all(dim=1).float().mean()),
                     "energies_equal": bool(torch.equal(ti.bufs.E, tp.bufs.E))})
        print(f"[equal_cut] fp32 n-pass vs incremental step {i + 1}: {times[-1]:.3f}s {rows[-1]}",
              file=sys.stderr, flush=True)
    return rows, times


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="maxcut10k_h2000")
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0, 1, 2])
    ap.add_argument("--plain-steps", type=int, default=2, help="side-by-side n-pass steps (agreement, step time)")
    ap.add_argument("--direct", action="store_true", help="train the n-pass form for every step too")
    ap.add_argument("--log-every", type=int, default=50)
    a = ap.parse_args()

    forms = ["bf16_incremental", "fp32_incremental"] + (["fp32_plain"] if a.direct else [])
    trajs = {f: {} for f in forms}
    w = None
    for f in forms:
        wd, algo = FORMS[f]
        for s in a.seeds:
            w, tr = build(a.workload, wd, algo, a.lr, 2 + s)
            trajs[f][s] = run(tr, a.steps, a.log_every, f"{f} seed {s}")
            W_tot = tr.H.W_tot
            del tr
    agree, plain_times = agreement(a.workload, a.lr, 2 + a.seeds[0], a.plain_steps)
    t_plain = statistics.fmean(plain_times)

    target = min(t[-1]["best_cut"] for f in forms for t in trajs[f].values())
    out = {"workload": w.name, "n": w.n, "h": w.h, "B": w.B, "steps": a.steps, "lr": a.lr,
           "training_seeds": a.seeds, "W_tot": W_tot, "target_cut": target,
           "target_rule": "lowest final best cut over all forms and seeds", "forms": {}}
    for f in forms:
        hits = {s: first_reach(t, target) for s, t in trajs[f].items()}
        out["forms"][f] = {
            "final_best_cut": spread(t[-1]["best_cut"] for t in trajs[f].values()),
            "final_mean_cut": spread(t[-1]["mean_cut"] for t in trajs[f].values()),
            "step_to_target": spread(hits[s]["step"] for s in a.seeds),
            "wall_to_target_s": spread(hits[s]["wall_s"] for s in a.seeds),
            "ms_per_step": spread(1e3 * t[-1]["wall_s"] / a.steps for t in trajs[f].values()),
            "measured": True,
        }
    out["fp32_plain_vs_incremental_agreement"] = {
        "steps": agree, "trajectory_identical": all(r["strings_equal_fraction"] == 1.0 for r in agree),
        "n_pass_s_per_step": spread(plain_times)}
    if not a.direct:
        steps_f32 = out["forms"]["fp32_incremental"]["step_to_target"]["values"]
        out["forms"]["fp32_plain"] = {
            "measured": False,
            "derived": "FP32 incremental steps to the target (per seed) x measured n-pass step time",
            "s_per_step_measured": t_plain,
            "wall_to_target_s": spread(k * t_plain for k in steps_f32),
        }
    bf = out["forms"]["bf16_incremental"]["wall_to_target_s"]["mean"]
    out["speedup_to_target_vs_fp32_plain"] = out["forms"]["fp32_plain"]["wall_to_target_s"]["mean"] / bf
    out["speedup_to_target_vs_fp32_incremental"] = out["forms"]["fp32_incremental"]["wall_to_target_s"]["mean"] / bf
    print(json.dumps(out))


if __name__ == "__main__":
    main()
