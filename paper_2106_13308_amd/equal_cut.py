"""BF16 + incremental sampling vs FP32 + the paper's n-pass full recompute, at equal cut.

Both forms train the same MADE (same initial weights, seeds and Adam settings) on the
same Max-Cut instance.  The best cut found so far is tracked after every update and
the wall time to first reach a target cut is measured without evaluation time
(the hitting-time protocol of Table 5 / Sec. 6: evaluate after each update, exclude
evaluation time).

The FP32 n-pass form draws the same samples as the FP32 incremental form (the two
samplers compute the same conditionals; the parity tests check they agree), so its
trajectory over T steps is the FP32 incremental trajectory.  Running it for hundreds
of steps at n = 10^4 costs seconds per step, so this script runs it for
``--plain-steps`` steps, checks that its spins and energies equal the FP32 incremental
ones step by step, and reports its time to the target as
(FP32 steps to reach the target) x (measured FP32 n-pass step time), marked as
derived.

    python -m paper_2106_13308_amd.equal_cut --workload maxcut10k_h2000 --steps 500

Prints one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import torch

from . import binding as B
from . import inputs
from .vqmc import Trainer


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="maxcut10k_h2000")
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--log-every", type=int, default=50)
    a = ap.parse_args()

    w, tb = build(a.workload, B.BF16, 0, a.lr, a.seed)
    traj_bf16 = run(tb, a.steps, a.log_every, "bf16-incremental")
    del tb
    w, tf = build(a.workload, B.F32, 0, a.lr, a.seed)
    traj_f32 = run(tf, a.steps, a.log_every, "fp32-incremental")
    del tf

    # FP32 n-pass form: a few real steps, checked against the FP32 incremental trajectory
    w, ti = build(a.workload, B.F32, 0, a.lr, a.seed)
    w, tp = build(a.workload, B.F32, 1, a.lr, a.seed)
    plain_times, same = [], []
    for i in range(a.plain_steps):
        ti.step(log=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tp.step(log=False)
        torch.cuda.synchronize()
        plain_times.append(time.perf_counter() - t0)
        same.append({"step": i + 1,
                     "spins_equal_fraction": float((ti.bufs.S == tp.bufs.S).all(dim=1).float().mean()),
                     "energies_equal": bool(torch.equal(ti.bufs.E, tp.bufs.E))})
        print(f"[equal_cut] fp32-plain step {i + 1}: {plain_times[-1]:.2f}s {same[-1]}", file=sys.stderr,
              flush=True)
    t_plain = sum(plain_times) / len(plain_times)

    target = min(traj_bf16[-1]["best_cut"], traj_f32[-1]["best_cut"])
    hb = first_reach(traj_bf16, target)
    hf = first_reach(traj_f32, target)
    out = {
        "workload": w.name, "n": w.n, "h": w.h, "B": w.B, "steps": a.steps, "lr": a.lr,
        "target_cut": target, "W_tot": tp.H.W_tot,
        "bf16_incremental": {"final_best_cut": traj_bf16[-1]["best_cut"], "final_mean_cut": traj_bf16[-1]["mean_cut"],
                             "step_to_target": hb["step"], "wall_to_target_s": hb["wall_s"],
                             "total_wall_s": traj_bf16[-1]["wall_s"],
                             "ms_per_step": 1e3 * traj_bf16[-1]["wall_s"] / a.steps},
        "fp32_incremental": {"final_best_cut": traj_f32[-1]["best_cut"], "final_mean_cut": traj_f32[-1]["mean_cut"],
                             "step_to_target": hf["step"], "wall_to_target_s": hf["wall_s"],
                             "total_wall_s": traj_f32[-1]["wall_s"],
                             "ms_per_step": 1e3 * traj_f32[-1]["wall_s"] / a.steps},
        "fp32_plain": {"measured_steps": a.plain_steps, "s_per_step": t_plain, "agreement": same,
                       "step_to_target": hf["step"], "wall_to_target_s_derived": hf["step"] * t_plain},
        "speedup_to_target": hf["step"] * t_plain / hb["wall_s"],
        "trajectory_every_10": {"bf16": [(r["step"], r["best_cut"], round(r["mean_cut"], 1)) for r in traj_bf16[9::10]],
                                "fp32": [(r["step"], r["best_cut"], round(r["mean_cut"], 1)) for r in traj_f32[9::10]]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
