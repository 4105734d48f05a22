#!/usr/bin/env python3
"""Throughput of one VQMC optimisation step on one MI355X.

A step is the whole hot path on one batch, as one training iteration runs it after an
optimiser update: the working-precision weights and the sampler's tables re-derived
from the FP32 master weights (``vqmc_cast`` + ``vqmc_band``), incremental
autoregressive sampling of B strings (Algorithm 1), the Max-Cut local energy, FP64 batch
statistics, and the score-function gradient through the masked network, i.e. one
``vqmc_step`` call.  The Adam update itself (torch) is outside the step.

Workload (default): Max-Cut on a seeded random 10-regular graph with n = 10000 vertices
and integer weights in {1..5} (CSR), MADE with h = 1000 hidden units in BF16 weights,
B = 2048 samples per step.  Inputs are synthetic and resident in HBM before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]

Prints one JSON line.  Besides the headline BF16 + incremental step it reports the same
step in FP32 + incremental and FP32 + the paper's n-pass full recompute (``forms``),
per-call times, the roofline of the dominant kernel and the FP64 oracle timed on a
bounded sample of the same workload on the host cores (``cpu_baseline``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

GRAPH_DESC = {"maxcut10k": "random 10-regular, integer weights 1..5, CSR",
              "maxcut10k_h2000": "random 10-regular, unit weights, CSR",
              "sk2000": "SK dense J ~ N(0,1/n), FP64 energy",
              "maxcut500": "G(500, 0.02), unit weights, CSR"}
METRIC = "samples/s per VQMC step (sample+energy+grad) at n=10k, BF16 vs FP32 at equal cut"
PEAK = {"bf16_mfma_tflops": 2500.0, "fp32_mfma_tflops": 157.3, "fp32_vector_tflops": 157.3,
        "fp64_tflops": 78.6, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="maxcut10k")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP32 comparison forms")
    ap.add_argument("--no-tim", action="store_true", help="skip the TIM step reported beside the headline")
    ap.add_argument("--cpu-samples", type=int, default=2048)
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup + timed steps only (for rocprofv3)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--profile-call", default="sample",
                    help="library call timed by --profile-only after the steps (sample, sr_gram, ...)")
    ap.add_argument("--form", default="bf16", choices=["bf16", "fp32", "fp32_plain"],
                    help="step form timed by --profile-only")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup(workload: str, wdtype):
    import torch
    from paper_2106_13308_amd import binding as B
    from paper_2106_13308_amd import inputs
    w = inputs.WORKLOADS[workload]
    inst = inputs.make_instance(w)
    made = B.Made.from_dense(inst["W1"], inst["b1"], inst["W2"], inst["b2"], inst["degrees"],
                             wdtype=wdtype, device="cuda")
    if "edges" in inst:
        H = B.Hamiltonian.from_edges(w.n, inst["edges"], inst["weights"], device="cuda")
    elif "alpha" in inst:
        H = B.Tim(inst["alpha"], inst["beta"], inst["beta_ij"], device="cuda")
    else:
        H = B.Hamiltonian.dense(inst["J"], device="cuda")
    torch.cuda.synchronize()
    return w, inst, made, H


def time_steps(made, H, B_, steps, warmup, algo=0, seed=2):
    """Median-free whole-window timing: W untimed steps, then K steps between two
    synchronisations (plus HIP events on the launch stream)."""
    import torch
    from paper_2106_13308_amd import binding as B
    bufs = B.StepBuffers.allocate(made, H, B_)
    for i in range(warmup):
        made.refresh()
        B.step(made, H, B_, seed, i, bufs, algo=algo)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for i in range(steps):
        made.refresh()
        B.step(made, H, B_, seed, warmup + i, bufs, algo=algo)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall / steps, bufs


def time_calls(made, H, B_, reps=10, seed=2, names=None):
    """Average duration of each library call of the step (or of those in names), HIP events on
    its stream, over reps back-to-back calls after one untimed call."""
    import torch
    from paper_2106_13308_amd import binding as B
    bufs = B.StepBuffers.allocate(made, H, B_)
    B.step(made, H, B_, seed, 0, bufs)
    ws_bw = B.workspace(B.WS_BACKWARD, made, B_)
    ws_sr = B.workspace(B.WS_SR_GRAM, made, B_) if names is None or "sr_gram" in names else None
    K = torch.empty((B_, B_), dtype=torch.float32, device="cuda") if ws_sr is not None else None
    calls = {"refresh": made.refresh}
    if made.band is not None:
        # the calls vqmc_step makes: sampling with the forward byproducts, energy, statistics,
        # and the backward from those byproducts
        S, lp, Zs, Rt = B.sample_fwd(made, B_, seed, 1)
        ws_bs = B.workspace(B.WS_BACKWARD_SAMPLED, made, B_)
        calls["sample"] = lambda: B.sample_fwd(made, B_, seed, 1, S=S, logp=lp, Zs=Zs, Rt=Rt)
        calls["backward_sampled"] = lambda: B.backward_sampled(made, S, bufs.coef, Zs, Rt, ws=ws_bs)
        if names is None or "sr_direction" in names:
            # not part of the step: the SR (natural-gradient) direction of the batch gradient,
            # from the sampler's byproducts (Gram, FP64 Cholesky solve, one gradient pass)
            ws_sd = B.workspace(B.WS_SR_DIRECTION, made, B_)
            calls["sr_direction"] = lambda: B.sr_direction(made, S, bufs.coef, 1e-3, B=B_, Zs=Zs, Rt=Rt, ws=ws_sd)
    else:
        calls["sample"] = lambda: B.sample(made, B_, seed, 1, S=bufs.S, logp=bufs.logp)
    calls.update({
        "energy": lambda: B.energy(H, bufs.S, B_),
        "stats": lambda: B.batch_stats(bufs.E),
        "logprob_backward": lambda: B.logprob_backward(made, bufs.S, bufs.coef, ws=ws_bw),
        "logprob": lambda: B.logprob(made, bufs.S),
        # not part of the step: the sample-space Gram of the scores that an SR update solves with
        "sr_gram": lambda: B.sr_gram(made, bufs.S, B_, ws=ws_sr, K=K),
    })
    out = {}
    for name, fn in calls.items():
        if names is not None and name not in names:
            continue
        fn()
        torch.cuda.synchronize()
        if name == "sample" and made.band is not None:
            # in the step the sampler runs right after the refresh rewrote its tables; time
            # it in that context: events around each sampling launch only
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for e0, e1 in ev:
                made.refresh()
                e0.record()
                fn()
                e1.record()
            torch.cuda.synchronize()
            out[name] = sum(e0.elapsed_time(e1) for e0, e1 in ev) / reps
            continue
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


def algorithmic_work(w, made, H):
    """Algorithmic flops / bytes per launch of each call: the work the method defines, not the
    work the kernels do (masked halves and padding are not counted)."""
    c = made.c.cpu().numpy().astype(np.int64)
    n, h, B_ = w.n, w.h, w.B
    sum_c = int(c.sum())                     # sum_d c[d]: second-layer MACs per sample
    nh = n * h
    es = 2 if made.wdtype == 2 else 4
    work = {
        # sampler: n*h MACs per sample (dot over complete units + rank-1 update)
        "sample": {"flops": 2.0 * nh * B_, "bytes": nh * es + B_ * (n + 4)},
        # energy: read the spins once (+ the CSR, L2 resident) and write E
        "energy": ({"bytes": B_ * n + (H.nnz * 8 + (n + 1) * 8) + B_ * 8} if H.J is None else
                   # dense J: strict upper triangle, n^2/2 FP64 MACs per sample
                   {"flops": float(n) * (n - 1) * B_, "bytes": B_ * n + 4 * n * n + B_ * 8}),
        # forward: first layer sum_d (h - c[d]) + second layer sum_d c[d] = n*h MACs
        "logprob": {"flops": 2.0 * nh * B_},
        # backward: forward recompute (n*h) + hidden adjoint (sum_c) + weight gradient (n*h)
        "logprob_backward": {"flops": 2.0 * (2 * nh + sum_c) * B_},
        # SR Gram: forward recompute (n*h MACs) + hidden adjoint (sum_c) per sample, then per
        # unique Gram entry (B(B+1)/2 of them) n + h prefix multiply-adds (2 flops) and n + h
        # outer rows (a multiply and a multiply-add: 3 flops)
        "sr_gram": {"flops": 2.0 * (nh + sum_c) * B_ + 5.0 * (n + h) * B_ * (B_ + 1) / 2},
        # backward from the sampler's byproducts: hidden adjoint (sum_c) + weight gradient (n*h)
        "backward_sampled": {"flops": 2.0 * (nh + sum_c) * B_},
    }
    return work


# kernels behind each library call of the step, the file that holds them, and their bound
def _dominant_desc(call, made, H):
    bf16 = made.wdtype == 2
    mm = PEAK["bf16_mfma_tflops"] if bf16 else PEAK["fp32_mfma_tflops"]
    if call == "sample":
        if made.band is not None:
            k = "sample_pipe_kernel<bf16" if bf16 else "sample_pipe_kernel<float"  # prefix: <T, planes>
            return {"kernels": [k], "src": ["sample_pipe.hip"], "bound": "mfma", "peak": mm,
                    "unit": "TFLOP/s", "metric": "tflops"}
        if made.h <= 2048:
            k = "sample_blocked_kernel<bf16>" if bf16 else "sample_blocked_kernel<float>"
            return {"kernels": [k], "src": ["sample_blocked.hip"], "bound": "mfma", "peak": mm,
                    "unit": "TFLOP/s", "metric": "tflops"}
        return {"kernels": ["sample_incremental_kernel"], "src": ["sample.hip"], "bound": "alu",
                "peak": PEAK["fp32_vector_tflops"], "unit": "TFLOP/s", "metric": "tflops"}
    if call == "energy":
        if H.J is not None:
            return {"kernels": ["energy_dense_kernel", "sum_partials_kernel"], "src": ["energy.hip"],
                    "bound": "mfma", "peak": PEAK["fp64_tflops"], "unit": "TFLOP/s", "metric": "tflops"}
        return {"kernels": ["energy_csr_bytes_kernel"], "src": ["energy.hip"], "bound": "hbm",
                "peak": PEAK["hbm_gbs"], "unit": "GB/s", "metric": "gbs"}
    t = "bf16" if bf16 else "float"
    if call == "backward_sampled" and bf16:
        # with the sampler tables the masked copy of P^T is ready and the weight-gradient launch
        # sums the bias partials, so these three are the call's launches
        return {"kernels": ["grad_out_kernel<bf16>", "bwd_hidden2_kernel", "bwd_weight2_kernel"],
                "src": ["gemm.hip", "gemm2.hip"], "bound": "mfma", "peak": mm, "unit": "TFLOP/s", "metric": "tflops"}
    if call == "backward_sampled":
        return {"kernels": [f"grad_out_kernel<{t}>", f"bwd_hidden_kernel<{t}>", f"bwd_weight_kernel<{t}, false>",
                            f"bwd_weight_kernel<{t}, true>", "sum_rows_kernel"],
                "src": ["gemm.hip"], "bound": "mfma", "peak": mm, "unit": "TFLOP/s", "metric": "tflops"}
    return {"kernels": [f"fwd_hidden_kernel<{t}, true>", f"fwd_out_kernel<{t}, 1>", f"bwd_hidden_kernel<{t}>",
                        f"bwd_weight_kernel<{t}, false>", f"bwd_weight_kernel<{t}, true>", "sum_rows_kernel"],
            "src": ["gemm.hip"], "bound": "mfma", "peak": mm, "unit": "TFLOP/s", "metric": "tflops"}


def _src_sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(HERE, "paper_2106_13308_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def _traffic(desc, workload):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
    or None when they are missing or the kernels' source changed since they were taken."""
    path = os.path.join(HERE, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256", {}).get(",".join(desc["src"])) != _src_sha(desc["src"]):
        return None
    tot = 0.0
    for k in desc["kernels"]:
        e = rec["kernels"].get(k)
        if e is None:  # a name prefix (template arguments chosen at launch)
            e = next((v for name, v in rec["kernels"].items() if name.startswith(k)), None)
        if e is None or e.get("fetch_bytes") is None or e.get("write_bytes") is None:
            return None
        tot += (e["fetch_bytes"] + e["write_bytes"]) * e.get("launches_per_call", 1)
    return tot


def serial_chain(made, w, sample_ms):
    """The sampler's serial chain, measured: vqmc_sample_cycles counts every wave's shader-clock
    cycles between the barriers of the 64-site blocks.  The floor is blocks x the sweep's cycles
    per block (the chain of Algorithm 1 that no product can shorten) at the measured clock; the
    slowest helper's cycles per block show how far the products are from it."""
    from paper_2106_13308_amd import binding as B
    B.sample_cycles(made, w.B, 2, 0)
    _, _, cyc = B.sample_cycles(made, w.B, 2, 1)
    nb = (w.n + 63) // 64
    cyc = cyc.astype(np.float64)
    sweep = cyc[:, :2, 0].mean(axis=1)
    helpers = cyc[:, 2:, 0].max(axis=1)
    ghz = float((cyc[:, 0, 1] / (cyc[:, 0, 2] / 100e6)).mean() / 1e9)
    floor_ms = float(sweep.mean()) / (ghz * 1e9) * 1e3  # the sweep's cycles summed over the blocks
    return {"blocks": nb, "sweep_cycles_per_block": float(sweep.mean()) / nb,
            "slowest_helper_cycles_per_block": float(helpers.mean()) / nb,
            "cycles_per_block": float(cyc[:, 0, 1].mean()) / nb, "shader_clock_ghz": ghz,
            "floor_ms": floor_ms, "kernel_ms": sample_ms, "frac": floor_ms / sample_ms}


def roofline(call, kernels, made, H, workload):
    desc = _dominant_desc(call, made, H)
    ach = kernels[call][desc["metric"]]
    return {"kernel": "+".join(desc["kernels"]), "call": f"vqmc_{call}", "bound": desc["bound"],
            "achieved": ach, "peak": desc["peak"], "unit": desc["unit"], "frac": ach / desc["peak"],
            "traffic": _traffic(desc, workload)}


def cpu_baseline(w, inst, nsamp):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload."""
    from oracle import energy as oen, estimator as oest, philox as oph, sampling as osmp
    from oracle import bf16 as obf16
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
    except Exception:
        threads = 1
    p = dict(inst)
    p["W1"] = obf16.round_to_bf16(inst["W1"])
    p["W2"] = obf16.round_to_bf16(inst["W2"])
    t0 = time.perf_counter()
    U = oph.uniforms(2, 0, np.arange(nsamp), w.n)
    S, lp = osmp.sample_plain(p, U)
    E = (oen.energy_edges(inst["edges"], inst["weights"], S) if "edges" in inst
         else oen.energy_dense(inst["J"], S))
    st = oest.batch_stats(E)
    oest.logp_grad(p, S, st["coef"])
    dt = time.perf_counter() - t0
    return {"value": nsamp / dt, "unit": "samples/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{nsamp} of the {w.B} samples of one step (sample_plain + energy + stats + "
                      f"analytic gradient, FP64 NumPy), {dt:.1f} s; cost is linear in B",
            "seconds": dt, "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def tim_work(made, B_):
    """Algorithmic work of one vqmc_tim_energy launch: the contraction that gives the logit changes
    (2 sum_{i<d} (c[d] - c[i]) flops per sample, on MFMA) and the B n (n - 1) / 2 log-sigmoid
    differences, 7 flops each (the FMA forming the changed logit, one exponential, one logarithm,
    a minimum, the difference and the accumulation)."""
    c = made.c.cpu().numpy().astype(np.int64)
    n = c.shape[0]
    idx = np.arange(n, dtype=np.int64)
    pair_units = int((c * idx).sum() - (c * (n - 1 - idx)).sum())   # sum_{i<d} (c[d] - c[i])
    elems = B_ * n * (n - 1) // 2
    return {"contraction_flops": 2.0 * pair_units * B_, "elements": elems, "epilogue_flops": 7.0 * elems}


def time_tim_calls(made, H, B_, reps=10, seed=2):
    """HIP-event durations of the calls of one TIM step (vqmc_tim_step makes the same launches)."""
    import torch
    from paper_2106_13308_amd import binding as B
    S, lp, Zs, Rt = B.sample_fwd(made, B_, seed, 1)
    ws_t = B.workspace(B.WS_TIM_ENERGY, made, B_)
    E = torch.empty(B_, dtype=torch.float64, device="cuda")
    st, coef = B.batch_stats(B.tim_energy(made, H, S, B_, ws=ws_t, E=E))
    ws_bs = B.workspace(B.WS_BACKWARD_SAMPLED, made, B_)
    calls = {"refresh": made.refresh,
             "sample": lambda: B.sample_fwd(made, B_, seed, 1, S=S, logp=lp, Zs=Zs, Rt=Rt),
             "tim_energy": lambda: B.tim_energy(made, H, S, B_, ws=ws_t, E=E),
             "stats": lambda: B.batch_stats(E),
             "backward_sampled": lambda: B.backward_sampled(made, S, coef, Zs, Rt, ws=ws_bs)}
    out = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


def tim_report(w, made, H, steps, warmup):
    """One TIM step timed (vqmc_refresh + vqmc_tim_step), its calls, and the roofline of the local
    energy (bound: the FP32 vector ALU of its log-sigmoid epilogue)."""
    ms, _, bufs = time_steps(made, H, w.B, steps, warmup)
    calls = time_tim_calls(made, H, w.B)
    wk = tim_work(made, w.B)
    t = calls["tim_energy"] / 1e3
    ach = wk["epilogue_flops"] / t / 1e12
    return bufs, {
        "ms_per_step": ms, "samples_per_s": w.B / (ms / 1e3),
        "calls_ms": calls,
        "roofline": {"kernel": "tim_flip_kernel (+ forward, masked W2 copy, dense diagonal energy, combine)",
                     "call": "vqmc_tim_energy", "bound": "alu", "achieved": ach,
                     "peak": PEAK["fp32_vector_tflops"], "unit": "TFLOP/s", "frac": ach / PEAK["fp32_vector_tflops"],
                     "traffic": None,
                     "elements_per_s": wk["elements"] / t,
                     "contraction_tflops": wk["contraction_flops"] / t / 1e12},
    }


def cpu_baseline_tim(w, inst, nsites=160):
    """The FP64 oracle's TIM step on a bounded sample: one sample drawn (sample_plain), its diagonal
    entry, its single-flip log-ratios at nsites of the n sites and the analytic gradient; the
    flip ratios' cost is scaled to all n sites (it is linear in the number of sites)."""
    from oracle import bf16 as obf16, estimator as oest, philox as oph, sampling as osmp, tim as otim
    try:
        import threadpoolctl
        threads = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] or [1])
    except Exception:
        threads = 1
    p = dict(inst)
    if w.wdtype == "bf16":
        p["W1"] = obf16.round_to_bf16(inst["W1"])
        p["W2"] = obf16.round_to_bf16(inst["W2"])
    sites = np.linspace(0, w.n - 1, nsites).astype(np.int64)
    t0 = time.perf_counter()
    U = oph.uniforms(2, 0, np.arange(1), w.n)
    S, _ = osmp.sample_plain(p, U)
    otim.diag_energy(inst["beta"], inst["beta_ij"], S)
    oest.logp_grad(p, S, np.ones(1))
    t_fixed = time.perf_counter() - t0
    t1 = time.perf_counter()
    otim.flip_logratio(p, S, sites=sites)
    t_flip = time.perf_counter() - t1
    per_sample = t_fixed + t_flip * w.n / nsites
    return {"value": 1.0 / per_sample, "unit": "samples/s", "cores": int(threads), "kind": "oracle",
            "sample": f"1 sample: sample_plain, diagonal energy, gradient ({t_fixed:.1f} s) and the single-flip "
                      f"log-ratios at {nsites} of {w.n} sites ({t_flip:.1f} s, scaled to all sites: the cost is "
                      f"linear in the sites and in B)", "seconds": t_fixed + t_flip, "cpu_model": _cpu_model()}


def main_tim(a):
    import torch
    from paper_2106_13308_amd import binding as B
    from paper_2106_13308_amd import inputs
    w = inputs.WORKLOADS[a.workload]
    wd = B.BF16 if w.wdtype == "bf16" else B.F32
    w, inst, made, H = setup(a.workload, wd)
    log(f"TIM setup done: n={w.n} h={w.h} B={w.B} ({w.wdtype})")
    if a.profile_only:
        ms, _, _ = time_steps(made, H, w.B, a.steps, a.warmup)
        log(f"tim step: {ms:.3f} ms")
        return
    bufs, rep = tim_report(w, made, H, a.steps, a.warmup)
    log(f"tim step: {rep['ms_per_step']:.3f} ms; calls " + json.dumps({k: round(v, 4) for k, v in rep['calls_ms'].items()}))
    st = B.stats_to_dict(bufs.stats)
    out = {
        "metric": "samples/s per VQMC step (sample+local energy+grad), transverse-field Ising model",
        "value": rep["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": rep["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": w.wdtype, "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "h": w.h, "global_batch": w.B,
                   "hamiltonian": "TIM, alpha ~ U(0,1), beta_i and beta_ij ~ U(-1,1), dense",
                   "sampler": "incremental", "weights": w.wdtype, "parallelism": "single GPU"},
        "roofline": rep["roofline"], "calls_ms": rep["calls_ms"],
        "step_stats": {"mean_E": st["mean"], "min_E": st["min"], "var_E": st["var"]},
    }
    if not a.no_cpu:
        log("oracle CPU baseline (TIM, bounded sample) ...")
        out["cpu_baseline"] = cpu_baseline_tim(w, inst)
        log(f"oracle: {out['cpu_baseline']['value']:.4f} samples/s")
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py runs on exactly one GPU; multi-GPU data parallelism is not "
                                   "implemented (shards would draw B/N samples each at sample_offset "
                                   "rank * B/N and all-reduce the gradient)", "n_gpus": a.gpus}))
        sys.exit(2)
    import torch
    from paper_2106_13308_amd import binding as B
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"device {torch.cuda.get_device_name(0)}; workload {a.workload}")
    if a.workload.startswith("tim"):
        return main_tim(a)
    if a.calib_copy:
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 256 MiB device-to-device")
        del x, y
    wd = B.F32 if (a.workload == "maxcut500" or a.form != "bf16") else B.BF16
    w, inst, made, H = setup(a.workload, wd)
    log(f"setup done: n={w.n} h={w.h} B={w.B}")
    if a.profile_only and a.form == "fp32_plain":
        ms, wall_ms, _ = time_steps(made, H, w.B, a.steps, a.warmup, algo=1)
        log(f"fp32 plain step: {ms:.3f} ms")
        return
    ms, wall_ms, bufs = time_steps(made, H, w.B, a.steps, a.warmup)
    log(f"bf16 incremental step: {ms:.3f} ms (event), {wall_ms * 1e3:.3f} ms (wall)")
    if a.profile_only:
        # then one library call (by default the sampler as the roofline times it: one untimed
        # launch, then five launches each right after a refresh), so that the trace holds it too
        calls = time_calls(made, H, w.B, reps=5, names=(a.profile_call,))
        log("per-call ms (profiled loop): " + json.dumps({k: round(v, 4) for k, v in calls.items()}))
        return
    value = w.B / (ms / 1e3)
    st = B.stats_to_dict(bufs.stats)
    calls = time_calls(made, H, w.B)
    log("per-call ms: " + json.dumps({k: round(v, 4) for k, v in calls.items()}))
    work = algorithmic_work(w, made, H)
    kernels = {}
    for name, t in calls.items():
        wk = work.get(name, {})
        d = {"ms": t}
        if "flops" in wk:
            d["tflops"] = wk["flops"] / (t / 1e3) / 1e12
        if "bytes" in wk:
            d["gbs"] = wk["bytes"] / (t / 1e3) / 1e9
        kernels[name] = d
    grad_call = "backward_sampled" if "backward_sampled" in calls else "logprob_backward"
    step_calls = {k: calls[k] for k in ("refresh", "sample", "energy", "stats", grad_call)}
    dom = max(step_calls, key=step_calls.get)
    roof = roofline(dom, kernels, made, H, w.name)
    if dom == "sample" and made.band is not None:
        roof["serial_chain"] = serial_chain(made, w, calls["sample"])
        log("sampler serial chain: " + json.dumps({k: round(v, 4) for k, v in roof["serial_chain"].items()}))
    forms = {"bf16_incremental": {"ms_per_step": ms, "samples_per_s": value}}
    if not a.no_forms:
        made32 = B.Made(made.n, made.h, made.P32, made.b1, made.b2, made.c, wdtype=B.F32)
        ms32, _, _ = time_steps(made32, H, w.B, max(3, a.steps // 4), 1)
        forms["fp32_incremental"] = {"ms_per_step": ms32, "samples_per_s": w.B / (ms32 / 1e3)}
        log(f"fp32 incremental step: {ms32:.3f} ms")
        # the paper's form: n full forward passes per sample batch (one timed step)
        msp, _, _ = time_steps(made32, H, w.B, 1, 0, algo=1)
        forms["fp32_plain"] = {"ms_per_step": msp, "samples_per_s": w.B / (msp / 1e3),
                               "note": "one timed step, no warmup step (launch-bound form)"}
        log(f"fp32 plain step: {msp:.1f} ms")
    wname = "bf16" if wd == B.BF16 else "f32"  # the weights the timed step computes with
    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": wname, "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "h": w.h, "global_batch": w.B,
                   "graph": GRAPH_DESC.get(w.name, w.description),
                   "sampler": "incremental", "weights": wname, "parallelism": "single GPU"},
        "roofline": roof, "kernels": kernels, "forms": forms,
        "step_stats": {"mean_E": st["mean"], "min_E": st["min"], "var_E": st["var"]},
    }
    if not a.no_tim:
        # the paper's other Hamiltonian at the same n: the TIM step (its local energy needs the
        # n single-flip ratios of every sample), reported beside the headline
        from paper_2106_13308_amd import inputs
        wt = inputs.WORKLOADS["tim10k"]
        _, _, made_t, H_t = setup("tim10k", B.BF16)
        _, rep = tim_report(wt, made_t, H_t, max(3, a.steps // 4), 2)
        rep["config"] = {"workload": wt.name, "n": wt.n, "h": wt.h, "global_batch": wt.B, "weights": "bf16"}
        out["tim_step"] = rep
        log(f"tim10k step: {rep['ms_per_step']:.3f} ms")
        del made_t, H_t
    if not a.no_cpu:
        log(f"oracle CPU baseline on {a.cpu_samples} samples ...")
        out["cpu_baseline"] = cpu_baseline(w, inst, a.cpu_samples)
        log(f"oracle: {out['cpu_baseline']['value']:.3f} samples/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
