"""Error against the FP64 oracle of every result of one step at n = 10^4, h = 1000,
B = 2048 (random 10-regular Max-Cut, integer weights), for BF16 and FP32 weights.

Prints one JSON line per form (`[error-report] {...}`) and asserts the bars:
energies bit-exact; statistics exact (mean) / 1e-12 (variance); sampled spins equal to
the oracle's draw on their own prefix wherever |u - p| > 1e-4; log p within the
normalised bound; gradient within 1e-4 (FP32) / 3e-2 (BF16) of its largest entry."""
import json

import numpy as np
import pytest
import torch

from oracle import energy as oen
from oracle import estimator as oest
from oracle import philox as oph
from oracle import sampling as osmp
from paper_2106_13308_amd import inputs

from gpu_util import DEV, build_made, logit_scale, logp_bound, oracle_params, spins_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wd", ["bf16", "f32"])
def test_error_report_bench_workload(wd):
    from paper_2106_13308_amd import binding as B
    print(f"[gpu] error report maxcut10k {wd}", flush=True)
    wdtype = B.F32 if wd == "f32" else B.BF16
    w = inputs.WORKLOADS["maxcut10k"]
    inst = inputs.make_instance(w)
    M = build_made(inst, wdtype)
    H = B.Hamiltonian.from_edges(w.n, inst["edges"], inst["weights"], device=DEV)
    bufs = B.StepBuffers.allocate(M, H, w.B)
    B.step(M, H, w.B, 2, 0, bufs)
    torch.cuda.synchronize()
    S = spins_np(bufs.S, w.n)
    q = oracle_params(inst, wdtype)
    rep = {"form": wd}
    # energies and statistics: whole batch
    E = bufs.E.cpu().numpy()
    Eo = oen.energy_edges(inst["edges"], inst["weights"], S)
    rep["energy_max_abs_err"] = int(np.abs(E - Eo).max())
    st = B.stats_to_dict(bufs.stats)
    so = oest.batch_stats(Eo)
    rep["mean_abs_err"] = abs(st["mean"] - so["mean"])
    rep["var_rel_err"] = abs(st["var"] - so["var"]) / so["var"]
    rep["min_equal"] = bool(st["min"] == so["min"] and st["argmin"] == so["argmin"])
    # sampled spins and log p: a 64-sample subset (oracle cost)
    sub = np.arange(0, w.B, w.B // 64)
    U = oph.uniforms(2, 0, sub, w.n)
    mism, amb, _ = osmp.teacher_forced_check(q, S[sub], U, 1e-4)
    rep["spin_mismatches"] = mism
    rep["ambiguous_sites"] = amb
    rep["sites_checked"] = int(U.size)
    f, sc = logit_scale(q, S[sub])
    lp = bufs.logp.cpu().numpy().astype(np.float64)[sub]
    rep["logp_max_abs_err"] = float(np.abs(lp - f["logp"]).max())
    rep["logp_max_rel_err"] = float((np.abs(lp - f["logp"]) / np.abs(f["logp"])).max())
    bound_ratio = np.abs(lp - f["logp"]) / logp_bound(f, S[sub], sc["z"], 1.0)
    rep["logp_normalised_err"] = float(bound_ratio.max())
    # gradient over the same subset (c_b from the whole batch)
    coef = bufs.coef.cpu().numpy()
    mask = np.zeros(w.B, np.float32)
    mask[sub] = 1
    dP, db1, db2 = B.logprob_backward(M, bufs.S, torch.from_numpy(coef * mask).to(DEV))
    dW1, dW2 = M.unpack(dP)
    g = oest.logp_grad(q, S[sub], coef[sub].astype(np.float64))
    for k, got in (("W1", dW1), ("W2", dW2), ("b1", db1), ("b2", db2)):
        got = got.cpu().numpy()
        rep[f"grad_{k}_maxnorm_err"] = float(np.abs(got - g[k]).max() / np.abs(g[k]).max())
        rep[f"grad_{k}_rel_frobenius"] = float(np.linalg.norm(got - g[k]) / np.linalg.norm(g[k]))
    print("[error-report] " + json.dumps(rep), flush=True)
    assert rep["energy_max_abs_err"] == 0 and rep["mean_abs_err"] == 0 and rep["min_equal"]
    assert rep["var_rel_err"] < 1e-12
    assert mism == 0
    assert rep["logp_normalised_err"] <= 1e-5
    tol = 1e-4 if wd == "f32" else 3e-2
    for k in ("W1", "W2", "b1", "b2"):
        assert rep[f"grad_{k}_maxnorm_err"] <= tol, k
