"""Error against the FP64 oracle of every result of one step at n = 10^4, h = 1000,
B = 2048 (random 10-regular Max-Cut, integer weights), for BF16 and FP32 weights.

Prints one JSON line per form (`[error-report] {...}`) and asserts the bars:
energies bit-exact; statistics exact (mean) / 1e-12 (variance); sampled spins equal to
the oracle's draw on their own prefix wherever |u - p| > 1e-4; log p within the
normalised bound; the gradient that vqmc_step itself returned (the whole batch, the
kernels the bench times) within 1e-4 (FP32) / 3e-2 (BF16) of its largest entry, with the
ReLU side teacher-forced where a pre-activation lies within rounding of 0."""
import json

import numpy as np
import pytest
import torch

from oracle import energy as oen
from oracle import estimator as oest
from oracle import philox as oph
from oracle import sampling as osmp
from paper_2106_13308_amd import inputs

from gpu_util import DEV, build_made, logit_scale, logp_bound, oracle_params, relu_gates, spins_np

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
    # the same draw through vqmc_sample_fwd exposes relu(A), the ReLU side the step's
    # backward took (vqmc_step runs exactly these kernels on the same counters)
    S2, _, _, Rt = B.sample_fwd(M, w.B, 2, 0)
    torch.cuda.synchronize()
    assert torch.equal(S2, bufs.S)
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
    # sampled spins and log p: whole batch
    U = oph.uniforms(2, 0, np.arange(w.B), w.n)
    mism, amb, _ = osmp.teacher_forced_check(q, S, U, 1e-4)
    rep["spin_mismatches"] = mism
    rep["ambiguous_sites"] = amb
    rep["sites_checked"] = int(U.size)
    f, sc = logit_scale(q, S)
    lp = bufs.logp.cpu().numpy().astype(np.float64)
    rep["logp_max_abs_err"] = float(np.abs(lp - f["logp"]).max())
    rep["logp_max_rel_err"] = float((np.abs(lp - f["logp"]) / np.abs(f["logp"])).max())
    bound_ratio = np.abs(lp - f["logp"]) / logp_bound(f, S, sc["z"], 1.0)
    rep["logp_normalised_err"] = float(bound_ratio.max())
    # the step's own gradient, whole batch, against the oracle on the step's coefficients
    coef = bufs.coef.cpu().numpy().astype(np.float64)
    assert np.array_equal(coef.astype(np.float32), ((Eo - so["mean"]) / w.B).astype(np.float32))
    gate, n_forced, n_flipped = relu_gates(q, S, Rt)
    rep["relu_teacher_forced"] = n_forced
    rep["relu_sides_differing"] = n_flipped
    g = oest.logp_grad(q, S, coef, active=gate)
    dW1, dW2 = M.unpack(bufs.dP)
    for k, got in (("W1", dW1), ("W2", dW2), ("b1", bufs.db1), ("b2", bufs.db2)):
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
