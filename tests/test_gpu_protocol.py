"""End-to-end training under the paper's Max-Cut protocol (Sec. 5.1) on the n = 20
instance of its recipe, checked against the exact optimum that the oracle finds by
enumeration."""
import numpy as np
import pytest
import torch

from oracle import energy as oenergy
from oracle import exact
from paper_2106_13308_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wd", ["f32", "bf16"])
def test_paper_protocol_n20_reaches_exact_optimum(wd):
    from paper_2106_13308_amd import binding as B
    from paper_2106_13308_amd import protocol
    n = 20
    e = inputs.paper_maxcut_graph(n, 0)
    w = inputs.unit_weights(len(e))
    best, _ = exact.max_cut_brute(n, oenergy.energy_edges(e, w, exact.all_strings(n)), oenergy.total_weight(w))
    print(f"[protocol-test] n={n} wd={wd} exact optimum {best}", flush=True)
    tr, _ = protocol.make_trainer(n, 0, protocol.DTYPES[wd])
    r = protocol.run_one(tr, 300, {"opt": best})
    # the evaluation batch's energies are the oracle's energies of the same spins
    S, _ = B.sample(tr.made, 1024, tr.seed, tr.t, tag=B.TAG_EVAL, want_logp=False)
    E = B.energy(tr.H, S, 1024).cpu().numpy()
    assert np.array_equal(E, oenergy.energy_edges(e, w, S[:, :n].cpu().numpy()))
    assert r["final_eval_best_cut"] == best
    assert r["hit_best"]["opt"] is not None
    # after 300 iterations the model concentrates on optimal cuts
    assert best - 1.0 <= r["final_eval_mean_cut"] <= best


def test_paper_protocol_n20_sr_reaches_exact_optimum():
    """The paper's SGD + SR configuration (Sec. 5.1: lr 0.1, lambda 1e-3) on the same instance."""
    from paper_2106_13308_amd import protocol
    n = 20
    e = inputs.paper_maxcut_graph(n, 0)
    w = inputs.unit_weights(len(e))
    best, _ = exact.max_cut_brute(n, oenergy.energy_edges(e, w, exact.all_strings(n)), oenergy.total_weight(w))
    print(f"[protocol-test] n={n} sr exact optimum {best}", flush=True)
    tr, _ = protocol.make_trainer(n, 0, protocol.DTYPES["f32"], lr=0.1, optimizer="sr")
    r = protocol.run_one(tr, 300, {"opt": best})
    assert r["hit_best"]["opt"] is not None
    assert r["final_eval_best_cut"] == best
    assert r["final_eval_mean_cut"] >= best - 2.0
