"""The non-finite parameter guard: vqmc_refresh sets its flag when a NaN or an infinity sits
in P32, b1 or b2 (a diverged update), and Made.check_finite() turns it into VQMC_ENONFINITE.
Also: the binding refuses tensors of the wrong type or shape before any call."""
import numpy as np
import pytest
import torch

from gpu_util import DEV, build_made, instance

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wd", ["f32", "bf16"])
@pytest.mark.parametrize("where", ["P32", "b1", "b2"])
def test_refresh_flags_nonfinite_parameters(where, wd):
    from paper_2106_13308_amd import binding as B
    print(f"[gpu] non-finite guard {where} {wd}", flush=True)
    p, _ = instance(130, 70, seed=41, graph=None)
    M = build_made(p, B.F32 if wd == "f32" else B.BF16)
    M.check_finite()                                        # clean parameters pass
    t = getattr(M, where)
    with torch.no_grad():
        if where == "P32":
            t[129, 69] = float("inf")                       # the last element: the ragged tile
        else:
            t[-1] = float("nan")
    M.refresh()
    with pytest.raises(B.VqmcError) as ei:
        M.check_finite()
    assert ei.value.status == B.ENONFINITE
    # sticky until the caller clears it
    with torch.no_grad():
        t.zero_()
    M.refresh()
    with pytest.raises(B.VqmcError):
        M.check_finite()
    M.nonfinite.zero_()
    M.refresh()
    M.check_finite()


def test_binding_validates_sr_arguments():
    from paper_2106_13308_amd import binding as B
    print("[gpu] binding validation", flush=True)
    p, _ = instance(67, 33, seed=42, graph=None)
    M = build_made(p, B.BF16)
    S, _, Zs, Rt = B.sample_fwd(M, 16, 1, 0)
    coef = torch.zeros(16, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        B.sr_gram(M, S.to(torch.int32), 16)                 # spins must be int8
    with pytest.raises(ValueError):
        B.sr_gram(M, S, 17)                                 # more samples than rows
    with pytest.raises(ValueError):
        B.sr_gram_sampled(M, S, Zs, Rt.float(), 16)         # Rt in the weight dtype
    with pytest.raises(ValueError):
        B.sr_direction(M, S, coef, 1e-3, Zs=Zs)             # Zs without Rt
    with pytest.raises(ValueError):
        B.sr_jvp(M, S, torch.zeros((33, 67), device=DEV), torch.zeros(33, device=DEV), torch.zeros(67, device=DEV))
    x = B.sr_direction(M, S, coef, 1e-3, Zs=Zs, Rt=Rt)     # zero coefficients: zero direction
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in x)
