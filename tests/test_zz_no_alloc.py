"""vqmc_logprob_noalloc (the library's fixed scratch in place of a workspace) against
vqmc_logprob (a caller workspace): the same kernels, so log pi and the logits must agree bit
for bit.  Two calls in a row on one GPU, the second with a smaller input, so the second runs
on scratch the first left behind; then a size beyond the fixed scratch is refused."""
import numpy as np
import pytest
import torch

from paper_2106_13308_amd import inputs

from gpu_util import DEV, build_made

pytestmark = pytest.mark.gpu


def _case(n, h, B, wd, seed):
    from paper_2106_13308_amd import binding as B_
    p = inputs.made_init(n, h, seed)
    M = build_made(p, B_.BF16 if wd == "bf16" else B_.F32)
    S = torch.zeros((B, B_.ld(n)), dtype=torch.int8, device=DEV)
    S[:, :n] = torch.from_numpy(inputs.random_spins(B, n, seed + 7)).to(DEV)
    return M, S


@pytest.mark.parametrize("wd", ["bf16", "f32"])
def test_logprob_noalloc_equals_logprob_two_calls(wd):
    from paper_2106_13308_amd import binding as B_
    # (n, h, B): first the bench shape, then a smaller one, then the first model again at a
    # smaller batch (a ragged tail of 37 samples)
    cases = [(10000, 1000, 2048), (300, 200, 70)]
    models = [(_case(n, h, B, wd, 11 + i), B) for i, (n, h, B) in enumerate(cases)]
    runs = [models[0], models[1], (models[0][0], 37)]
    for (M, S), B in runs:
        print(f"[gpu] logprob_noalloc {wd} n={M.n} h={M.h} B={B}", flush=True)
        lp_a, Z_a = B_.logprob_noalloc(M, S, B, want_z=True)
        lp_b, Z_b = B_.logprob(M, S, B, want_z=True)
        torch.cuda.synchronize()
        assert torch.isfinite(lp_a).all()
        assert torch.equal(lp_a, lp_b), float((lp_a - lp_b).abs().max())
        assert torch.equal(Z_a[:, :M.n], Z_b[:, :M.n])
        # and without Z
        lp_c = B_.logprob_noalloc(M, S, B)
        torch.cuda.synchronize()
        assert torch.equal(lp_c, lp_b)


def test_logprob_noalloc_refuses_beyond_its_scratch():
    from paper_2106_13308_amd import binding as B_
    M, S = _case(2000, 2000, 64, "bf16", 3)
    B = 20000   # needs more than the fixed scratch (checked on the host before any launch)
    need = B_.lib.vqmc_workspace_bytes(B_.WS_LOGPROB, M.n, M.h, B, M.wdtype)
    assert need > B_.NOALLOC_SCRATCH_BYTES
    S_big = torch.zeros((B, B_.ld(M.n)), dtype=torch.int8, device=DEV)
    with pytest.raises(RuntimeError, match="fixed"):
        B_.logprob_noalloc(M, S_big, B)
    # the refused call left the scratch usable
    lp_a = B_.logprob_noalloc(M, S, 64)
    lp_b = B_.logprob(M, S, 64)
    torch.cuda.synchronize()
    assert torch.equal(lp_a, lp_b)
