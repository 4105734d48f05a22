"""The hand-written adjoint of log pi behind torch.autograd (vqmc.LogProb): gradients that
torch.autograd propagates through it against the FP64 oracle's analytic gradient and
against central finite differences of the library's own log pi.

Bars: FP32 weights 2e-5 of the largest entry (each entry is a sum of B products of
FP32-accurate factors), BF16 weights 3e-2 (the backward products round the activations
and adjoints to BF16); the directional finite difference within 2e-3 relative."""
import numpy as np
import pytest
import torch

from oracle import estimator as oest
from paper_2106_13308_amd import inputs

from gpu_util import DEV, build_made, instance, logit_scale, oracle_params

pytestmark = pytest.mark.gpu


def _spins(B_, B, n, seed):
    S_np = inputs.random_spins(B, n, seed)
    S = torch.zeros((B, B_.ld(n)), dtype=torch.int8, device=DEV)
    S[:, :n] = torch.from_numpy(S_np).to(DEV)
    return S_np, S


@pytest.mark.parametrize("wd", ["f32", "bf16"])
@pytest.mark.parametrize("n,h,B", [(20, 40, 64), (300, 200, 70), (10000, 1000, 64)])
def test_autograd_adjoint_matches_oracle(n, h, B, wd):
    from paper_2106_13308_amd import binding as B_
    from paper_2106_13308_amd import vqmc
    print(f"[gpu] autograd adjoint n={n} h={h} B={B} {wd}", flush=True)
    wdtype = B_.F32 if wd == "f32" else B_.BF16
    p, _ = instance(n, h, seed=31, graph=None, scale=2.0)
    M = build_made(p, wdtype, band=False)
    for t in (M.P32, M.b1, M.b2):
        t.requires_grad_(True)
    S_np, S = _spins(B_, B, n, 32)
    up = np.random.default_rng(33).standard_normal(B).astype(np.float32)
    lp = vqmc.log_prob(M, S)
    assert lp.requires_grad and lp.shape == (B,)
    (lp * torch.from_numpy(up).to(DEV)).sum().backward()
    torch.cuda.synchronize()
    q = oracle_params(p, wdtype)
    g = oest.logp_grad(q, S_np, up.astype(np.float64))
    dW1, dW2 = M.unpack(M.P32.grad.contiguous())
    tol = 2e-5 if wd == "f32" else 3e-2
    for k, got in (("W1", dW1), ("W2", dW2), ("b1", M.b1.grad), ("b2", M.b2.grad)):
        got = got.cpu().numpy()
        rel = np.abs(got - g[k]).max() / np.abs(g[k]).max()
        print(f"  {k}: max-normalised error {rel:.2e}")
        assert rel <= tol, k
    # the forward value is the library's log pi
    f, _ = logit_scale(q, S_np)
    assert np.abs(lp.detach().cpu().numpy() - f["logp"]).max() <= (1e-4 if wd == "f32" else 2e-2) * \
        np.abs(f["logp"]).max()


def test_autograd_adjoint_matches_finite_differences():
    """<grad F, v> from the adjoint against (F(theta + eps v) - F(theta - eps v)) / (2 eps),
    F = sum_b u_b log pi(s_b) evaluated by vqmc_logprob after a refresh of the working copy.
    The direction leaves out the first-layer weights of every unit whose pre-activation
    could change sign within +-eps v (the oracle's FP64 pre-activations decide), so F is
    smooth along it and the difference quotient has no kink error."""
    from oracle import made as omade
    from paper_2106_13308_amd import binding as B_
    from paper_2106_13308_amd import vqmc
    print("[gpu] autograd adjoint vs finite differences", flush=True)
    n, h, B, eps = 20, 40, 4, 1e-2
    p, _ = instance(n, h, seed=35, graph=None, scale=2.0)
    M = build_made(p, B_.F32, band=False)
    for t in (M.P32, M.b1, M.b2):
        t.requires_grad_(True)
    S_np, S = _spins(B_, B, n, 36)
    u = torch.from_numpy(np.random.default_rng(37).standard_normal(B).astype(np.float32)).to(DEV)
    (vqmc.log_prob(M, S) * u).sum().backward()
    rng = np.random.default_rng(38)
    base = [t.detach().clone() for t in (M.P32, M.b1, M.b2)]
    dirs = [torch.from_numpy(rng.standard_normal(tuple(t.shape)).astype(np.float32)).to(DEV) for t in base]
    # units whose pre-activation may cross 0 along the direction keep their W1 row and b1 fixed
    vW1, _ = M.unpack(dirs[0])
    M1, _ = omade.masks(n, p["degrees"])
    dA = S_np.astype(np.float64) @ (M1 * vW1.cpu().numpy()).T + dirs[1].cpu().numpy()
    A = omade.forward(oracle_params(p, B_.F32), S_np)["A"]
    risky = (np.abs(A) <= 2 * eps * np.abs(dA)).any(axis=0)
    assert risky.sum() < h // 2
    c = M.c.cpu().numpy()
    w1_part = torch.from_numpy(np.arange(h)[None, :] >= c[:, None]).to(DEV)
    keep = torch.from_numpy(~risky).to(DEV)
    dirs[0] = torch.where(w1_part & ~keep[None, :], torch.zeros_like(dirs[0]), dirs[0])
    dirs[1] = torch.where(keep, dirs[1], torch.zeros_like(dirs[1]))
    analytic = sum(float((t.grad.double() * v.double()).sum()) for t, v in zip((M.P32, M.b1, M.b2), dirs))

    def F(e):
        with torch.no_grad():
            for t, b0, v in zip((M.P32, M.b1, M.b2), base, dirs):
                t.copy_(b0 + e * v)
            M.refresh()
            return float((B_.logprob(M, S).double() * u.double()).sum())

    fd = (F(eps) - F(-eps)) / (2 * eps)
    F(0.0)
    print(f"  directional derivative: adjoint {analytic:.6e}, central difference {fd:.6e} "
          f"({int(risky.sum())} of {h} units left out of the W1 direction)")
    assert abs(fd - analytic) <= 2e-3 * abs(analytic)
