"""Helpers shared by the GPU parity tests (test code, not product code)."""
import numpy as np
import torch

from oracle import bf16 as obf16
from oracle import made as omade
from paper_2106_13308_amd import inputs

DEV = "cuda"


def oracle_params(p: dict, wdtype: int) -> dict:
    """The parameters the oracle evaluates: BF16-rounded weights for the BF16 path."""
    from paper_2106_13308_amd import binding as B
    q = dict(p)
    if wdtype == B.BF16:
        q["W1"] = obf16.round_to_bf16(p["W1"])
        q["W2"] = obf16.round_to_bf16(p["W2"])
    return q


def build_made(p: dict, wdtype: int, band: bool = True):
    """band=True selects the pipelined sampler, band=False the blocked one."""
    from paper_2106_13308_amd import binding as B
    return B.Made.from_dense(p["W1"], p["b1"], p["W2"], p["b2"], p["degrees"], wdtype=wdtype, device=DEV,
                             band=band)


def spins_np(S: torch.Tensor, n: int) -> np.ndarray:
    return S[:, :n].cpu().numpy().astype(np.int8)


def logit_scale(p: dict, S) -> tuple[np.ndarray, dict]:
    """Oracle forward plus, per (b, d), the sum of |summands| of the logit z_d and,
    per (b, k), the sum of |summands| of the pre-activation a_k."""
    f = omade.forward(p, S)
    n = S.shape[1]
    M1, M2 = omade.masks(n, p["degrees"])
    W1 = np.abs(M1 * np.asarray(p["W1"], np.float64))
    W2 = np.abs(M2 * np.asarray(p["W2"], np.float64))
    zscale = f["R"] @ W2.T + np.abs(np.asarray(p["b2"], np.float64))
    ascale = np.abs(S).astype(np.float64) @ W1.T + np.abs(np.asarray(p["b1"], np.float64))
    return f, {"z": zscale, "a": ascale}


def logp_bound(f: dict, S, zscale: np.ndarray, rtol: float) -> np.ndarray:
    """|d lp| <= rtol * (|lp| + sum_d sigma(-s z) * scale_d): the first-order effect of
    a relative error rtol on every logit summand."""
    Sf = np.asarray(S, np.float64)
    sens = omade.sigmoid(-Sf * f["Z"])
    return rtol * (np.abs(f["logp"]) + (sens * zscale).sum(axis=1))


def instance(n, h, seed=1, graph="regular", deg=3, gseed=0, scale=1.0):
    p = inputs.made_init(n, h, seed)
    if scale != 1.0:
        p["W1"] = (p["W1"] * scale).astype(np.float32)
        p["W2"] = (p["W2"] * scale).astype(np.float32)
    if graph == "regular":
        edges = inputs.random_regular_graph(n, deg, gseed)
    elif graph == "er":
        edges = inputs.erdos_renyi_graph(n, 0.05, gseed)
    else:
        edges = None
    return p, edges


def relu_gates(p: dict, S, Rt: torch.Tensor, tau: float = 1e-5):
    """The ReLU gate for the oracle's gradient, teacher-forced where the pre-activation is
    within rounding of 0.

    Rt is the evaluated path's relu(A), h x ld(B) (as vqmc_sample_fwd writes it); its gate
    is Rt > 0.  Where |a_ref| <= tau * (sum of |summands| of a) the oracle takes that side,
    elsewhere its own sign.  Returns (gate B x h, number of teacher-forced entries, number
    of those where the two sides differ)."""
    f, sc = logit_scale(p, S)
    B = S.shape[0]
    gpu = (Rt[:, :B].float().cpu().numpy().T > 0)
    amb = np.abs(f["A"]) <= tau * sc["a"]
    gate = np.where(amb, gpu, f["A"] > 0)
    # outside the ambiguous band the evaluated path must agree with the oracle's sign
    assert np.array_equal(gpu[~amb], (f["A"] > 0)[~amb]), "ReLU side differs away from 0"
    return gate, int(amb.sum()), int((gpu != (f["A"] > 0))[amb].sum())
