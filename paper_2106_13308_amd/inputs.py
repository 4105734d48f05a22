"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This module only draws random numbers and builds problem instances; it holds none of
the method's arithmetic (no network evaluation, no sampling rule, no energy, no
gradient).  Everything it returns is a plain NumPy array so that the oracle and the
GPU path consume identical bytes.

Instances follow the problem statement of the paper (diagonal Ising / Max-Cut, Sec. 2.4,
eq. (hamiltonian) with alpha_i = beta_i = 0) and the MADE parametrisation of Sec. 2.3:

* graphs are undirected edge lists ``edges[e] = (i, j)`` with ``0 <= i < j < n``, each
  edge once, plus a weight per edge;
* dense couplings ``J`` are symmetric ``n x n`` float32 with a zero diagonal;
* MADE parameters are ``W1 (h x n)``, ``b1 (h)``, ``W2 (n x h)``, ``b2 (n)`` in float32,
  drawn U(-1/sqrt(fan_in), +1/sqrt(fan_in)) with the nominal dense fan-in (n for the
  first layer, h for the second).  Masked entries are drawn too: a correct
  implementation never reads them.
* MADE hidden-unit degrees ``m(k) = 1 + floor(k (n-1) / h)`` (1-based, sorted, in
  [1, n-1]), the deterministic degree rule of Germain et al. (2015) that the paper's
  MADE follows (Sec. 2.3).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "made_degrees", "made_init", "random_regular_graph", "erdos_renyi_graph",
    "cycle_graph", "complete_graph", "integer_weights", "unit_weights",
    "sk_couplings", "random_spins", "paper_maxcut_graph", "paper_latent_size",
    "PAPER_MAXCUT_SIZES", "PAPER_TARGET_CUTS", "Workload", "WORKLOADS", "make_instance",
]


def made_degrees(n: int, h: int) -> np.ndarray:
    """Sorted 1-based MADE degrees m(k) in [1, n-1] for k = 0..h-1 (int32)."""
    if n < 2 or h < 1:
        raise ValueError("need n >= 2 and h >= 1")
    k = np.arange(h, dtype=np.int64)
    return (1 + (k * (n - 1)) // h).astype(np.int32)


def made_init(n: int, h: int, seed: int) -> dict:
    """Random-initialised MADE parameters (float32), U(+-1/sqrt(fan_in))."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    r1 = 1.0 / math.sqrt(n)
    r2 = 1.0 / math.sqrt(h)
    W1 = rng.uniform(-r1, r1, size=(h, n)).astype(np.float32)
    b1 = rng.uniform(-r1, r1, size=(h,)).astype(np.float32)
    W2 = rng.uniform(-r2, r2, size=(n, h)).astype(np.float32)
    b2 = rng.uniform(-r2, r2, size=(n,)).astype(np.float32)
    return {"W1": W1, "b1": b1, "W2": W2, "b2": b2, "degrees": made_degrees(n, h)}


def _canonical(edges) -> np.ndarray:
    e = np.asarray(sorted((min(a, b), max(a, b)) for a, b in edges), dtype=np.int32)
    return e.reshape(-1, 2)


def random_regular_graph(n: int, d: int, seed: int, max_restarts: int = 1000) -> np.ndarray:
    """Uniform-ish random d-regular simple graph by pairing with rejection of
    unsuitable pairs (Steger & Wormald, 1999): stubs are paired two at a time, a pair is
    accepted only if it joins two different vertices not yet adjacent; a dead end
    restarts the pairing.  Returns an (n*d/2, 2) int32 edge list with i < j."""
    if (n * d) % 2 or d >= n or d < 0:
        raise ValueError("need n*d even and 0 <= d < n")
    rng = np.random.default_rng(np.random.PCG64(seed))
    for _ in range(max_restarts):
        stubs = np.repeat(np.arange(n, dtype=np.int64), d).tolist()
        adj = [set() for _ in range(n)]
        edges = []
        m = len(stubs)
        stuck = False
        while m:
            fails = 0
            while True:
                a, b = rng.integers(0, m, size=2)
                u, v = stubs[a], stubs[b]
                if u != v and v not in adj[u]:
                    break
                fails += 1
                if fails > 4 * m + 100:
                    # check whether any suitable pair remains at all
                    rest = stubs[:m]
                    ok = any(rest[x] != rest[y] and rest[y] not in adj[rest[x]]
                             for x in range(m) for y in range(x + 1, m))
                    if not ok:
                        stuck = True
                        break
                    fails = 0
            if stuck:
                break
            adj[u].add(v)
            adj[v].add(u)
            edges.append((u, v))
            for idx in sorted((a, b), reverse=True):
                m -= 1
                stubs[idx], stubs[m] = stubs[m], stubs[idx]
        if not stuck:
            return _canonical(edges)
    raise RuntimeError("random_regular_graph: too many restarts")


def erdos_renyi_graph(n: int, p: float, seed: int) -> np.ndarray:
    """G(n, p): each pair i < j is an edge independently with probability p."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.shape[0]) < p
    return np.stack([iu[keep], ju[keep]], axis=1).astype(np.int32)


def paper_maxcut_graph(n: int, seed: int) -> np.ndarray:
    """The Max-Cut instance recipe of the experimental setup (Sec. 5.1): draw an n x n
    matrix B with i.i.d. Bernoulli(1/2) entries once, form (B + B^T)/2, round it
    elementwise and zero the diagonal; the result is the adjacency matrix.

    (B_ij + B_ji)/2 is 0, 1/2 or 1.  Rounding half to even (NumPy's and PyTorch's
    ``round``) sends 1/2 to 0, so {i, j} is an edge exactly when B_ij = B_ji = 1: the
    graph is G(n, 1/4) with unit weights.  Returns the canonical edge list (i < j)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    Bm = (rng.random((n, n)) < 0.5).astype(np.float64)
    A = np.round((Bm + Bm.T) / 2.0)
    np.fill_diagonal(A, 0.0)
    iu, ju = np.nonzero(np.triu(A, 1))
    return np.stack([iu, ju], axis=1).astype(np.int32)


def paper_latent_size(n: int) -> int:
    """The MADE hidden size of the paper's Max-Cut runs, h = 5 (log n)^2 (Sec. 5.1,
    model architecture), with the natural logarithm, rounded to the nearest integer."""
    return max(1, int(round(5.0 * math.log(n) ** 2)))


# Problem sizes of the paper's Max-Cut benchmarks (Sec. 5.2) and the target cuts of its
# time-to-target table (Table 5).  The targets belong to the paper's own instance draws;
# on a fresh draw of the same recipe they are reference points, not guarantees.
PAPER_MAXCUT_SIZES = (20, 50, 100, 200, 500)
PAPER_TARGET_CUTS = {20: 41, 50: 190, 100: 730, 200: 2800, 500: 16800}


def cycle_graph(n: int) -> np.ndarray:
    return _canonical([(i, (i + 1) % n) for i in range(n)])


def complete_graph(n: int) -> np.ndarray:
    iu, ju = np.triu_indices(n, 1)
    return np.stack([iu, ju], axis=1).astype(np.int32)


def integer_weights(num_edges: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Integer edge weights uniform in {lo..hi} (int32)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, size=num_edges).astype(np.int32)


def unit_weights(num_edges: int) -> np.ndarray:
    return np.ones(num_edges, dtype=np.int32)


def sk_couplings(n: int, seed: int) -> np.ndarray:
    """Sherrington-Kirkpatrick couplings: J_ij ~ N(0, 1/n) for i < j, symmetric,
    zero diagonal, float32."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    J = np.zeros((n, n), dtype=np.float32)
    iu, ju = np.triu_indices(n, 1)
    vals = (rng.standard_normal(iu.shape[0]) / math.sqrt(n)).astype(np.float32)
    J[iu, ju] = vals
    J[ju, iu] = vals
    return J


def tim_couplings(n: int, seed: int) -> dict:
    """Transverse-field Ising instance (Sec. 5.1): alpha_i ~ U(0, 1), beta_i ~ U(-1, 1) and
    beta_ij ~ U(-1, 1) for i < j, drawn once; beta_ij stored dense, symmetric, zero diagonal
    (float32)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    alpha = rng.uniform(0.0, 1.0, size=n).astype(np.float32)
    beta = rng.uniform(-1.0, 1.0, size=n).astype(np.float32)
    Bm = np.zeros((n, n), dtype=np.float32)
    iu, ju = np.triu_indices(n, 1)
    vals = rng.uniform(-1.0, 1.0, size=iu.shape[0]).astype(np.float32)
    Bm[iu, ju] = vals
    Bm[ju, iu] = vals
    return {"alpha": alpha, "beta": beta, "beta_ij": Bm}


def random_spins(B: int, n: int, seed: int) -> np.ndarray:
    """B x n int8 spins, uniform on {-1, +1}."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    return (2 * rng.integers(0, 2, size=(B, n)) - 1).astype(np.int8)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: problem instance + model + batch."""
    name: str
    n: int
    h: int
    B: int
    graph: str            # "regular3", "er0.02", "sk", "regular10", "paper"
    weights: str          # "unit", "int1-5", "dense"
    wdtype: str           # arithmetic type of the network weights: "f64", "f32", "bf16"
    description: str


WORKLOADS = {
    "maxcut20": Workload("maxcut20", 20, 40, 1024, "regular3", "unit", "f64",
                         "Max-Cut n=20, random 3-regular graph, unit weights; MADE h=40; B=1024"),
    "maxcut500": Workload("maxcut500", 500, 500, 4096, "er0.02", "unit", "f32",
                          "Max-Cut n=500, G(n, 0.02), unit weights; MADE h=500 FP32; B=4096"),
    "sk2000": Workload("sk2000", 2000, 2000, 8192, "sk", "dense", "bf16",
                       "SK n=2000, dense J ~ N(0,1/n); MADE h=2000 BF16; B=8192"),
    "maxcut10k": Workload("maxcut10k", 10000, 1000, 2048, "regular10", "int1-5", "bf16",
                          "Max-Cut n=10000, random 10-regular graph, integer weights 1..5 (CSR); "
                          "MADE h=1000; B=2048"),
    "maxcut10k_h2000": Workload("maxcut10k_h2000", 10000, 2000, 2048, "regular10", "unit", "bf16",
                                "Max-Cut n=10000, random 10-regular graph, unit weights; "
                                "MADE h=2000; B=2048"),
}
# transverse-field Ising model (Sec. 5.1 instance recipe; MADE h = 5 (ln n)^2 as in Sec. 5.1;
# the samples per GPU of the paper's runs are 2^9 at n = 1000 and 4 at n = 10^4, Table 7)
WORKLOADS["tim20"] = Workload("tim20", 20, 45, 1024, "tim", "dense", "f32",
                              "TIM n=20, alpha ~ U(0,1), beta_i, beta_ij ~ U(-1,1); MADE h=45; B=1024")
WORKLOADS["tim1k"] = Workload("tim1k", 1000, 239, 512, "tim", "dense", "bf16",
                              "TIM n=1000; MADE h=5(ln n)^2=239 BF16; B=512")
WORKLOADS["tim10k"] = Workload("tim10k", 10000, 424, 256, "tim", "dense", "bf16",
                               "TIM n=10000; MADE h=5(ln n)^2=424 BF16; B=256")
for _n in PAPER_MAXCUT_SIZES:
    _h = paper_latent_size(_n)
    WORKLOADS[f"paper_maxcut{_n}"] = Workload(
        f"paper_maxcut{_n}", _n, _h, 1024, "paper", "unit", "f32",
        f"Max-Cut n={_n}, the paper's instance recipe (G(n, 1/4), unit weights); "
        f"MADE h=5(ln n)^2={_h} FP32; B=1024")


def make_instance(w: Workload, graph_seed: int = 0, init_seed: int = 1) -> dict:
    """Build the Hamiltonian and initial MADE parameters of a workload.

    Returns a dict with ``n, h, B`` and either ``edges``/``weights`` (sparse Max-Cut) or
    ``J`` (dense SK), plus the MADE parameter arrays of :func:`made_init`.
    """
    out = {"n": w.n, "h": w.h, "B": w.B, "name": w.name}
    if w.graph == "regular3":
        edges = random_regular_graph(w.n, 3, graph_seed)
    elif w.graph == "regular10":
        edges = random_regular_graph(w.n, 10, graph_seed)
    elif w.graph == "paper":
        edges = paper_maxcut_graph(w.n, graph_seed)
    elif w.graph.startswith("er"):
        edges = erdos_renyi_graph(w.n, float(w.graph[2:]), graph_seed)
    elif w.graph in ("sk", "tim"):
        edges = None
    else:
        raise ValueError(w.graph)
    if edges is not None:
        out["edges"] = edges
        if w.weights == "unit":
            out["weights"] = unit_weights(len(edges))
        else:
            out["weights"] = integer_weights(len(edges), 1, 5, graph_seed + 1000)
    elif w.graph == "tim":
        out.update(tim_couplings(w.n, graph_seed))
    else:
        out["J"] = sk_couplings(w.n, graph_seed)
    out.update(made_init(w.n, w.h, init_seed))
    return out
