"""Training-side glue: the autograd wrapper of log pi and the VQMC optimisation loop.

Sec. 4 of the paper: each iteration samples a batch, computes the local energies,
back-propagates the score-function surrogate and applies the optimiser update (Adam,
Sec. 5.1).  All compute runs in ``libvqmc.so``; torch holds the FP32 master parameters
and runs Adam on them.
"""
from __future__ import annotations

import json
import time

import torch
from safetensors.torch import load_file, save_file

from . import binding as B

CHECKPOINT_FORMAT = "vqmc-trainer-1"


def save_checkpoint(path: str, tensors: dict, meta: dict) -> None:
    """Write named tensors (copied to host memory) and a JSON header to one safetensors file."""
    host = {k: v.detach().to("cpu").contiguous() for k, v in tensors.items()}
    save_file(host, path, metadata={"format": CHECKPOINT_FORMAT, "meta": json.dumps(meta)})


def load_checkpoint(path: str) -> tuple[dict, dict]:
    """Read a file written by save_checkpoint: (host tensors, JSON header).  safetensors parses
    tensors and strings only; nothing in the file is executed."""
    from safetensors import safe_open

    with safe_open(path, framework="pt") as f:
        hdr = f.metadata() or {}
    if hdr.get("format") != CHECKPOINT_FORMAT:
        raise ValueError(f"{path}: not a trainer checkpoint (format {hdr.get('format')!r})")
    return load_file(path), json.loads(hdr["meta"])


class LogProb(torch.autograd.Function):
    """log pi(S) with a hand-written adjoint.

    forward(P32, b1, b2, made, S) calls ``vqmc_logprob``; backward(grad) calls
    ``vqmc_logprob_backward`` with coef = grad, which recomputes the hidden activations
    instead of keeping B x h of them alive between the two passes.  ``made`` supplies
    the working-precision copies of P32 (call ``made.refresh()`` after changing P32)."""

    @staticmethod
    def forward(ctx, P32, b1, b2, made: B.Made, S):
        ctx.made = made
        ctx.save_for_backward(S)
        return B.logprob(made, S)

    @staticmethod
    def backward(ctx, grad):
        (S,) = ctx.saved_tensors
        dP, db1, db2 = B.logprob_backward(ctx.made, S, grad.contiguous().float())
        return dP, db1, db2, None, None


def log_prob(made: B.Made, S: torch.Tensor) -> torch.Tensor:
    return LogProb.apply(made.P32, made.b1, made.b2, made, S)


class Trainer:
    """VQMC with a MADE on a diagonal Hamiltonian, minimising E = sum_{i<j} J_ij s_i s_j.

    Each ``step()`` is one optimisation iteration: ``vqmc_step`` (sample, energy,
    statistics, gradient) followed by Adam on the FP32 master parameters and a refresh
    of the working-precision copies."""

    def __init__(self, made: B.Made, H: B.Hamiltonian, batch: int, seed: int = 2, lr: float = 1e-3,
                 algo: int = 0, betas=(0.9, 0.999), eps: float = 1e-8):
        self.made, self.H, self.batch, self.seed, self.algo = made, H, batch, seed, algo
        for t in (made.P32, made.b1, made.b2):
            t.requires_grad_(True)
        self.opt = torch.optim.Adam([made.P32, made.b1, made.b2], lr=lr, betas=betas, eps=eps)
        self.bufs = B.StepBuffers.allocate(made, H, batch)
        self.t = 0
        self.best_E = None

    def step(self, log: bool = True) -> dict | None:
        with torch.no_grad():
            B.step(self.made, self.H, self.batch, self.seed, self.t, self.bufs, algo=self.algo)
            self.made.P32.grad = self.bufs.dP
            self.made.b1.grad = self.bufs.db1
            self.made.b2.grad = self.bufs.db2
            self.opt.step()
            self.made.refresh()
        self.t += 1
        if not log:
            return None
        self.made.check_finite()
        st = B.stats_to_dict(self.bufs.stats)
        if self.best_E is None or st["min"] < self.best_E:
            self.best_E = st["min"]
        out = {"step": self.t, "mean_E": st["mean"], "var_E": st["var"], "min_E": st["min"],
               "best_E": self.best_E}
        if self.H.W_tot is not None:
            out["best_cut"] = (self.H.W_tot - self.best_E) / 2
            out["mean_cut"] = (self.H.W_tot - st["mean"]) / 2
        return out

    # ------------------------------------------------------------ checkpoint / resume
    # The sampler's random numbers are Philox(seed, step, sample, site): a trainer restored from
    # a checkpoint taken after step t draws, from step t on, exactly the strings the original run
    # draws, so a resumed run reproduces the uninterrupted one bit for bit.
    def state(self) -> tuple[dict, dict]:
        m = self.made
        tensors = {"P32": m.P32, "b1": m.b1, "b2": m.b2}
        params = [m.P32, m.b1, m.b2]
        for i, p in enumerate(params):
            st = self.opt.state.get(p, {})
            for k, v in st.items():
                tensors[f"opt.{i}.{k}"] = v if torch.is_tensor(v) else torch.tensor(v)
        meta = {"kind": type(self).__name__, "n": m.n, "h": m.h, "wdtype": m.wdtype, "batch": self.batch,
                "seed": self.seed, "algo": self.algo, "t": self.t, "best_E": self.best_E,
                "param_groups": [{k: v for k, v in g.items() if k != "params"} for g in self.opt.param_groups]}
        return tensors, meta

    def save(self, path: str) -> None:
        """Parameters, optimiser state, step counter and seed to one file (safetensors)."""
        tensors, meta = self.state()
        save_checkpoint(path, tensors, meta)

    def load(self, path: str) -> None:
        """Restore what save() wrote into this trainer (same n, h, batch and kind), then refresh
        the working-precision copies of the parameters."""
        tensors, meta = load_checkpoint(path)
        m = self.made
        mine = {"kind": type(self).__name__, "n": m.n, "h": m.h, "batch": self.batch}
        for k, v in mine.items():
            if meta.get(k) != v:
                raise ValueError(f"{path}: checkpoint has {k} = {meta.get(k)!r}, this trainer {v!r}")
        params = [m.P32, m.b1, m.b2]
        with torch.no_grad():
            for name, p in zip(("P32", "b1", "b2"), params):
                if tensors[name].shape != p.shape:
                    raise ValueError(f"{path}: {name} has shape {tuple(tensors[name].shape)}")
                p.copy_(tensors[name])
        for i, p in enumerate(params):
            st = {k.split(".", 2)[2]: v for k, v in tensors.items() if k.startswith(f"opt.{i}.")}
            if st:
                # 'step' stays a host tensor (torch.optim's default); the moments live with p
                self.opt.state[p] = {k: (v if k == "step" else v.to(p.device)) for k, v in st.items()}
            else:
                self.opt.state.pop(p, None)
        for g, saved in zip(self.opt.param_groups, meta["param_groups"]):
            g.update({k: (tuple(v) if isinstance(v, list) else v) for k, v in saved.items()})
        self.seed, self.algo, self.t, self.best_E = meta["seed"], meta["algo"], meta["t"], meta["best_E"]
        self._restore(meta)
        m.refresh()

    def _restore(self, meta: dict) -> None:
        pass

    def evaluate(self, batch: int = 1024) -> dict:
        """Mean energy of a fresh batch drawn with the evaluation tag (Sec. 5.1: a batch of
        test samples from the trained model, report their mean energy)."""
        S, _ = B.sample(self.made, batch, self.seed, self.t, tag=B.TAG_EVAL, want_logp=False)
        E = B.energy(self.H, S, batch)
        st, _ = B.batch_stats(E, want_coef=False)
        d = B.stats_to_dict(st)
        if self.H.W_tot is not None:
            d["mean_cut"] = (self.H.W_tot - d["mean"]) / 2
            d["best_cut"] = (self.H.W_tot - d["min"]) / 2
        return d


def train(trainer: Trainer, steps: int, jsonl: str | None = None, target_cut=None, every: int = 1):
    """Run ``steps`` iterations; optionally stop at the first step whose best cut reaches
    ``target_cut`` (hitting-time protocol of Sec. 6: evaluation excluded from timing)."""
    f = open(jsonl, "a") if jsonl else None
    wall = 0.0
    hit = None
    rec = None
    for i in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trainer.step(log=False)
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        trainer.made.check_finite()
        if (i + 1) % every == 0 or i + 1 == steps or target_cut is not None:
            st = B.stats_to_dict(trainer.bufs.stats)
            if trainer.best_E is None or st["min"] < trainer.best_E:
                trainer.best_E = st["min"]
            rec = {"step": trainer.t, "wall_s": wall, "mean_E": st["mean"], "var_E": st["var"],
                   "min_E": st["min"], "best_E": trainer.best_E}
            if trainer.H.W_tot is not None:
                rec["best_cut"] = (trainer.H.W_tot - trainer.best_E) / 2
                rec["mean_cut"] = (trainer.H.W_tot - st["mean"]) / 2
            if f:
                f.write(json.dumps(rec) + "\n")
                f.flush()
            if target_cut is not None and rec.get("best_cut", -1) >= target_cut and hit is None:
                hit = rec
                break
    if f:
        f.close()
    return rec, hit


def sr_direction(made: B.Made, S: torch.Tensor, coef: torch.Tensor, lam: float, n_samples: int | None = None,
                 Zs: torch.Tensor | None = None, Rt: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Stochastic-reconfiguration (natural-gradient) direction of the batch gradient
    g = sum_b coef_b grad log pi(s_b): x = (I_hat + lam I)^{-1} g with I_hat = O^T O / B the batch
    Fisher matrix of the per-sample scores (Sec. 2.1) and the ridge lam of Sec. 5.1.  One library
    call (vqmc_sr_direction): the Gram K = O O^T, the FP64 Cholesky solve (K + lam B I) y = B coef
    and x = O^T y, all on the device.  Returns x packed like the gradient (n x h, h, n)."""
    return B.sr_direction(made, S, coef, lam, B=n_samples, Zs=Zs, Rt=Rt, ws=ws)


class SRTrainer(Trainer):
    """VQMC with stochastic reconfiguration (Sec. 2.1 natural gradient; Sec. 5.1: SGD on the SR
    direction, learning rate 0.1, ridge lambda = 0.001).  Each step samples with the forward
    byproducts (vqmc_sample_fwd), computes the energies and the coefficients c_b, takes the SR
    direction of the batch gradient from those (vqmc_sr_direction; the gradient itself is never
    formed) and applies theta -= lr x to the FP32 master parameters, then refreshes the working
    copies."""

    def __init__(self, made: B.Made, H: B.Hamiltonian, batch: int, seed: int = 2, lr: float = 0.1,
                 lam: float = 1e-3, algo: int = 0):
        super().__init__(made, H, batch, seed=seed, lr=lr, algo=algo)
        self.lr, self.lam = lr, lam
        dev = made.P.device
        self.fused = made.band is not None and algo == 0
        if self.fused:
            self.Zs = torch.empty((batch, B.ld(made.n)), dtype=torch.float32, device=dev)
            rdt = torch.bfloat16 if made.wdtype == B.BF16 else torch.float32
            self.Rt = torch.empty((made.h, B.ld(batch)), dtype=rdt, device=dev)
        self.sr_ws = B.workspace(B.WS_SR_DIRECTION, made, batch)

    def state(self) -> tuple[dict, dict]:
        tensors, meta = super().state()
        meta.update(sr_lr=self.lr, lam=self.lam)
        return tensors, meta

    def _restore(self, meta: dict) -> None:
        self.lr, self.lam = meta["sr_lr"], meta["lam"]

    def step(self, log: bool = True) -> dict | None:
        with torch.no_grad():
            bufs = self.bufs
            if self.fused:
                B.sample_fwd(self.made, self.batch, self.seed, self.t, S=bufs.S, logp=bufs.logp, Zs=self.Zs,
                             Rt=self.Rt)
                bufs.E = B.energy(self.H, bufs.S, self.batch)
                bufs.stats, bufs.coef = B.batch_stats(bufs.E)
                xP, xb1, xb2 = sr_direction(self.made, bufs.S, bufs.coef, self.lam, self.batch, Zs=self.Zs,
                                            Rt=self.Rt, ws=self.sr_ws)
            else:
                B.step(self.made, self.H, self.batch, self.seed, self.t, bufs, algo=self.algo)
                xP, xb1, xb2 = sr_direction(self.made, bufs.S, bufs.coef, self.lam, self.batch, ws=self.sr_ws)
            self.made.P32.sub_(self.lr * xP)
            self.made.b1.sub_(self.lr * xb1)
            self.made.b2.sub_(self.lr * xb2)
            self.made.refresh()
        self.t += 1
        if not log:
            return None
        self.made.check_finite()
        st = B.stats_to_dict(self.bufs.stats)
        if self.best_E is None or st["min"] < self.best_E:
            self.best_E = st["min"]
        out = {"step": self.t, "mean_E": st["mean"], "var_E": st["var"], "min_E": st["min"], "best_E": self.best_E}
        if self.H.W_tot is not None:
            out["best_cut"] = (self.H.W_tot - self.best_E) / 2
            out["mean_cut"] = (self.H.W_tot - st["mean"]) / 2
        return out
