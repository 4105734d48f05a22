"""The checkpoint file format on the host: named tensors and a JSON header round-trip
exactly, and a file of another kind is refused."""
import pytest
import torch
from safetensors.torch import save_file


def test_roundtrip(tmp_path):
    from paper_2106_13308_amd.vqmc import load_checkpoint, save_checkpoint
    g = torch.Generator().manual_seed(0)
    t = {"P32": torch.randn(7, 5, generator=g), "opt.0.step": torch.tensor(3.0),
         "opt.0.exp_avg": torch.randn(7, 5, generator=g, dtype=torch.float64)}
    meta = {"t": 3, "seed": 2, "best_E": -12.0, "param_groups": [{"lr": 0.01, "betas": [0.9, 0.999]}]}
    p = str(tmp_path / "c.safetensors")
    save_checkpoint(p, t, meta)
    t2, meta2 = load_checkpoint(p)
    assert meta2 == meta
    assert set(t2) == set(t)
    for k in t:
        assert t2[k].dtype == t[k].dtype and torch.equal(t2[k], t[k])


def test_refuses_foreign_file(tmp_path):
    from paper_2106_13308_amd.vqmc import load_checkpoint
    p = str(tmp_path / "x.safetensors")
    save_file({"a": torch.zeros(2)}, p)
    with pytest.raises(ValueError, match="not a trainer checkpoint"):
        load_checkpoint(p)
