"""Checkpoint / resume of a trainer: parameters, optimiser state, step counter and seed.  The
sampler's random numbers are keyed by (seed, step), so a run resumed from a checkpoint taken
after step t must reproduce the uninterrupted run bit for bit."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("wd,opt", [("f32", "adam"), ("bf16", "adam"), ("f32", "sr"), ("bf16", "sr")])
def test_resume_reproduces_uninterrupted_run(tmp_path, wd, opt):
    from paper_2106_13308_amd import protocol
    n, t0, t1 = 20, 4, 3
    lr = 0.1 if opt == "sr" else 0.01
    print(f"[checkpoint-test] n={n} wd={wd} opt={opt}", flush=True)
    a, _ = protocol.make_trainer(n, 0, protocol.DTYPES[wd], lr=lr, batch=256, optimizer=opt)
    for _ in range(t0 + t1):
        a.step(log=True)
    b, _ = protocol.make_trainer(n, 0, protocol.DTYPES[wd], lr=lr, batch=256, optimizer=opt)
    for _ in range(t0):
        b.step(log=True)
    path = str(tmp_path / "ckpt.safetensors")
    b.save(path)
    # a trainer started from another initialisation, then restored
    c, _ = protocol.make_trainer(n, 5, protocol.DTYPES[wd], lr=lr, batch=256, optimizer=opt)
    assert not torch.equal(c.made.P32, b.made.P32)
    c.load(path)
    assert c.t == t0 and c.seed == b.seed and c.best_E == b.best_E
    for name in ("P32", "b1", "b2"):
        assert torch.equal(getattr(c.made, name), getattr(b.made, name))
    for _ in range(t1):
        c.step(log=True)
    torch.cuda.synchronize()
    for name in ("P32", "b1", "b2"):
        assert torch.equal(getattr(c.made, name), getattr(a.made, name)), name
    assert torch.equal(c.bufs.S, a.bufs.S) and torch.equal(c.bufs.E, a.bufs.E)
    assert c.best_E == a.best_E


def test_load_refuses_other_shape(tmp_path):
    from paper_2106_13308_amd import protocol
    a, _ = protocol.make_trainer(20, 0, protocol.DTYPES["f32"], batch=256)
    a.step(log=False)
    path = str(tmp_path / "ckpt.safetensors")
    a.save(path)
    b, _ = protocol.make_trainer(20, 0, protocol.DTYPES["f32"], batch=128)
    with pytest.raises(ValueError, match="batch"):
        b.load(path)
