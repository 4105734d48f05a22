"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
and host-side validation rejects bad arguments before anything is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vqmc.h")
LIB = os.path.join(ROOT, "paper_2106_13308_amd", "libvqmc.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libvqmc.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(vqmc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for want in ("vqmc_sample", "vqmc_energy", "vqmc_logprob", "vqmc_logprob_backward", "vqmc_step"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def B():
    from paper_2106_13308_amd import binding
    return binding


def test_host_helpers(B):
    assert B.ld(1) == 64 and B.ld(64) == 64 and B.ld(65) == 128
    assert B.lib.vqmc_error_string(-1) == b"invalid argument"
    assert B.lib.vqmc_workspace_bytes(B.WS_BACKWARD, 1, 5, 10, B.F32) == 0
    a = B.lib.vqmc_workspace_bytes(B.WS_BACKWARD, 500, 500, 4096, B.F32)
    b = B.lib.vqmc_workspace_bytes(B.WS_BACKWARD, 500, 500, 4096, B.BF16)
    assert a > b > 0


def test_csr_from_edges_host(B):
    edges = np.array([[3, 1], [0, 2], [1, 2], [0, 1]], np.int32)
    w = np.array([5, 7, 9, 11], np.int32)
    n, m = 4, 4
    rowptr = np.zeros(n + 1, np.int64)
    col = np.zeros(m, np.int32)
    wo = np.zeros(m, np.int32)
    vp = ctypes.c_void_p
    rc = B.lib.vqmc_csr_from_edges(n, m, edges.ctypes.data_as(vp), w.ctypes.data_as(vp), B.H_CSR_INT,
                                   rowptr.ctypes.data_as(vp), col.ctypes.data_as(vp), wo.ctypes.data_as(vp))
    assert rc == 0
    assert rowptr.tolist() == [0, 2, 4, 4, 4]
    assert col.tolist() == [1, 2, 2, 3]
    assert wo.tolist() == [11, 7, 9, 5]
    bad = np.array([[0, 0]], np.int32)
    rc = B.lib.vqmc_csr_from_edges(n, 1, bad.ctypes.data_as(vp), w.ctypes.data_as(vp), B.H_CSR_INT,
                                   rowptr.ctypes.data_as(vp), col.ctypes.data_as(vp), wo.ctypes.data_as(vp))
    assert rc == B.EINVAL and b"self loop" in B.lib.vqmc_last_error()
    dup = np.array([[0, 1], [1, 0]], np.int32)
    rc = B.lib.vqmc_csr_from_edges(n, 2, dup.ctypes.data_as(vp), w.ctypes.data_as(vp), B.H_CSR_INT,
                                   rowptr.ctypes.data_as(vp), col.ctypes.data_as(vp), wo.ctypes.data_as(vp))
    assert rc == B.EINVAL


def test_validation_rejects_before_launch(B):
    """Every entry point validates on the host and returns an error without touching
    the device (these calls run on a machine with no GPU)."""
    lib = B.lib
    fake = 0x1000  # never dereferenced: validation fails first
    bad = B.MadeC(1, 4, B.F32, fake, fake, fake, fake, fake)
    assert lib.vqmc_sample(ctypes.byref(bad), 8, 0, 0, 0, 0, fake, None, None) == B.EINVAL
    dt = B.MadeC(8, 4, 7, fake, fake, fake, fake, fake)
    assert lib.vqmc_sample(ctypes.byref(dt), 8, 0, 0, 0, 0, fake, None, None) == B.EDTYPE
    ok = B.MadeC(8, 4, B.F32, fake, fake, fake, fake, fake)
    assert lib.vqmc_sample(ctypes.byref(ok), 0, 0, 0, 0, 0, fake, None, None) == B.EINVAL
    w = ctypes.c_int32(-1)
    banded = B.MadeC(8, 4, B.F32, fake, fake, fake, fake, fake, fake)
    assert lib.vqmc_sample_cycles(ctypes.byref(ok), 8, 0, 0, fake, None, fake, ctypes.byref(w), None) == B.EINVAL
    assert b"band" in lib.vqmc_last_error()
    assert lib.vqmc_sample_cycles(ctypes.byref(banded), 8, 0, 0, fake, None, None, ctypes.byref(w), None) == B.EINVAL
    assert lib.vqmc_sample_cycles(ctypes.byref(banded), 0, 0, 0, fake, None, fake, ctypes.byref(w), None) == B.EINVAL
    assert lib.vqmc_sample_cycles(ctypes.byref(banded), 8, 0, 0, fake + 1, None, fake, ctypes.byref(w), None) == B.EINVAL
    assert w.value == -1
    assert lib.vqmc_sample(ctypes.byref(ok), 8, 0, 0, -1, 0, fake, None, None) == B.EINVAL
    big = B.MadeC(8, 5000, B.F32, fake, fake, fake, fake, fake)
    assert lib.vqmc_sample(ctypes.byref(big), 8, 0, 0, 0, 0, fake, None, None) == B.EINVAL
    assert lib.vqmc_sample(None, 8, 0, 0, 0, 0, fake, None, None) == B.EINVAL
    assert lib.vqmc_logprob(ctypes.byref(ok), fake, 8, fake, None, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_logprob_backward(ctypes.byref(ok), fake, 8, fake, fake, fake, fake, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_sample_plain(ctypes.byref(ok), 8, 0, 0, 0, 0, fake, fake, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_sr_gram(ctypes.byref(ok), fake, 8, fake, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_sr_gram(ctypes.byref(ok), fake, 0, fake, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_sr_gram(ctypes.byref(ok), fake, 65537, fake, fake, 1 << 40, None) == B.EINVAL
    assert lib.vqmc_sr_gram(ctypes.byref(ok), fake, 8, None, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_sr_gram_sampled(ctypes.byref(ok), fake, 8, fake, fake, fake, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_sr_gram_sampled(ctypes.byref(ok), fake, 8, fake + 4, fake, fake, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_sr_gram_sampled(ctypes.byref(ok), fake, 8, None, fake, fake, fake, 1 << 30, None) == B.EINVAL
    nopt = B.MadeC(8, 4, B.F32, fake, None, fake, fake, fake)
    assert lib.vqmc_logprob(ctypes.byref(nopt), fake, 8, fake, None, fake, 1 << 30, None) == B.EINVAL
    # TIM local energy and step: host-side checks
    T8 = B.TimC(8, fake, fake, fake)
    T9 = B.TimC(9, fake, fake, fake)
    assert lib.vqmc_tim_energy(ctypes.byref(ok), ctypes.byref(T9), fake, 8, fake, None, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_tim_energy(ctypes.byref(ok), None, fake, 8, fake, None, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_tim_energy(ctypes.byref(ok), ctypes.byref(T8), fake, 8, fake, None, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_tim_energy(ctypes.byref(ok), ctypes.byref(T8), fake + 8, 8, fake, None, fake, 1 << 30,
                               None) == B.EINVAL                                  # spins misaligned
    wide_f32 = B.MadeC(8, 600, B.F32, fake, fake, fake, fake, fake)
    assert lib.vqmc_tim_energy(ctypes.byref(wide_f32), ctypes.byref(T8), fake, 8, fake, None, fake, 1 << 30,
                               None) == B.EINVAL and b"too large" in lib.vqmc_last_error()
    assert lib.vqmc_tim_step(ctypes.byref(ok), ctypes.byref(T8), 8, 0, 0, 0, fake, None, fake, fake, fake, fake,
                             fake, fake, fake, 1 << 30, None) == B.EINVAL         # no band
    assert lib.vqmc_workspace_bytes(B.WS_TIM_STEP, 100, 50, 64, B.BF16) > \
        lib.vqmc_workspace_bytes(B.WS_TIM_ENERGY, 100, 50, 64, B.BF16) > 0
    # the no-allocation variant refuses a size beyond its fixed scratch before touching the device
    wide = B.MadeC(2000, 2000, B.BF16, fake, fake, fake, fake, fake)
    assert lib.vqmc_workspace_bytes(B.WS_LOGPROB, 2000, 2000, 20000, B.BF16) > B.NOALLOC_SCRATCH_BYTES
    assert lib.vqmc_logprob_noalloc(ctypes.byref(wide), fake, 20000, fake, None, None) == B.EWORKSPACE
    assert b"fixed" in lib.vqmc_last_error()
    assert lib.vqmc_logprob_noalloc(ctypes.byref(nopt), fake, 8, fake, None, None) == B.EINVAL
    assert lib.vqmc_logprob_noalloc(ctypes.byref(ok), fake, 8, None, None, None) == B.EINVAL
    H = B.HamC(8, 9, 0, fake, fake, fake, None)
    assert lib.vqmc_energy(ctypes.byref(H), fake, 8, fake, None, 0, None) == B.EINVAL
    Hd = B.HamC(8, B.H_DENSE_F32, 0, None, None, None, fake)
    assert lib.vqmc_energy(ctypes.byref(Hd), fake, 8, fake, None, 0, None) == B.EWORKSPACE
    Hi = B.HamC(8, B.H_CSR_INT, 3, fake, fake, fake, None)
    assert lib.vqmc_energy(ctypes.byref(Hi), fake + 8, 8, fake, None, 0, None) == B.EINVAL  # spins misaligned
    assert b"16-byte" in lib.vqmc_last_error()
    Hc = B.HamC(9, B.H_CSR_INT, 3, fake, fake, fake, None)
    assert lib.vqmc_step(ctypes.byref(ok), ctypes.byref(Hc), 8, 0, 0, 0, 0, fake, fake, fake, fake, fake,
                         fake, fake, fake, fake, 1 << 30, None) == B.EINVAL  # n mismatch
    Hc8 = B.HamC(8, B.H_CSR_INT, 3, fake, fake, fake, None)
    assert lib.vqmc_step(ctypes.byref(ok), ctypes.byref(Hc8), 8, 0, 0, 0, 2, fake, fake, fake, fake, fake,
                         fake, fake, fake, fake, 1 << 30, None) == B.EINVAL  # algo
    assert lib.vqmc_batch_stats(None, 1, 8, fake, None, None) == B.EINVAL
    assert lib.vqmc_cast(8, 4, fake, B.F64, fake, fake, None) == B.EDTYPE
    assert lib.vqmc_uniforms(0, 8, 0, 0, 0, 0, fake, None) == B.EINVAL
    deg = np.array([2, 1, 3], np.int32)   # unsorted
    assert lib.vqmc_pack(8, 3, fake, fake, deg.ctypes.data_as(ctypes.c_void_p), fake, fake, None) == B.EINVAL
    assert b"not sorted" in lib.vqmc_last_error()
    deg = np.array([0, 1, 3], np.int32)   # out of range
    assert lib.vqmc_pack(8, 3, fake, fake, deg.ctypes.data_as(ctypes.c_void_p), fake, fake, None) == B.EINVAL
    # non-finite guard: the flag value turns into a status on the host
    assert lib.vqmc_check_nonfinite(0) == B.OK
    assert lib.vqmc_check_nonfinite(1) == B.ENONFINITE and b"NaN" in lib.vqmc_last_error()
    assert lib.vqmc_refresh(8, 4, fake, B.F32, fake, fake, None, None, fake, None, fake, None) == B.EINVAL
    assert lib.vqmc_refresh(8, 4, fake, B.F64, fake, fake, fake, fake, fake, None, None, None) == B.EDTYPE
    # SR solve and direction
    assert lib.vqmc_sr_solve(8, fake, 0.0, fake, 1.0, fake, fake, 1 << 30, None) == B.EINVAL      # shift <= 0
    assert lib.vqmc_sr_solve(8, fake, float("nan"), fake, 1.0, fake, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_sr_solve(0, fake, 1.0, fake, 1.0, fake, fake, 1 << 30, None) == B.EINVAL
    assert lib.vqmc_sr_solve(8, fake, 1.0, fake, 1.0, fake, fake, 16, None) == B.EWORKSPACE
    assert lib.vqmc_sr_solve_workspace_bytes(65) == 128 * 128 * 8 + 2 * 1024
    assert lib.vqmc_sr_direction(ctypes.byref(ok), fake, 8, fake, fake, None, 1e-3, fake, fake, fake, None, fake,
                                 1 << 30, None) == B.EINVAL    # Zs without Rt
    assert lib.vqmc_sr_direction(ctypes.byref(ok), fake, 8, fake, None, None, 0.0, fake, fake, fake, None, fake,
                                 1 << 30, None) == B.EINVAL    # lambda
    assert lib.vqmc_sr_direction(ctypes.byref(ok), fake, 8, fake, None, None, 1e-3, fake, fake, fake, None, fake,
                                 16, None) == B.EWORKSPACE
    assert lib.vqmc_workspace_bytes(B.WS_SR_DIRECTION, 8, 4, 8, B.F32) > lib.vqmc_workspace_bytes(B.WS_SR_GRAM, 8, 4,
                                                                                                   8, B.F32)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the package without libvqmc.so cannot be used: importing the binding raises
    (there is no CPU or eager fallback for any call)."""
    import shutil
    import subprocess
    import sys
    pkg = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2106_13308_amd")
    dst = tmp_path / "paper_2106_13308_amd"
    shutil.copytree(pkg, dst, ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "csrc"))
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n    import paper_2106_13308_amd.binding\nexcept ImportError as e:\n"
            "    print('raised', e); sys.exit(0)\nsys.exit(1)\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "libvqmc.so is missing" in r.stdout
