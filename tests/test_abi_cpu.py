"""The C ABI on a machine without a GPU: the library loads, exports every
function include/hmm.h declares, and its host-side logic (argument checks,
blocking plan, status strings) works without touching a device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmm.h")
LIB = os.path.join(ROOT, "paper_2003_03508_amd", "libhmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b((?:hmm|mcmc|mlp)_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2003_03508_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("hmm_ctx_create", "hmm_ctx_destroy", "hmm_loglik", "hmm_emission",
                 "hmm_ctx_set_blocking", "hmm_blocked_plan", "hmm_status_string",
                 "hmm_loglik_batched", "hmm_autotune_batched", "mcmc_create", "mcmc_step",
                 "mcmc_train_proposal", "mlp_forward", "mlp_loss_grad", "hmm_philox",
                 "hmm_theta_to_params"):
        assert want in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name), name


def test_binding_declares_every_entry_point():
    """Every declared function has ctypes argument types in the binding (a
    missing declaration would pass 64-bit pointers as C ints)."""
    from paper_2003_03508_amd import binding
    for name in declared_functions():
        fn = getattr(binding._lib, name)
        assert fn.argtypes is not None, name
        assert fn.restype is not None, name


def test_library_carries_gfx950_code_object():
    """The fat binary embedded in our own build targets gfx950 (and only gfx950)."""
    data = open(LIB, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx\w+)", data))
    assert targets == {b"gfx950"}, targets


def test_host_argument_checks(lib):
    lib.hmm_loglik.restype = ctypes.c_int
    lib.hmm_loglik.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 5 + [
        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
        ctypes.c_void_p]
    # null context
    assert lib.hmm_loglik(None, 3, 1, 1, 1, 1, 1, 10, 1, 1, 1, None, 1) == -1
    lib.hmm_ctx_set_blocking.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32]
    assert lib.hmm_ctx_set_blocking(None, 0, 0) == -1
    lib.hmm_status_string.restype = ctypes.c_char_p
    assert lib.hmm_status_string(0) == b"ok"
    assert lib.hmm_status_string(-2) == b"unsupported"


def test_blocked_plan_without_device(lib):
    f = lib.hmm_blocked_plan
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64] + [ctypes.c_void_p] * 3
    L, nb, lv = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    assert f(None, 25, 1_000_000, ctypes.byref(L), ctypes.byref(nb), ctypes.byref(lv)) == 0
    assert L.value >= 32 and nb.value == -(-1_000_000 // L.value)
    assert nb.value >= 1024  # enough independent segments to fill 256 CUs
    assert 1 <= lv.value <= 3  # the combination tree is shallow
    assert f(None, 81, 1000, ctypes.byref(L), ctypes.byref(nb), ctypes.byref(lv)) == -2
    assert f(None, 0, 1000, ctypes.byref(L), ctypes.byref(nb), ctypes.byref(lv)) == -1
    assert f(None, 3, 0, ctypes.byref(L), ctypes.byref(nb), ctypes.byref(lv)) == 0 and nb.value == 0


def test_context_needs_a_device(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib.hmm_ctx_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    h = ctypes.c_void_p()
    assert lib.hmm_ctx_create(ctypes.byref(h), 0) == -3


def test_binding_fails_loudly_without_library(tmp_path):
    """The binding has no CPU fallback: without libhmm.so its import raises."""
    import shutil
    pkg = tmp_path / "paper_2003_03508_amd"
    pkg.mkdir()
    for f in ("__init__.py", "binding.py"):
        shutil.copy(os.path.join(ROOT, "paper_2003_03508_amd", f), pkg / f)
    r = subprocess.run(["python", "-c", "import paper_2003_03508_amd.binding"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0 and "libhmm.so" in r.stderr


def test_mcmc_host_argument_checks(lib):
    vp = ctypes.c_void_p
    lib.mcmc_create.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, vp, vp, vp,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(vp)]
    box = (ctypes.c_double * 4)(0, 1, 0, 1)
    h = vp()
    assert lib.mcmc_create(None, 3, 4, 10, 1, 1, box, 0, 8, ctypes.byref(h)) == -1
    lib.mcmc_step.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, vp]
    assert lib.mcmc_step(None, 1, 0, 0.1, None) == -1
    lib.mcmc_train_proposal.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        ctypes.c_int64, vp, vp]
    assert lib.mcmc_train_proposal(None, 1, 1, 1, 1e-3, 0, None, None) == -1
    lib.hmm_philox.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                               ctypes.c_int64, ctypes.c_int32, vp, vp]
    assert lib.hmm_philox(None, 0, 1, 0, 0, 4, 0, 1, None) == -1
    lib.mcmc_set_companion.argtypes = [vp, vp, vp]
    assert lib.mcmc_set_companion(None, 1, None) == -1
    lib.mcmc_set_twalk.argtypes = [vp, vp]
    tw = (ctypes.c_double * 6)(0.4918, 0.4918, 0.0082, 6.0, 1.5, 4.0)
    assert lib.mcmc_set_twalk(None, tw) == -1
    assert lib.mcmc_step(None, 1, 2, 0.0, None) == -1


def test_mcmc_view_layout_matches_binding(tmp_path):
    """The ctypes mirror of mcmc_view has the C struct's field offsets."""
    from paper_2003_03508_amd import binding  # needs only the library file, not a GPU
    fields = [f[0] for f in binding.McmcView._fields_]
    src = tmp_path / "off.c"
    body = "\n".join(f'printf("%s %zu\\n", "{f}", offsetof(mcmc_view, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "hmm.h"\nint main(void){'
                   + body + 'printf("size %zu\\n", sizeof(mcmc_view));return 0;}\n')
    exe = tmp_path / "off"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(binding.McmcView, f).offset, f
    assert int(out["size"]) == ctypes.sizeof(binding.McmcView)


def test_xy_alignment_and_launch_limits_checked_on_host(lib):
    """xy is read as 16-byte words: a pointer that is not 16-byte aligned is
    rejected before anything is enqueued, and so is a request whose
    launches would exceed HIP's 2^32 threads per launch.  The checks come
    before the context is used, so a zero-filled stand-in serves as the
    context here (no device is touched)."""
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    fake = ctypes.create_string_buffer(4096)
    ctx = ctypes.addressof(fake)
    dev, flag, good, odd = 0x10000, 0x20000, 0x30000, 0x30008   # never dereferenced
    f = lib.hmm_loglik
    f.restype = ctypes.c_int
    f.argtypes = [vp, i32] + [vp] * 5 + [i64, vp, vp, i32, vp, vp]
    assert f(ctx, 3, dev, dev, dev, dev, dev, 10, flag, odd, 1, None, dev) == -1
    e = lib.hmm_emission
    e.restype = ctypes.c_int
    e.argtypes = [vp, i32, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp]
    assert e(ctx, 3, dev, dev, dev, 10, flag, odd, None, dev, dev, dev) == -1
    # T = 2^32 chunks of 64 observations would need 2^32 + 64 threads
    assert e(ctx, 3, dev, dev, dev, 2 ** 32, flag, good, None, dev, dev, dev) == -2
    v = lib.hmm_viterbi
    v.restype = ctypes.c_int
    v.argtypes = [vp, i32] + [vp] * 5 + [i64, vp, vp, vp, vp, vp, vp]
    assert v(ctx, 25, dev, dev, dev, dev, dev, 10, flag, odd, None, dev, dev, dev) == -1
    # 2^36 steps in segments of at most 512: 2^27 segments of one wavefront each
    assert v(ctx, 25, dev, dev, dev, dev, dev, 2 ** 36, flag, good, None, dev, dev, dev) == -2
    assert v(ctx, 50, dev, dev, dev, dev, dev, 2 ** 35, flag, good, None, dev, dev, dev) == -2
    b = lib.hmm_loglik_batched
    b.restype = ctypes.c_int
    b.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp, vp, vp, i64, i32, vp, vp]
    K = (ctypes.c_int32 * 1)(3)
    T = (ctypes.c_int64 * 1)(10)
    zero = (ctypes.c_int64 * 1)(0)
    assert b(ctx, 1, K, T, zero, dev, 3 * 10, zero, flag, odd, 10, 1, None, dev) == -1
    m = lib.mcmc_create
    m.restype = ctypes.c_int
    m.argtypes = [vp, i32, i32, i64, vp, vp, vp, ctypes.c_uint64, i64, ctypes.POINTER(vp)]
    box = (ctypes.c_double * 4)(0, 1, 0, 1)
    h = vp()
    assert m(ctx, 3, 2, 10, flag, odd, box, 0, 8, ctypes.byref(h)) == -1
