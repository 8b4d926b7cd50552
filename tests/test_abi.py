"""The C ABI library on the CPU: it loads, exports every symbol include/sso.h
declares, and validates configurations without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2110_01470_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "sso.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sso_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("sso_init", "sso_step", "sso_run", "sso_get_best", "sso_batch_init",
                     "sso_batch_run", "sso_batch_tune", "sso_batch_get_results", "sso_eval",
                     "sso_polish"):
        assert required in names
    assert len(names) == 29


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def cfg(**kw):
    base = dict(n=100, d=30, kind="sphere", lo=-100.0, hi=100.0, cg=0.4, cp=0.7, cw=0.9,
                seed=1, s=np.zeros(30, np.float32))
    base.update(kw)
    if "d" in kw and "s" not in kw:
        base["s"] = np.zeros(base["d"], np.float32)
    return binding.make_config(**base)


def test_workspace_bytes_for_valid_configs():
    c, keep = cfg()
    nbytes = binding.workspace_bytes(c)
    # two rows of 32 floats per particle, plus fitness, state, shift, trace
    assert nbytes >= 2 * 100 * 32 * 4 + 100 * 8 + 4096 * 12
    c, keep = cfg(n=65536, d=1000, kind="ripple", w=np.ones(1000, np.float32), storage="f32")
    f32_bytes = binding.workspace_bytes(c)
    assert f32_bytes >= 2 * 65536 * 1024 * 4
    # 24-bit grid indices: 4 variables in 3 words, rows of 768 words for D=1000.
    c, keep = cfg(n=65536, d=1000, kind="ripple", w=np.ones(1000, np.float32))
    u24_bytes = binding.workspace_bytes(c)
    assert 2 * 65536 * 768 * 4 <= u24_bytes < f32_bytes
    c, keep = cfg(n=16384, d=256, kind="dense", a=np.eye(256, dtype=np.float32))
    assert binding.workspace_bytes(c) >= 2 * 16384 * 256 * 4 + 256 * 256 * 4


@pytest.mark.parametrize("d", [256, 100, 1])
def test_split_contraction_adds_the_bf16_parts_of_a(d):
    """The split contraction keeps A's three bf16 parts beside the FP32
    copies: 3 x dp^2 halves, dp = d rounded up to 32 (256-byte aligned)."""
    a = np.eye(d, dtype=np.float32)
    c32, k1 = cfg(n=1000, d=d, kind="dense", a=a, contraction="f32")
    c3, k2 = cfg(n=1000, d=d, kind="dense", a=a, contraction="bf16x3")
    ca, k3 = cfg(n=1000, d=d, kind="dense", a=a)
    dp = (d + 31) // 32 * 32
    extra = (3 * dp * dp * 2 + 255) // 256 * 256
    assert binding.workspace_bytes(c3) - binding.workspace_bytes(c32) == extra
    # AUTO is the split contraction.
    assert binding.workspace_bytes(ca) == binding.workspace_bytes(c3)
    # Separable objectives ignore the field.
    cs, k4 = cfg(n=1000, d=d, contraction="bf16x3")
    cf, k5 = cfg(n=1000, d=d, contraction="f32")
    assert binding.workspace_bytes(cs) == binding.workspace_bytes(cf)


def test_f16x2_contraction_needs_a_scalable_instance():
    """The fp16 split scales each row of A and the differences x - s by
    powers of two into fp16's range; instances it cannot scale (a
    non-finite entry, magnitudes beyond 2^+-100) are refused when asked for
    explicitly, and AUTO then takes the bf16 split (same workspace)."""
    d = 64
    rng = np.random.Generator(np.random.PCG64(5))
    a = (rng.standard_normal((d, d)) / 8).astype(np.float32)
    good, k1 = cfg(n=100, d=d, kind="dense", a=a, contraction="f16x2")
    b3, k2 = cfg(n=100, d=d, kind="dense", a=a, contraction="bf16x3")
    assert binding.workspace_bytes(good) == binding.workspace_bytes(b3) > 0
    for bad_a in (np.where(np.eye(d) > 0, np.float32(np.inf), a).astype(np.float32),
                  (a * np.float32(1e35)).astype(np.float32),
                  (a * np.float32(1e-33)).astype(np.float32)):
        c, k3 = cfg(n=100, d=d, kind="dense", a=bad_a, contraction="f16x2")
        with pytest.raises(binding.SSOError):
            binding.workspace_bytes(c)
        c, k4 = cfg(n=100, d=d, kind="dense", a=bad_a)
        assert binding.workspace_bytes(c) == binding.workspace_bytes(b3)
    # A box far beyond the shift: differences up to 3e35.
    c, k5 = cfg(n=100, d=d, kind="dense", a=a, lo=-3e35, hi=3e35, contraction="f16x2")
    with pytest.raises(binding.SSOError):
        binding.workspace_bytes(c)


@pytest.mark.parametrize("kw", [
    dict(n=0), dict(d=0), dict(lo=1.0, hi=1.0), dict(lo=float("nan")),
    dict(cg=0.8), dict(cp=0.95), dict(cw=1.0 - 2.0 ** -8), dict(cw=1.5),
    dict(kind=7), dict(order=2), dict(engine=5), dict(lanes=12), dict(lanes=128),
    dict(trace_cap=3), dict(kind="ripple"), dict(kind="dense"),
    dict(kind="dense", d=257, a=np.eye(257, dtype=np.float32)),
    dict(engine="resident", n=2000), dict(lo=-3e38, hi=3e38),
    dict(storage=7), dict(storage="u24", engine="resident"),
    dict(kind="f4", s=None, d=50, n=300, engine="resident"),   # 5 particles per thread
    dict(kind="f4", s=None, d=300, n=20, engine="resident"),   # 75 chunks, 64 lanes
    dict(polish_every=50, polish_steps=5), dict(kind="ripple", w=np.ones(30, np.float32), polish_every=1),
    dict(kind="dense", a=np.eye(30, dtype=np.float32), polish_lr=float("nan")),
    dict(storage="u24", kind="dense", a=np.eye(30, dtype=np.float32)),
    dict(contraction=4), dict(contraction=-1),
])
def test_invalid_configs_are_rejected(kw):
    c, keep = cfg(**kw)
    with pytest.raises(binding.SSOError):
        binding.workspace_bytes(c)


def test_null_config_and_strerror():
    lib = binding.load()
    assert lib.sso_workspace_bytes(None) == 0
    assert lib.sso_strerror(0) == b"ok"
    assert lib.sso_strerror(-2) == b"workspace too small"
    assert lib.sso_strerror(99) == b"unknown error"
    lib.sso_destroy(None)


def test_init_rejects_bad_workspace_before_touching_a_device():
    lib = binding.load()
    c, keep = cfg()
    nbytes = binding.workspace_bytes(c)
    ctx = ctypes.c_void_p()
    # misaligned
    assert lib.sso_init(ctypes.byref(c), ctypes.c_void_p(4096 + 8), nbytes, None,
                        ctypes.byref(ctx)) == binding.E_INVAL
    # too small
    assert lib.sso_init(ctypes.byref(c), ctypes.c_void_p(4096), nbytes - 1, None,
                        ctypes.byref(ctx)) == binding.E_NOMEM
    assert ctx.value is None


def test_static_run_rejects_before_touching_a_device():
    """sso_run_static refuses invalid configurations, the dense objective and
    swarms whose state exceeds its static array before any HIP call."""
    lib = binding.load()
    P = ctypes.c_void_p
    assert lib.sso_run_static(None, 1, None, None, None, None) == binding.E_INVAL
    c, keep = cfg(n=0)
    assert lib.sso_run_static(ctypes.byref(c), 1, None, None, None, None) == binding.E_INVAL
    c, keep = cfg(n=64, d=16, kind="dense", a=np.eye(16, dtype=np.float32))
    assert lib.sso_run_static(ctypes.byref(c), 1, None, None, None, None) == binding.E_UNSUPPORTED
    assert b"DENSE" in lib.sso_last_error(None)
    # The ripple workload's state (about 400 MB) exceeds the 64 MiB array.
    c, keep = cfg(n=65536, d=1000, kind="ripple", w=np.ones(1000, np.float32))
    assert binding.workspace_bytes(c) > binding.STATIC_SCRATCH_BYTES
    assert lib.sso_run_static(ctypes.byref(c), 5, None, P(4096), P(4096), P(4096)) == binding.E_NOMEM
    msg = lib.sso_last_error(None).decode()
    assert str(binding.STATIC_SCRATCH_BYTES) in msg and str(binding.workspace_bytes(c)) in msg


def batch_cfgs(*changes):
    """A batch of ripple swarms; changes[k] (a dict) alters swarm k."""
    out = []
    for k, ch in enumerate(changes):
        d = ch.get("d", 20)
        base = dict(n=50 + k, d=d, kind="ripple", lo=-10.0, hi=10.0, cg=0.4, cp=0.7, cw=0.9,
                    seed=k, swarm_id=k, s=np.zeros(d, np.float32), w=np.ones(d, np.float32))
        base.update(ch)
        out.append(binding.make_config(**base))
    arr = (binding.Config * len(out))(*[c for c, _ in out])
    return arr, [keep for _, keep in out]


def test_batch_workspace_bytes_adds_up_the_swarms():
    lib = binding.load()
    arr, keep = batch_cfgs({}, {"n": 1000, "d": 500}, {"d": 3})
    nbytes = lib.sso_batch_workspace_bytes(arr, 3)
    # 24-bit rows: 3 words per 4 variables, two rows per particle, packed.
    rows = sum(2 * n * 3 * ((d + 3) // 4) * 4 for n, d in ((50, 20), (1000, 500), (52, 3)))
    assert nbytes >= rows + 3 * 4096 * 12
    arr, keep = batch_cfgs({"storage": "f32"}, {"n": 1000, "d": 500, "storage": "f32"},
                           {"d": 3, "storage": "f32"})
    f32 = lib.sso_batch_workspace_bytes(arr, 3)
    assert f32 > nbytes
    # A swarm small enough for the one-swarm resident engine still runs in a
    # batch (on the STREAM body), 24-bit rows included.
    arr, keep = batch_cfgs({"n": 1, "d": 1, "storage": "u24"})
    assert lib.sso_batch_workspace_bytes(arr, 1) > 0


@pytest.mark.parametrize("changes", [
    ({}, {"kind": "sphere", "w": None}),        # mixed kinds
    ({}, {"order": 1, "cg": 0.9, "cw": 0.4}),   # mixed orders
    ({}, {"storage": "f32"}),                   # mixed storage
    ({"kind": "dense", "d": 8, "a": np.eye(8, dtype=np.float32)},),
    ({"engine": "resident"},),
    ({"d": 1025},),
    ({}, {"cg": 0.95}),                          # one invalid swarm
])
def test_invalid_batches_are_rejected(changes):
    lib = binding.load()
    arr, keep = batch_cfgs(*changes)
    assert lib.sso_batch_workspace_bytes(arr, len(changes)) == 0
    assert lib.sso_batch_last_error(None)


def test_batch_init_rejects_bad_arguments_before_touching_a_device():
    lib = binding.load()
    arr, keep = batch_cfgs({}, {})
    assert lib.sso_batch_workspace_bytes(arr, 0) == 0
    assert lib.sso_batch_workspace_bytes(None, 2) == 0
    nbytes = lib.sso_batch_workspace_bytes(arr, 2)
    b = ctypes.c_void_p()
    assert lib.sso_batch_init(arr, 2, ctypes.c_void_p(4096 + 8), nbytes, None,
                              ctypes.byref(b)) == binding.E_INVAL
    assert lib.sso_batch_init(arr, 2, ctypes.c_void_p(4096), nbytes - 1, None,
                              ctypes.byref(b)) == binding.E_NOMEM
    assert b.value is None
    lib.sso_batch_destroy(None)


def test_rocrand_cross_check_helper_loads():
    """The tests' rocRAND helper (a second Philox4x32-10 for the GPU parity
    tests) is built in-tree and exports its one entry point."""
    import ctypes

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rocrand_ref",
                        "librocrand_philox.so")
    assert os.path.exists(path), "build() compiles tests/rocrand_ref/librocrand_philox.so"
    lib = ctypes.CDLL(path)
    assert hasattr(lib, "rocrand_philox_blocks")


def test_header_is_plain_c(tmp_path):
    """include/sso.h compiles as C99 (no C++ in the boundary), and a C
    program that takes the address of every declared function links against
    libsso.so."""
    import subprocess

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    names = declared_functions()
    src = tmp_path / "use_sso.c"
    src.write_text('#include "sso.h"\n#include <stdio.h>\ntypedef void (*fn_t)(void);\n'
                   'int main(void) {\n    fn_t fns[] = {\n'
                   + "".join(f"        (fn_t)&{n},\n" for n in names)
                   + "    };\n    printf(\"%d\\n\", (int)(sizeof fns / sizeof fns[0]));\n"
                   "    return sso_strerror(SSO_OK)[0] == 'o' ? 0 : 1;\n}\n")
    exe = tmp_path / "use_sso"
    lib_dir = os.path.dirname(binding.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", "-I",
                    os.path.join(root, "include"), str(src), "-o", str(exe), "-L", lib_dir, "-lsso",
                    f"-Wl,-rpath,{lib_dir}"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert int(out) == len(names)
