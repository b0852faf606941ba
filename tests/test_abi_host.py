"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/rid.h declares, the ctypes structs match the C layout,
and argument validation happens before any device call."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rid.h")


@pytest.fixture(scope="module")
def L():
    from paper_2405_16076_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2405_16076_amd import build
        build.build()
    _lib.lib()
    return _lib


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\S.*?\b(rid_[a-z_0-9]+)\s*\(", text, re.M)))


def test_every_declared_function_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (rid_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(names) == set(L.SIGNATURES), set(names) ^ set(L.SIGNATURES)


def test_struct_layouts_match_c(L):
    src = """
#include <stdio.h>
#include <stddef.h>
#include "rid.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(rid_config), sizeof(rid_update), sizeof(rid_info), sizeof(rid_error),
         sizeof(rid_batch_info), sizeof(rid_profile));
  printf("%zu %zu %zu %zu\\n", offsetof(rid_config, n_max), offsetof(rid_update, flags), offsetof(rid_info, device_bytes),
         offsetof(rid_batch_info, tune_ms));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        exe = os.path.join(d, "p")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    sizes = [int(x) for x in lines[0].split()]
    assert sizes == [C.sizeof(L.rid_config), C.sizeof(L.rid_update), C.sizeof(L.rid_info), C.sizeof(L.rid_error),
                     C.sizeof(L.rid_batch_info), C.sizeof(L.rid_profile)]
    offs = [int(x) for x in lines[1].split()]
    assert offs == [L.rid_config.n_max.offset, L.rid_update.flags.offset, L.rid_info.device_bytes.offset,
                    L.rid_batch_info.tune_ms.offset]


def test_status_strings_and_defaults(L):
    lib = L.lib()
    for s in range(8):
        assert lib.rid_status_string(s).decode().startswith("RID_")
    cfg = L.rid_config()
    assert lib.rid_config_default(C.byref(cfg)) == 0
    assert (cfg.delta, cfg.eps, cfg.c_sample, cfg.ridge_floor) == (0.05, 0.5, 1.0, 1e-8)
    assert lib.rid_config_default(None) == L.RID_EINVAL


@pytest.mark.parametrize("field,value,msg", [
    ("m", 0, "m must be"), ("ell", 3, "ell must"), ("ell", 513, "ell must"), ("k", 41, "k must"),
    ("t", 41, "t must"), ("n_max", 0, "n_max"), ("sketch_prec", 0, "f64 sketch"), ("delta", 1.5, "delta"),
    ("hutch_n1", 25, "n1"), ("sketch_tile", 3, "sketch_tile"), ("sketch_tile", 2, "wide sketch tile"),
    ("coeff_mode", 2, "coeff_mode"), ("gram_mode", 3, "gram_mode"), ("gram_mode", -1, "gram_mode"),
])
def test_invalid_configs_rejected_before_device(L, field, value, msg):
    expect = L.RID_ENOTSUP if msg == "wide sketch tile" else L.RID_EINVAL
    lib = L.lib()
    cfg = L.rid_config()
    lib.rid_config_default(C.byref(cfg))
    cfg.m, cfg.ell, cfg.k, cfg.t, cfg.n_max = 1000, 40, 20, 20, 100
    setattr(cfg, field, value)
    h = C.c_void_p()
    st = lib.rid_init_stream(C.byref(cfg), None, C.byref(h))
    assert st == expect
    buf = C.create_string_buffer(256)
    lib.rid_last_error(None, buf, 256)
    assert msg in buf.value.decode()
    assert not h.value


def test_best4_needs_t_at_most_154(L):
    lib = L.lib()
    cfg = L.rid_config()
    lib.rid_config_default(C.byref(cfg))
    cfg.m, cfg.ell, cfg.k, cfg.t, cfg.n_max = 1000, 400, 200, 200, 1000
    cfg.coeff_mode = L.RID_COEFF_BEST4
    h = C.c_void_p()
    assert lib.rid_init_stream(C.byref(cfg), None, C.byref(h)) == L.RID_ENOTSUP
    assert lib.rid_get_coeff_choice(None, 0, None, None) == L.RID_EINVAL


def test_split_gram_needs_binary32_data(L):
    lib = L.lib()
    cfg = L.rid_config()
    lib.rid_config_default(C.byref(cfg))
    assert cfg.gram_mode == L.RID_GRAM_AUTO
    cfg.m, cfg.ell, cfg.k, cfg.t, cfg.n_max = 1000, 40, 20, 20, 100
    cfg.data_dtype, cfg.sketch_prec, cfg.gram_mode = L.RID_F64, L.RID_SKETCH_F64, L.RID_GRAM_SPLIT
    h = C.c_void_p()
    assert lib.rid_init_stream(C.byref(cfg), None, C.byref(h)) == L.RID_EINVAL
    buf = C.create_string_buffer(256)
    lib.rid_last_error(None, buf, 256)
    assert b"RID_GRAM_SPLIT" in buf.value


def test_split_gram_with_best_of_four_is_rejected(L):
    lib = L.lib()
    cfg = L.rid_config()
    lib.rid_config_default(C.byref(cfg))
    cfg.m, cfg.ell, cfg.k, cfg.t, cfg.n_max = 1000, 40, 20, 20, 100
    cfg.coeff_mode, cfg.gram_mode = L.RID_COEFF_BEST4, L.RID_GRAM_SPLIT
    h = C.c_void_p()
    assert lib.rid_init_stream(C.byref(cfg), None, C.byref(h)) == L.RID_ENOTSUP


def test_null_handles_are_rejected(L):
    lib = L.lib()
    assert lib.rid_push_snapshots(None, None, 10, 1, 0) == L.RID_EINVAL
    assert lib.rid_finalize(None) == L.RID_EINVAL
    assert lib.rid_destroy(None) == L.RID_EINVAL
    assert lib.rid_omega_block(9, 1, 8, 0, 1, None, 8, None) == L.RID_EINVAL
    assert lib.rid_push_batch(None, None, None, None, 0) == L.RID_EINVAL
    assert lib.rid_finalize_batch(None) == L.RID_EINVAL
    assert lib.rid_destroy_batch(None) == L.RID_EINVAL
    assert lib.rid_batch_stream(None, 0, None) == L.RID_EINVAL


@pytest.mark.parametrize("args,expect,msg", [
    ((9, 1, 40, 1000, 16, 1000, 4, 16, 16, None), "EINVAL", "unknown sketch precision"),
    ((2, 1, 0, 1000, 16, 1000, 4, 16, 16, None), "EINVAL", "bad sizes"),
    ((2, 1, 40, 1000, 16, 999, 4, 16, 16, None), "EINVAL", "bad sizes"),
    ((2, 1, 40, 1000, None, 1000, 4, 16, 16, None), "EINVAL", "bad sizes"),
    ((2, 1, 40, 1000, 8, 1000, 4, 16, 16, None), "EINVAL", "16-byte"),
    ((2, 1, 40, 1001, 16, 1001, 4, 16, 16, None), "EINVAL", "16-byte"),
    # 4096 columns of 50M rows at l = 300: the partial sketches cannot fit
    ((2, 1, 300, 50_000_000, 16, 50_000_000, 4096, 16, 16, None), "ECAPACITY", "MiB work space"),
])
def test_sketch_columns_rejects_bad_arguments_before_device(L, args, expect, msg):
    # every rejected call returns before touching the device (the pointers
    # below are never dereferenced)
    lib = L.lib()
    st = lib.rid_sketch_columns(*args, None)
    assert st == getattr(L, "RID_" + expect)
    buf = C.create_string_buffer(256)
    lib.rid_last_error(None, buf, 256)
    assert msg in buf.value.decode()


def test_invalid_batches_rejected_before_device(L):
    lib = L.lib()
    cfgs = (L.rid_config * 2)()
    for c in cfgs:
        lib.rid_config_default(C.byref(c))
        c.m, c.ell, c.k, c.t, c.n_max = 1000, 40, 20, 20, 100
    b = C.c_void_p()
    assert lib.rid_init_batch(0, cfgs, None, 0, C.byref(b)) == L.RID_EINVAL
    assert lib.rid_init_batch(2, cfgs, None, 64, C.byref(b)) == L.RID_EINVAL
    cfgs[1].k = 41
    assert lib.rid_init_batch(2, cfgs, None, 0, C.byref(b)) == L.RID_EINVAL
    buf = C.create_string_buffer(256)
    lib.rid_batch_last_error(None, buf, 256)
    assert "k must" in buf.value.decode()
    assert not b.value


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2405_16076_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "oracle/" not in text, f
