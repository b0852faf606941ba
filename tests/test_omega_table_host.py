"""Host checks of the library's constant table of Omega's magnitudes
(csrc/omega_table.h, written by csrc/gen_omega_table.py): the committed header
is the generator's output, and every format it holds is the oracle's rounding
of the same binary64 quantile (binary64 itself within a few ulp: the two sides
compute the quantiles with different algorithms)."""
import os
import re
import subprocess
import sys
import tempfile

import numpy as np

from oracle.omega import omega_table, quantize_fp8_omega, round_to_bf16

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_16076_amd", "csrc")
HEADER = os.path.join(CSRC, "omega_table.h")


def _array(text, name):
    body = re.search(name + r"\[kOmegaTabSize\] = \{(.*?)\};", text, re.S).group(1)
    return [v.strip() for v in body.replace("\n", " ").split(",") if v.strip()]


def test_header_is_the_generator_output():
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "omega_table.h")
        code = ("import importlib.util, sys; s = importlib.util.spec_from_file_location('g', sys.argv[1]); "
                "m = importlib.util.module_from_spec(s); s.loader.exec_module(m); m.main(sys.argv[2])")
        subprocess.run([sys.executable, "-c", code, os.path.join(CSRC, "gen_omega_table.py"), out], check=True)
        assert open(out).read() == open(HEADER).read()


def test_every_format_rounds_the_oracle_quantiles():
    text = open(HEADER).read()
    T = omega_table()
    f64 = np.array([float.fromhex(v) for v in _array(text, "kOmegaTabF64")])
    assert np.max(np.abs(f64 - T) / np.spacing(T)) <= 8
    f32 = np.array([int(v.rstrip("u"), 16) for v in _array(text, "kOmegaTabF32")], dtype=np.uint32).view(np.float32)
    assert np.array_equal(f32, T.astype(np.float32))
    b16 = (np.array([int(v, 16) for v in _array(text, "kOmegaTabBf16")], dtype=np.uint32) << 16).view(np.float32)
    assert np.array_equal(b16.astype(np.float64), round_to_bf16(T))

    def e4m3(c):
        e, m = (c >> 3) & 15, c & 7
        return (1 + m / 8) * 2.0 ** (e - 7) if e else m / 8 * 2.0 ** -6

    e8 = np.array([e4m3(int(v, 16)) for v in _array(text, "kOmegaTabE4M3")]) / 64.0
    assert np.array_equal(e8, quantize_fp8_omega(T))


def test_signed_tables_index_the_same_entries():
    """The bfloat16 and e4m3 sketch kernels look Omega entries up in a signed
    2048-entry copy of their table (entry j: entry j mod 1024 with the sign bit
    set for j >= 1024), indexed by bits 15..5 of the Philox half.  Over every
    16-bit half this is the definition's sign-and-magnitude entry:
    (-1)^(bit 15) T[bits 14..5]."""
    text = open(HEADER).read()
    h = np.arange(1 << 16, dtype=np.uint32)
    j = np.arange(2048, dtype=np.uint32)
    for name, sign in (("kOmegaTabBf16", 0x8000), ("kOmegaTabE4M3", 0x80)):
        tab = np.array([int(v, 16) for v in _array(text, name)], dtype=np.uint32)
        signed = tab[j & 1023] | np.where(j & 1024, sign, 0).astype(np.uint32)
        direct = tab[(h >> 5) & 1023] | np.where(h & 0x8000, sign, 0).astype(np.uint32)
        assert np.array_equal(signed[(h >> 5) & 2047], direct)
