"""GPU test of the allocation-free one-shot sketch (rid_sketch_columns_noalloc,
through the C ABI): two calls in a row on the library's fixed work space, the
second with a smaller input, each equal bit for bit to rid_sketch_columns on
the same input (same slab geometry and kernels), for every sketch form; a call
whose work space would pass the fixed maximum is rejected before the device."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_16076_amd import _lib
    _lib.lib()


def _block(rng, b, m, dt):
    ld = (m + 15) // 16 * 16
    Xp = torch.zeros((b, ld), dtype=dt, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(rng.standard_normal((b, m))).to(dt).to("cuda:0")
    return Xp[:, :m]


@pytest.mark.parametrize("sketch,big,small,ell", [
    ("bf16", (300, 200_003), (17, 70_001), 300),
    ("fp8", (256, 100_000), (40, 30_017), 300),
    ("f32", (300, 65_536), (33, 4_097), 200),
    ("f64", (64, 50_001), (9, 3_001), 40),
])
def test_noalloc_matches_allocating_call_twice(sketch, big, small, ell):
    from paper_2405_16076_amd import sketch_columns
    from paper_2405_16076_amd.stream import sketch_columns_noalloc
    rng = np.random.default_rng(ell + big[0])
    dt = torch.float64 if sketch == "f64" else torch.float32
    for b, m in (big, small):
        log(f"no-alloc sketch {sketch} b={b} m={m} l={ell}")
        X = _block(rng, b, m, dt)
        S_ref, q_ref, f_ref = sketch_columns(X, ell, 123, sketch)
        S = torch.full((b, ell), float("nan"), dtype=torch.float64, device="cuda:0")
        q = torch.full((b,), float("nan"), dtype=torch.float64, device="cuda:0")
        f = torch.full((1,), 7, dtype=torch.int32, device="cuda:0")
        sketch_columns_noalloc(X, ell, 123, sketch, S, q, f)
        torch.cuda.synchronize()
        assert torch.equal(S.T, S_ref) and torch.equal(q, q_ref)
        assert int(f.item()) == 0 and int(f_ref.item()) == 0


def test_noalloc_rejects_work_space_overflow_before_device():
    from paper_2405_16076_amd import _lib as L
    # 4096 columns of 50M rows at l = 300 need far more than the fixed work
    # space: rejected on the host (the pointers are never dereferenced)
    st = L.lib().rid_sketch_columns_noalloc(2, 1, 300, 50_000_000, C.c_void_p(16), 50_000_000, 4096,
                                            C.c_void_p(16), C.c_void_p(16), None, None)
    assert st == L.RID_ECAPACITY
    buf = C.create_string_buffer(256)
    L.lib().rid_last_error(None, buf, 256)
    assert "MiB work space" in buf.value.decode()
