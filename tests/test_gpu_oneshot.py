"""GPU parity of the one-shot sketch (rid_sketch_columns, through the C ABI):
S = Omega A and the column norms of a block of snapshots against the oracle's
product of the same operands, with the bounds of the stream's sketch (relative
Frobenius and worst column), norms to 1e-13, and the non-finite flag."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import S_COL_BOUND, col_max_rel, log, rel_fro

pytestmark = pytest.mark.gpu

S_FRO_BOUND = {"f64": 1e-12, "f32": 2e-5, "bf16": 1e-5, "fp8": 1e-3}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_16076_amd import _lib
    _lib.lib()


def _device_block(A, ld=None):
    """(b, m) host array -> (b, m) device view with rows ld elements apart."""
    b, m = A.shape
    ld = ld or (m + 15) // 16 * 16
    dt = torch.float64 if A.dtype == np.float64 else torch.float32
    Xp = torch.zeros((b, ld), dtype=dt, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(A).to("cuda:0")
    return Xp[:, :m]


@pytest.mark.parametrize("sketch,m,b,ell", [
    ("f64", 4096, 37, 40), ("f64", 20_001, 64, 71),
    ("f32", 100_003, 33, 40), ("f32", 65_536, 300, 200),
    ("bf16", 100_003, 45, 40), ("bf16", 1_000_000, 16, 300), ("bf16", 70_000, 257, 300),
    # one ragged 64-row chunk (a 16-byte piece straddles the last row), and two
    # chunks plus one row over two column tiles; l not a multiple of 8
    ("bf16", 37, 5, 13), ("bf16", 129, 260, 70),
    ("fp8", 100_003, 45, 40), ("fp8", 65_536, 300, 300),
])
def test_sketch_columns_matches_oracle(sketch, m, b, ell):
    from paper_2405_16076_amd import sketch_columns
    log("one-shot sketch", sketch, m, b, ell)
    rng = np.random.default_rng(m + b)
    A = rng.standard_normal((b, m)).astype(np.float64 if sketch == "f64" else np.float32)
    X = _device_block(A)
    S, q, flag = sketch_columns(X, ell, 91, sketch)
    torch.cuda.synchronize()
    S, q = S.cpu().numpy(), q.cpu().numpy()
    So, qo = oracle.sketch_columns(A.T, 91, ell, operand=sketch)
    e, ec = rel_fro(S, So), col_max_rel(S, So)
    log(f"  S rel fro {e:.2e} col {ec:.2e}; norms max rel {np.max(np.abs(q - qo) / qo):.2e}")
    assert e <= S_FRO_BOUND[sketch] and ec <= S_COL_BOUND[sketch]
    assert np.max(np.abs(q - qo) / qo) <= 1e-13
    assert int(flag.item()) == 0


def test_sketch_columns_flags_non_finite_columns():
    from paper_2405_16076_amd import sketch_columns
    A = np.ones((5, 3000), dtype=np.float32)
    A[3, 1234] = np.nan
    X = _device_block(A)
    S, q, flag = sketch_columns(X, 40, 3, "bf16")
    torch.cuda.synchronize()
    assert int(flag.item()) == 1
    q = q.cpu().numpy()
    assert np.all(np.isfinite(q[[0, 1, 2, 4]])) and not np.isfinite(q[3])
    # the flag is cleared by the next call
    A[3, 1234] = 1.0
    S, q, flag = sketch_columns(_device_block(A), 40, 3, "bf16")
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
