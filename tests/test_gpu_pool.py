"""The pool of basis columns under the split Gram (binary32 data).

Inside a flush the split Gram reads the columns selected during the flush
from the caller's borrowed snapshots and copies into the pool, at the
flush's last update, only those still in the basis (a column that enters and
leaves the basis within one flush is never copied; when the last update
brings no column a copy kernel does it).  Once the release watermark passes
a column the caller may overwrite it: here every released column of the
borrowed buffer is overwritten with NaN, and rid_reconstruct must still
return A_J P from the pool, equal to the product of the original bytes with
the stream's own J and P (binary64 on the host)."""
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


def _run(A, ell, t, lookahead, push, gram="auto"):
    from paper_2405_16076_amd import OnlineRID, StreamConfig
    n, m = A.shape
    cfg = StreamConfig(m=m, ell=ell, k=t, t=t, n_max=n, dtype=torch.float32, sketch="f32", omega_seed=61,
                       select_seed=62, lookahead=lookahead, gram=gram)
    s = OnlineRID(cfg)
    ld = (m + 15) // 16 * 16
    Xp = torch.zeros((n, ld), dtype=torch.float32, device="cuda:0")
    Xp[:, :m] = torch.from_numpy(A).to("cuda:0")
    X = Xp[:, :m]
    released = 0
    for j0 in range(0, n, push):
        s.push(X[j0:j0 + push], borrow=True)
        wm = int(s.info().release_watermark)
        if wm > released:            # the caller reuses what the library released
            Xp[released:wm].fill_(float("nan"))
            released = wm
    s.finalize()
    assert int(s.info().release_watermark) == n
    Xp.fill_(float("nan"))
    torch.cuda.synchronize()
    J, P = s.select(), s.coefficients()
    occ = np.flatnonzero(J >= 0)
    R = s.reconstruct(0, n).double().cpu().numpy()
    Ro = P[occ].T @ A[J[occ]].astype(np.float64)
    err = float(np.linalg.norm(R - Ro) / np.linalg.norm(Ro))
    fills = [s.update(u)["n_filled"] for u in range(int(s.info().n_updates))]
    log(f"  fills per update {fills}; reconstruction after the buffer was overwritten: rel {err:.2e}")
    assert np.isfinite(R).all()
    assert err <= 1e-6, err
    s.close()
    return fills


def test_one_flush_columns_entering_and_leaving():
    # columns growing in norm make earlier ones lose leverage: slots refill at
    # most updates of the single flush (lookahead >= n)
    rng = np.random.default_rng(71)
    n, m, t = 400, 20_011, 40
    A = (rng.standard_normal((n, m)) * (1.03 ** np.arange(n))[:, None]).astype(np.float32)
    fills = _run(A, 2 * t, t, 1024, 100)
    assert sum(fills[1:]) > 0, fills


def test_one_flush_whose_last_update_brings_nothing():
    # the snapshots after the first t are zero: no later update prunes or
    # fills, so the flush's last update runs no Gram and the copy kernel moves
    # the first update's columns into the pool
    rng = np.random.default_rng(72)
    n, m, t = 120, 9_001, 40
    A = np.zeros((n, m), dtype=np.float32)
    A[:t] = rng.standard_normal((t, m)).astype(np.float32)
    fills = _run(A, 2 * t, t, 1024, n)
    assert fills[0] == t and fills[-1] == 0, fills


def test_streaming_flushes_with_released_columns_overwritten():
    rng = np.random.default_rng(73)
    n, m, t = 480, 12_007, 40
    A = (rng.standard_normal((n, m)) * (1.02 ** np.arange(n))[:, None]).astype(np.float32)
    fills = _run(A, 2 * t, t, 2 * t, t)
    assert sum(fills[1:]) > 0, fills


def test_exact_gram_pool_unchanged():
    # binary64 products copy each update's new columns at once: the same
    # overwrite must leave the reconstruction intact
    rng = np.random.default_rng(74)
    n, m, t = 240, 8_011, 40
    A = (rng.standard_normal((n, m)) * (1.03 ** np.arange(n))[:, None]).astype(np.float32)
    _run(A, 2 * t, t, 1024, 80, gram="exact")
