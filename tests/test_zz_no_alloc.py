"""te_knn_counts_noalloc (static device scratch, no allocation in the call) against
te_knn_counts (caller workspace) through the C interface: radii, the three counts and
the estimates identical bit for bit, on two calls in a row (the second smaller, other
dimensions), and the size limit rejected on the host."""
import sys

import numpy as np
import pytest

from synth.rng import derive_key, normal64

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def te():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_4068_amd as te
    te.lib()
    return te


def _soa(sizes, D, seed):
    off = np.zeros(len(sizes) + 1, np.int64)
    off[1:] = np.cumsum(sizes)
    stride = int(off[-1]) + 19
    soa = np.zeros((D, stride), np.float32)
    soa[:, :off[-1]] = normal64(derive_key(seed, D, len(sizes)), int(off[-1]) * D).reshape(-1, D).T
    return soa, off


def _both(te, sizes, d_y, d_x, k, seed):
    import torch
    D = 1 + d_y + d_x
    soa, off = _soa(sizes, D, seed)
    total = int(off[-1])
    say("no-alloc case", dict(sizes=sizes, d_y=d_y, d_x=d_x, k=k, seed=seed))
    pts = torch.from_numpy(soa).cuda()
    eps_ws, cnt_ws, te_ws = te.knn_counts(pts, off, d_y, d_x, k)
    # outputs pre-filled with garbage: every entry must be written
    eps = torch.full((total,), -7.0, dtype=torch.float32, device="cuda")
    cnt = torch.full((3, total), -7, dtype=torch.int32, device="cuda")
    te_na = te.knn_counts_noalloc(pts, off, d_y, d_x, k, eps, cnt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(eps.cpu().numpy(), eps_ws.cpu().numpy())
    np.testing.assert_array_equal(cnt.cpu().numpy(), cnt_ws.cpu().numpy())
    np.testing.assert_array_equal(te_na, te_ws)
    assert np.all(np.isfinite(te_na))


def test_noalloc_matches_workspace_entry_two_calls(te):
    # first call: several chunks, one above the LDS sort size (global sort scratch)
    _both(te, [20000, 4100, 700, 33], 3, 3, 4, seed=1)
    # second call, smaller and of other dimensions: the scratch keeps the first call's contents
    _both(te, [900, 65, 6], 2, 1, 5, seed=2)


def test_noalloc_rejects_inputs_beyond_its_scratch(te):
    import torch
    from paper_1401_4068_amd._lib import NOALLOC_SCRATCH_BYTES, TEError
    total = 700_000
    need = te.lib().te_knn_counts_workspace_bytes(1, total)
    assert need > NOALLOC_SCRATCH_BYTES
    pts = torch.zeros((5, total), dtype=torch.float32, device="cuda")
    eps = torch.empty(total, dtype=torch.float32, device="cuda")
    cnt = torch.empty((3, total), dtype=torch.int32, device="cuda")
    with pytest.raises(TEError, match="static scratch holds"):
        te.knn_counts_noalloc(pts, np.array([0, total], np.int64), 2, 2, 4, eps, cnt)
    # the entry point still works afterwards
    _both(te, [300, 129], 2, 2, 4, seed=3)
