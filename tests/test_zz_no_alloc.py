"""ubs_relocate_noalloc (the relocation with its workspace in a static device
array, for callers that cannot allocate) against ubs_relocate with a
caller workspace, through the C ABI: two calls in a row, the second on a
smaller scene, so the second call runs on the array the first one left.
Relocation is deterministic (integer atomics only), so every output is
compared bit for bit."""
import numpy as np
import pytest
import torch

from _gpu_common import gpu_ready, log, to_dev
from oracle.preprocess import field_slices, n_params

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_ready(), reason="needs a GPU")]


def _scene(dim, rot, n, dead_frac, seed):
    rng = np.random.default_rng(seed)
    F = n_params(dim, rot)
    P = rng.normal(size=(F, n)).astype(np.float32)
    o = rng.uniform(0.0, 1.0, size=n)
    o[rng.uniform(size=n) < dead_frac] = 0.001
    P[field_slices(dim, rot)["o"].start] = o.astype(np.float32)
    M = rng.normal(size=(F, n)).astype(np.float32)
    V = np.abs(rng.normal(size=(F, n))).astype(np.float32)
    return P, M, V, rng.uniform(size=n)


def _relocate(noalloc, P, M, V, u, dim, rot):
    from paper_2510_03312_amd import _lib
    n = P.shape[1]
    p, m, v = to_dev(P), to_dev(M), to_dev(V)
    uu = torch.from_numpy(u).cuda()
    tg = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    if noalloc:
        _lib.ubs_relocate_noalloc(dim, rot, n, p.data_ptr(), m.data_ptr(), v.data_ptr(),
                                  uu.data_ptr(), 0.005, tg.data_ptr(), nd.data_ptr(), s)
    else:
        need = _lib.ubs_relocate(dim, rot, n, 0, 0, 0, 0, 0.005, 0, 0, 0, 0, 0)
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        _lib.ubs_relocate(dim, rot, n, p.data_ptr(), m.data_ptr(), v.data_ptr(), uu.data_ptr(),
                          0.005, ws.data_ptr(), ws.numel(), tg.data_ptr(), nd.data_ptr(), s)
    torch.cuda.synchronize()
    k = int(nd.item())
    return p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy(), tg.cpu().numpy()[:k], k


def test_noalloc_relocate_matches_relocate_on_consecutive_calls():
    from paper_2510_03312_amd import _lib
    cases = [(7, 0, 1_500_000, 0.3, 1), (6, 1, 200_003, 0.5, 2)]   # second call smaller
    for dim, rot, n, dead, seed in cases:
        log(f"[noalloc] relocate dim {dim} rot {rot} n {n}")
        P, M, V, u = _scene(dim, rot, n, dead, seed)
        ref = _relocate(False, P, M, V, u, dim, rot)
        got = _relocate(True, P, M, V, u, dim, rot)
        assert ref[4] == got[4] and ref[4] > 0
        for a, b in zip(ref[:4], got[:4]):
            np.testing.assert_array_equal(a, b)
    # beyond the static workspace: rejected on the host, nothing launched
    big = _lib.UBS_RELOCATE_NOALLOC_MAX_N + 1
    code = _lib.ubs_relocate_noalloc(7, 0, big, 0, 0, 0, 0, 0.005, 0, 0, 0, check=False)
    assert code == _lib.UBS_ERR_CAPACITY
