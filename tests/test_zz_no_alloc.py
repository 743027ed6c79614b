"""The allocation-free sort (gs_sort_pairs_static, for callers that cannot
allocate) against gs_sort_pairs with a caller workspace, through the C ABI:
bit-exact on two calls in a row, the second smaller than the first, plus the
capacity limit."""
import ctypes

import numpy as np
import pytest
import torch

import gs_inputs

pytestmark = pytest.mark.gpu


def _pairs(n, bits, seed):
    g = gs_inputs.rng(seed)
    keys = g.integers(0, 1 << min(bits, 62), size=n, dtype=np.uint64)
    keys[: n // 7] = keys[n // 3: n // 3 + n // 7]  # equal keys: ties keep the value order
    return keys, np.arange(n, dtype=np.uint32)[::-1].copy()


def _dev(keys, vals):
    return (torch.from_numpy(keys.view(np.int64).copy()).cuda(), torch.from_numpy(vals.view(np.int32).copy()).cuda())


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


@pytest.mark.parametrize("sizes", [((700_001, 45), (50_003, 33)), ((1 << 20, 64), (1, 8))])
def test_static_sort_equals_workspace_sort(gpu_lib, sizes):
    from paper_2411_12788_amd import _lib as L
    lib = L.lib()
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for call, (n, bits) in enumerate(sizes):
        print(f"static sort call {call}: n={n} bits={bits}", flush=True)
        keys, vals = _pairs(n, bits, 100 + n + bits)
        ka, va = _dev(keys, vals)
        kb, vb = _dev(keys, vals)
        ws = torch.empty(lib.gs_sort_workspace_size(n), dtype=torch.uint8, device="cuda")
        assert lib.gs_sort_pairs(_p(ka), _p(va), n, bits, _p(ws), ws.numel(), None) == L.GS_OK
        assert lib.gs_sort_pairs_static(_p(kb), _p(vb), n, bits, _p(status), None) == L.GS_OK
        torch.cuda.synchronize()
        assert status.item() == 0
        assert torch.equal(ka, kb) and torch.equal(va, vb)
        perm = np.lexsort((np.arange(n), keys & np.uint64((1 << bits) - 1) if bits < 64 else keys))
        assert np.array_equal(vb.cpu().numpy().view(np.uint32), vals[perm])
        status.fill_(7)


def test_static_sort_limits(gpu_lib):
    from paper_2411_12788_amd import _lib as L
    lib = L.lib()
    k = torch.zeros(4, dtype=torch.int64, device="cuda")
    v = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    assert lib.gs_sort_pairs_static(_p(k), _p(v), L.GS_SORT_STATIC_MAX_PAIRS + 1, 40, None, None) == L.GS_ERR_CAPACITY
    assert b"GS_SORT_STATIC_MAX_PAIRS" in lib.gs_last_error()
    assert lib.gs_sort_pairs_static(_p(k), _p(v), 0, 40, _p(st), None) == L.GS_OK
    torch.cuda.synchronize()
    assert st.item() == 0
