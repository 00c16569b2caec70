"""tvc_contract_noalloc (scratch in the library's fixed device array) against
tvc_contract (scratch in a caller workspace), called through the C ABI: the
same bits, on two calls in a row with the second input smaller, for shapes
whose contraction uses scratch (split contracted extents, E4M3 mode-0
weights), plus the size limit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2501_03121_amd import _lib as L
from paper_2501_03121_amd import core
from _util import host, stored_tensor, vec

pytestmark = pytest.mark.gpu


def _pair(dims, fmt, k, seed, dev):
    lib = L.lib()
    A, S, _ = stored_tensor(dims, fmt, seed, dev)
    x, _ = vec(dims[k], seed + 1, fmt, dev)
    desc = core.describe(A, S)
    need = lib.tvc_contract_workspace_bytes(desc, k)
    acc = torch.float64 if fmt == "f64" else torch.float32
    n_out = A.numel() // dims[k]
    y_ref = torch.empty(n_out, dtype=acc, device=dev)
    y_na = torch.full((n_out,), float("nan"), dtype=acc, device=dev)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=dev)
    wp = (ws.data_ptr() + 255) & ~255
    sh = torch.cuda.current_stream().cuda_stream
    L.check(lib.tvc_contract(desc, k, x.data_ptr(), y_ref.data_ptr(), 1.0, 0.0, wp, need, sh))
    L.check(lib.tvc_contract_noalloc(desc, k, x.data_ptr(), y_na.data_ptr(), 1.0, 0.0, sh))
    torch.cuda.synchronize()
    return need, y_ref, y_na


# (large case, smaller case): each pair contracts a split extent or E4M3
# mode-0 weights, so both calls put data in the shared scratch array
CASES = [
    (((1000003,), "f32", 0), ((200001,), "f32", 0)),
    (((3, 50000, 4), "f64", 1), ((3, 9000, 4), "f64", 1)),
    (((5, 2, 70001), "bf16", 2), ((5, 2, 30001), "bf16", 2)),
    (((1000003,), "e4m3", 0), ((70001,), "e4m3", 0)),
    (((3000, 1001), "f32", 0), ((1500, 1001), "f32", 0)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0][1]}-{'x'.join(map(str, c[0][0]))}")
def test_noalloc_matches_workspace_call(dev, case):
    for i, (dims, fmt, k) in enumerate(case):
        need, y_ref, y_na = _pair(dims, fmt, k, 40 + i, dev)
        assert 0 < need <= L.lib().tvc_contract_noalloc_max_scratch(), (dims, fmt, need)
        assert torch.equal(y_ref, y_na), (dims, fmt, k, i)


def test_noalloc_without_scratch_and_with_beta(dev):
    lib = L.lib()
    dims = (33, 40, 17)
    A, _, _ = stored_tensor(dims, "f32", 5, dev)
    desc = core.describe(A)
    sh = torch.cuda.current_stream().cuda_stream
    for k in range(3):
        x, _ = vec(dims[k], 6 + k, "f32", dev)
        y0 = torch.randn(A.numel() // dims[k], device=dev)
        y1 = y0.clone()
        L.check(lib.tvc_contract(desc, k, x.data_ptr(), y0.data_ptr(), 0.5, -2.0, None, 0, sh))
        L.check(lib.tvc_contract_noalloc(desc, k, x.data_ptr(), y1.data_ptr(), 0.5, -2.0, sh))
        torch.cuda.synchronize()
        assert torch.equal(y0, y1)


def test_noalloc_rejects_oversized_scratch(dev):
    # a 1-D contraction of 3,000,001 E4M3 values needs 12 MB of scaled
    # weights, above the 8 MiB array: rejected before anything is launched
    lib = L.lib()
    n = 3000001
    A = torch.empty(n, dtype=torch.uint8, device=dev)
    S = torch.ones(n, dtype=torch.float32, device=dev)
    desc = L.make_tensor(1, (n,), L.TVC_F8E4M3, A.data_ptr(), S.data_ptr())
    assert lib.tvc_contract_workspace_bytes(desc, 0) > lib.tvc_contract_noalloc_max_scratch()
    x = torch.zeros(n, dtype=torch.float32, device=dev)
    y = torch.zeros(1, dtype=torch.float32, device=dev)
    st = lib.tvc_contract_noalloc(desc, 0, x.data_ptr(), y.data_ptr(), 1.0, 0.0,
                                  torch.cuda.current_stream().cuda_stream)
    assert st == L.TVC_EWORKSPACE
    assert b"tvc_contract_noalloc" in lib.tvc_last_error()
