"""vif_mlp_forward_noalloc (no workspace argument, no device allocation; the
hidden layers in the library's fixed per-device array) against
vif_mlp_forward with a caller workspace, through the C ABI: identical outputs
(the same kernels on the same rows), on two calls in a row, the first with
more rows than one chunk of the fixed array holds (several chunks), the
second smaller, so a chunk of the second call reuses array memory that the
first call left filled."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _call_noalloc(lib, params, X, F, H, out32, out64):
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    return lib.vif_mlp_forward_noalloc(p(params), p(X), X.shape[0], F, H, p(out32), p(out64), st)


def _call_ws(lib, params, X, F, H, out32, out64):
    n = X.shape[0]
    ws = torch.empty(int(lib.vif_mlp_workspace_floats(n, F, H)), dtype=torch.float32, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    return lib.vif_mlp_forward(p(params), p(X), n, F, H, p(ws), p(out32), p(out64), st)


@pytest.mark.parametrize("H", [128, 512])
def test_noalloc_forward_matches_workspace_forward(H):
    from paper_2507_05064_amd.vif import WarmStartMLP, load_library
    lib = load_library()
    F = 16
    mlp = WarmStartMLP(H=H, seed=11)
    g = torch.Generator(device="cpu").manual_seed(H)
    rows = (6 * 1024 * 1024) // (3 * H) // 64 * 64
    for n in (2 * rows + 777, 1001):  # several chunks, then a smaller call
        print(f"[gpu] no-alloc MLP forward H={H} n={n}", flush=True)
        X = torch.randn((n, F), generator=g, dtype=torch.float32).to("cuda")
        ref32 = torch.empty(n, dtype=torch.float32, device="cuda")
        ref64 = torch.empty(n, dtype=torch.float64, device="cuda")
        assert _call_ws(lib, mlp.params, X, F, H, ref32, ref64) == 0
        got32 = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
        got64 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        assert _call_noalloc(lib, mlp.params, X, F, H, got32, got64) == 0
        torch.cuda.synchronize()
        assert torch.equal(got32, ref32) and torch.equal(got64, ref64)
        assert float(ref32.abs().max()) > 0


def test_noalloc_forward_rejects_bad_sizes():
    from paper_2507_05064_amd.vif import WarmStartMLP, load_library
    lib = load_library()
    mlp = WarmStartMLP(H=128, seed=1)
    X = torch.zeros((10, 16), dtype=torch.float32, device="cuda")
    out = torch.empty(10, dtype=torch.float32, device="cuda")
    assert _call_noalloc(lib, mlp.params, X, 16, 1024, out, None) == 1   # H > 512
    assert _call_noalloc(lib, mlp.params, X, 65, 128, out, None) == 1    # F > 64
    assert _call_noalloc(lib, mlp.params, X, 16, 128, None, None) == 1   # no output
