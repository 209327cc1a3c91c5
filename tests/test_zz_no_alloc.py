"""kct_project_noalloc, the forward projection that allocates nothing (for
callers that cannot call hipMalloc), through the C ABI, against kct_project
with a caller workspace: both run the same kernels on the same z-fastest copy,
so they must agree bit for bit.  Two calls in a row, the second on a smaller
input (the shared scratch keeps the first call's contents; the second must not
see them), then a 16-bit call; a volume beyond the fixed scratch is refused
with KCT_ERR_WORKSPACE before anything runs.  After the first call, further
calls leave the device's free memory unchanged."""
import ctypes

import numpy as np
import pytest

import kct_inputs as ki
from tests.gpu_util import dev, geometry, say, torch_mod

pytestmark = pytest.mark.gpu


def _noalloc(G, x, b):
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd import _lib
    return _lib.load().kct_project_noalloc(G.handle, kct._dtype_code(x.dtype), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(b.data_ptr()), kct._stream_handle(G.device))


def _case(g, seed, dtype):
    import paper_2110_13526_amd as kct
    torch = torch_mod()
    G = geometry(g)
    x = torch.from_numpy(ki.phantom(g, 8, seed)).to(dev()).to(dtype)
    ref = kct.project(G, x)  # with a workspace (the z-fastest copy in caller memory)
    out = torch.full(g.proj_shape, float("nan"), dtype=dtype, device=dev())
    st = _noalloc(G, x, out)
    torch.cuda.synchronize()
    return G, x, ref, out, st


def test_noalloc_projection_equals_workspace_projection():
    from paper_2110_13526_amd import _lib
    torch = torch_mod()
    big = ki.config("c5")                       # 192^3, 180 views, 256 x 256
    small = ki.config("c1")                     # 64^3, 90 views, 96 x 96
    say(f"[noalloc] call 1: {big.vol_shape} FP32")
    G1, x1, ref1, out1, st1 = _case(big, 11, torch.float32)
    assert st1 == _lib.KCT_OK, _lib.load().kct_last_error()
    assert torch.equal(out1, ref1)
    free0 = torch.cuda.mem_get_info()[0]
    say(f"[noalloc] call 2: {small.vol_shape} FP32 (smaller, after the larger one)")
    G2, x2, ref2, out2, st2 = _case(small, 12, torch.float32)
    assert st2 == _lib.KCT_OK, _lib.load().kct_last_error()
    assert torch.equal(out2, ref2)
    # a repeat of the small call allocates nothing
    free1 = torch.cuda.mem_get_info()[0]
    out3 = torch.empty_like(out2)
    free2 = torch.cuda.mem_get_info()[0]
    assert _noalloc(G2, x2, out3) == _lib.KCT_OK
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free2
    assert torch.equal(out3, ref2)
    say(f"[noalloc] free memory {free0} -> {free1} (torch tensors of the second case) -> {free2}, unchanged by the call")
    say("[noalloc] call 4: t16 off-centre BF16")
    G4, x4, ref4, out4, st4 = _case(ki.t16("offcenter"), 13, torch.bfloat16)
    assert st4 == _lib.KCT_OK, _lib.load().kct_last_error()
    assert torch.equal(out4, ref4)


def test_noalloc_refuses_a_volume_beyond_the_scratch():
    import paper_2110_13526_amd as kct
    from paper_2110_13526_amd import _lib
    torch = torch_mod()
    g = ki.config("c3").replace(n_views=4)      # 512^3 FP32 = 512 MiB > 64 MiB
    G = geometry(g)
    x = torch.zeros(1, dtype=torch.float32, device=dev())  # never read: refused before any launch
    b = torch.zeros(1, dtype=torch.float32, device=dev())
    st = _lib.load().kct_project_noalloc(G.handle, _lib.KCT_F32, ctypes.c_void_p(x.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), kct._stream_handle(G.device))
    assert st == _lib.KCT_ERR_WORKSPACE
    msg = _lib.load().kct_last_error().decode()
    say(f"[noalloc] refused: {msg}")
    assert "scratch" in msg
    assert g.n_vox * 4 > _lib.NOALLOC_SCRATCH_BYTES
    # 256^3 FP32 is exactly the scratch size and is accepted by the size check
    assert 256 ** 3 * 4 == _lib.NOALLOC_SCRATCH_BYTES
    assert np.isfinite(float(b.sum().item()))
