"""The allocation-free forward pass of the guess network
(sgw_mlp_forward_noalloc, static device scratch) against sgw_mlp_forward
(work space from the allocator) through the C-ABI: the same kernels on the
same inputs, so the outputs must be bitwise equal; two calls in a row, the
second with a smaller batch (the scratch keeps the first call's values),
and a batch beyond the scratch is rejected."""

import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_forward_matches_forward():
    import paper_2512_23027_amd as sgw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    L = sgw.lib()
    m = sgw.GuessModel(4, 1, 256, seed=5)
    rng = np.random.default_rng(3)
    for nb in (5000, 777):
        print("noalloc forward, batch %d" % nb, flush=True)
        x = torch.from_numpy(rng.standard_normal((nb, 4)).astype(np.float32)).cuda()
        ref = m.forward(x)
        y = torch.full((nb, 1), float("nan"), dtype=torch.float32, device="cuda")
        st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = L.sgw_mlp_forward_noalloc(m.m, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(y.data_ptr()), nb, st)
        assert rc == 0
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
    big = 8193  # 8193 x 2 x 256 floats exceed the 4 Mi-float scratch
    x = torch.zeros((big, 4), dtype=torch.float32, device="cuda")
    y = torch.zeros((big, 1), dtype=torch.float32, device="cuda")
    rc = L.sgw_mlp_forward_noalloc(m.m, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), big,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1  # SGW_EINVAL, nothing launched
    m.close()
