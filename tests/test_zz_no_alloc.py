"""The allocation-free norm reduction (bbwadg_l2norm2_noalloc) against bbwadg_l2norm2,
through the C ABI: equal bit for bit, on two calls in a row, the second with a smaller input
(fewer elements, lower degree, single precision)."""
import ctypes as C

import numpy as np
import pytest

from workloads import kuhn_cube_mesh, random_state

pytestmark = pytest.mark.gpu


def test_l2norm2_noalloc_equals_l2norm2():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_1808_08645_amd as bb
    lib = bb.load_library()
    for cells, N, M, dtype, seed in ((6, 5, 2, "f64", 71), (2, 3, 1, "f32", 72)):
        print(f"[noalloc] cube {cells}^3x6 N={N} {dtype}", flush=True)
        xyz, etov = kuhn_cube_mesh(cells)
        s = bb.Solver(xyz, etov, N, M, dtype=dtype)
        q = s.to_device(random_state(seed, s.K, s.Np))
        ref = s.l2norm2(q)
        out = torch.full((4,), np.nan, dtype=torch.float64, device="cuda")
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.bbwadg_l2norm2_noalloc(s._ctx, C.c_void_p(q.data_ptr()), C.c_void_p(out.data_ptr()), stream)
        assert rc == 0, bb.load_library().bbwadg_last_error()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref), (got, ref)
        # the binding's wrapper gives the same, and a NULL output is rejected
        assert np.array_equal(s.l2norm2_noalloc(q).cpu().numpy(), ref)
        assert lib.bbwadg_l2norm2_noalloc(s._ctx, C.c_void_p(q.data_ptr()), None, stream) == -1  # EINVAL
        s.close()
