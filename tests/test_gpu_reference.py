"""The bandwidth reference beside the sweep (hlbm_ref_stream_pattern): one
pull-streaming pass of the 19 FP32 rows of a periodic box, with the sweep's
row pitch and block widths, equals the pull written out in numpy from the
velocity set (dst_i(x) = src_i(x - c_i), periodic wrap); the porosity read
leaves the values alone; bad arguments are rejected."""
import ctypes

import numpy as np
import pytest

from tests.test_gpu_parity import H, say  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,pad,bx", [((37, 9, 6), 0, 64), ((70, 5, 4), 256, 128), ((256, 3, 2), 8448, 256)])
def test_stream_pattern_is_the_pull(H, shape, pad, bx):
    import torch
    nx, ny, nz = shape
    n = nx * ny * nz
    P = n + pad // 4
    say(f"stream pattern {shape}, pad {pad}, block {bx}")
    rng = np.random.default_rng(nx)
    src = rng.standard_normal((19, n)).astype(np.float32)
    a = torch.zeros(19 * P, dtype=torch.float32, device="cuda")
    for i in range(19):
        a[i * P:i * P + n] = torch.from_numpy(src[i])
    b = torch.full((19 * P,), 5.0, dtype=torch.float32, device="cuda")
    d = torch.from_numpy(rng.random(n).astype(np.float32)).cuda()
    lib = H.load()
    rc = lib.hlbm_ref_stream_pattern(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                     ctypes.c_void_p(d.data_ptr()), nx, ny, nz, pad, bx, None)
    assert rc == 0
    torch.cuda.synchronize()
    got = b.cpu().numpy().reshape(19, P)
    c, _ = H.lattice_info(19)
    for i in range(19):
        want = np.roll(src[i].reshape(nz, ny, nx), shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2)).ravel()
        assert np.array_equal(got[i, :n], want), i
        assert (got[i, n:] == 5.0).all()          # the pad is not written


def test_stream_pattern_rejects_bad_arguments(H):
    import torch
    lib = H.load()
    t = torch.zeros(19 * 64, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(t.data_ptr())
    assert lib.hlbm_ref_stream_pattern(None, p, p, 4, 4, 4, 0, 64, None) == H.EINVAL
    assert lib.hlbm_ref_stream_pattern(p, p, p, 0, 4, 4, 0, 64, None) == H.EINVAL
    assert lib.hlbm_ref_stream_pattern(p, p, p, 4, 4, 4, 2, 64, None) == H.EINVAL
    assert lib.hlbm_ref_stream_pattern(p, p, p, 4, 4, 4, 0, 96, None) == H.EINVAL
