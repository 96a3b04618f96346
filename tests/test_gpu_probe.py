"""The streaming-copy probe used for the measured HBM ceiling copies exactly."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_18205_amd import _abi  # noqa: E402


@pytest.mark.parametrize("nbytes", [0, 16, 4096 + 16, (1 << 22) + 48])
def test_stream_copy_is_exact(nbytes):
    print(f"stream copy {nbytes} bytes", flush=True)
    lib = _abi.load()
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 255, (nbytes + 64,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.rbffd_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes, st) == 0
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].sum()) == 0


def test_stream_copy_rejects_bad_arguments_on_the_host():
    lib = _abi.load()
    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    p = a.data_ptr()
    assert lib.rbffd_stream_copy(C.c_void_p(p), C.c_void_p(p + 32), 15, None) == _abi.EINVAL
    assert lib.rbffd_stream_copy(C.c_void_p(p + 8), C.c_void_p(p + 32), 16, None) == _abi.EINVAL
    assert lib.rbffd_stream_copy(None, C.c_void_p(p), 16, None) == _abi.EINVAL
