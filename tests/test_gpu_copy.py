"""The library's streaming copy (the practical-HBM-rate reference): exact copy
of sizes that exercise the four-wide body and the tail, and argument checks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("nbytes", [16, 4096, 16 * 1000003, 64 << 20])
def test_copy_is_exact(nbytes):
    from paper_2309_06427_amd import _lib
    lib = _lib.load()
    g = torch.Generator(device="cpu").manual_seed(nbytes % 1000)
    src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4 + 8,), dtype=torch.int32, generator=g).cuda()
    dst = torch.zeros_like(src)
    _lib.check(lib.ssp_copy_bytes(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream),
               "ssp_copy_bytes")
    torch.cuda.synchronize()
    k = nbytes // 4
    assert torch.equal(dst[:k], src[:k])
    assert (dst[k:] == 0).all()  # nothing written past the end


def test_copy_rejects_misaligned_sizes_and_pointers():
    from paper_2309_06427_amd import _lib
    lib = _lib.load()
    src = torch.zeros(64, dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.ssp_copy_bytes(src.data_ptr(), dst.data_ptr(), 20, s) == _lib.SSP_ERR_ARG
    assert lib.ssp_copy_bytes(src.data_ptr() + 4, dst.data_ptr(), 16, s) == _lib.SSP_ERR_ARG
    assert lib.ssp_copy_bytes(src.data_ptr(), dst.data_ptr(), 0, s) == 0
