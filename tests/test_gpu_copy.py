"""lbm_device_copy, the plain-copy bandwidth reference: bitwise copies of
ragged sizes (not multiples of one workgroup's 16 KiB), bytes past the end
untouched, zero bytes a no-op."""
import pytest
import torch

from paper_1202_6130_amd import lbm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [0, 16, 4096 + 16, (1 << 20) + 48, (64 << 20) + 16384 + 80])
def test_device_copy_bitwise(nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    pad = 4096
    src = torch.randint(0, 256, (nbytes + pad,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.full((nbytes + pad,), 7, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    lbm.lbm_device_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert bool((dst[nbytes:] == 7).all())
