"""The measurement copy kernel (df_stream_copy): bitwise copy, argument checks."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_03191_amd as m

    return m


def test_stream_copy_bitwise(dfm):
    import torch

    g = torch.Generator(device="cuda").manual_seed(3)
    for n in (4, 1000, (1 << 20) + 4):
        src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
        dst = torch.zeros_like(src)
        dfm.stream_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src), n


def test_stream_copy_rejects_bad_arguments(dfm):
    import torch

    a = torch.zeros(64, dtype=torch.int32, device="cuda")
    b = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(dfm.DFError):
        dfm.stream_copy(a[1:5], b[:4])  # 4-byte aligned only
    with pytest.raises(dfm.DFError):
        dfm.stream_copy(a[4:36], a[:32])  # overlapping
