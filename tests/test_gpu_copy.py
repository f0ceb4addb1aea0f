"""The bandwidth reference kernels of fe_stream_copy: an out-of-place copy
and the in-place rewrite (dst == src) return the source bytes exactly, for
both variants and sizes with a ragged last workgroup."""
import pytest

torch = pytest.importorskip("torch")
import paper_1412_8398_amd as fe  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nontemporal", [False, True])
@pytest.mark.parametrize("nvec", [1, 2047, 32768, 1000003])
def test_copy_and_in_place_rewrite_are_exact(nvec, nontemporal):
    g = torch.Generator(device="cuda").manual_seed(nvec)
    src = torch.randint(-(2**31), 2**31 - 1, (4 * nvec,), dtype=torch.int32, device="cuda", generator=g)
    ref = src.clone()
    dst = torch.zeros_like(src)
    fe.stream_copy(dst, src, nontemporal)
    fe.stream_copy(src, src, nontemporal)
    torch.cuda.synchronize()
    assert torch.equal(dst, ref)
    assert torch.equal(src, ref)


def test_partial_overlap_is_rejected():
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    with pytest.raises(fe.FeError):
        fe.stream_copy(buf[4:36], buf[0:32])
