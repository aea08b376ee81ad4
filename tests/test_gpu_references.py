"""The two HBM references the roofline is measured against move the bytes
they claim: the 16-byte copy (plain and non-temporal) copies exactly, and
the row pattern copies each of its rows and leaves the gaps between rows
untouched (sizes with a ragged last work-group)."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def glbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import lbm
    lbm.load_library()
    return lbm


@pytest.mark.parametrize("nontemporal", [False, True])
def test_copy_is_exact(glbm, nontemporal):
    n_words = (3 << 20) + 4 * 37          # 16-byte multiple, not a whole number of work-groups
    g = torch.Generator(device="cuda").manual_seed(5)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (n_words + 64,), dtype=torch.int32, device="cuda",
                        generator=g)
    dst = torch.full_like(src, 7)
    nbytes = n_words * 4
    glbm.lbm_stream_copy(src, dst, nbytes, nontemporal)
    torch.cuda.synchronize()
    assert torch.equal(dst[:n_words], src[:n_words])
    assert torch.all(dst[n_words:] == 7)


@pytest.mark.parametrize("rows", [1, 2, 4, 19])
def test_rows_copy_each_row_and_nothing_else(glbm, rows):
    row_bytes = 8 * ((1 << 16) + 13)       # a multiple of 8, ragged in work-groups
    stride = row_bytes + 4096
    words = rows * stride // 4
    g = torch.Generator(device="cuda").manual_seed(rows)
    src = torch.randint(-2 ** 31, 2 ** 31 - 1, (words,), dtype=torch.int32, device="cuda", generator=g)
    dst = torch.full_like(src, -3)
    glbm.lbm_stream_rows(src, dst, rows, stride, row_bytes)
    torch.cuda.synchronize()
    for r in range(rows):
        a, b = r * stride // 4, (r * stride + row_bytes) // 4
        assert torch.equal(dst[a:b], src[a:b]), r
        assert torch.all(dst[b:(r + 1) * stride // 4] == -3), r
