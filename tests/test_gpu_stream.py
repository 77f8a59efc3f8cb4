"""The bandwidth calibration kernels: the read's sum and the copy's bytes.

hz_stream_read sums a buffer's doubles in a fixed order (chunks of 2048
elements by block, then a block tree, then the blocks in index order), so it
must agree with a plain host sum to rounding and be bitwise repeatable;
hz_stream_copy must reproduce the buffer exactly, ragged tails included.
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hz():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2112_06465_amd as hz

    return hz


@pytest.mark.parametrize("n", [2, 2048, 2050, 4096 * 2048 + 6, 1 << 22])
def test_stream_read_sums_and_copy_reproduces(hz, n):
    rng = np.random.default_rng(n)
    h = rng.standard_normal(n)
    x = torch.from_numpy(h).to("cuda:0")
    s1 = hz.stream_read(x).item()
    s2 = hz.stream_read(x).item()
    assert s1 == s2
    assert abs(s1 - h.sum()) <= 1e-13 * np.abs(h).sum()
    y = torch.empty_like(x)
    hz.stream_copy(x, y)
    assert torch.equal(x, y)


def test_stream_rejects_bad_sizes(hz):
    x = torch.zeros(3, dtype=torch.float64, device="cuda:0")  # 24 bytes: not a multiple of 16
    with pytest.raises(ValueError):
        hz.stream_read(x)
    a = torch.zeros(4, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ValueError):
        hz.stream_copy(a, torch.zeros(2, dtype=torch.float64, device="cuda:0"))
