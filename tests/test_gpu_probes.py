"""GPU checks of the library's measurement utilities (not part of the method): the
read-only stream's partial XORs combine to the XOR of every 16-byte word (compared bit
for bit with the XOR computed on the host; every slot is written), and the copy kernel
copies exactly.  Sizes: one word, a
ragged count of words that is not a multiple of the launch width, and 64 MiB."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1902_08653_amd import cdm
    cdm.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("words", [1, 4 * 256 * 257 + 3, (64 << 20) // 16])
def test_stream_read_xor_and_copy(dev, words):
    from paper_1902_08653_amd import cdm
    rng = np.random.default_rng(words)
    host = rng.integers(0, 2**32, size=(words, 4), dtype=np.uint64).astype(np.uint32)
    src = torch.from_numpy(host.view(np.int32)).to(dev)
    acc = torch.full((cdm.STREAM_READ_SLOTS, 4), -1, dtype=torch.int32, device=dev)   # every slot written
    cdm.stream_read(src, acc)
    dst = torch.empty_like(src)
    cdm.stream_copy(src, dst)
    torch.cuda.synchronize()
    want = np.bitwise_xor.reduce(host, axis=0)
    got = np.bitwise_xor.reduce(acc.cpu().numpy().view(np.uint32), axis=0)
    assert np.array_equal(got, want)
    assert torch.equal(dst, src)
