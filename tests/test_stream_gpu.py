"""The streaming-read reference kernel reads every byte (GPU).

The bench compares the scan kernel's bandwidth with the read bandwidth this
kernel reaches; it is only a fair ceiling if it really reads the whole
buffer, so the xor it folds must equal the xor of all the buffer's words.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _xor_words(b: np.ndarray) -> int:
    nvec = b.size // 16
    words = b[: nvec * 16].view(np.uint32)
    x = int(np.bitwise_xor.reduce(words)) if words.size else 0
    for i, v in enumerate(b[nvec * 16:]):
        x ^= int(v) << (8 * (i & 3))
    return x


@pytest.mark.parametrize("n", [0, 15, 16, 1000, 4096 + 7, (1 << 22) + 13, 1 << 26])
def test_stream_read_folds_every_byte(n):
    import torch
    import paper_1405_5483_amd as mag
    assert torch.cuda.is_available()
    rng = np.random.default_rng(n)
    b = rng.integers(0, 256, n, dtype=np.uint8)
    d = torch.from_numpy(b).cuda() if n else torch.empty(0, dtype=torch.uint8, device="cuda")
    sink = mag.stream_read(d)
    torch.cuda.synchronize()
    got = int(np.bitwise_xor.reduce(sink.cpu().numpy().view(np.uint32)))
    assert got == _xor_words(b)


def test_stream_read_rejects_unaligned():
    import torch
    import paper_1405_5483_amd as mag
    d = torch.zeros(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(mag.MagError):
        mag.stream_read(d[1:])
