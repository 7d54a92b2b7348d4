"""GPU checks of the bandwidth probes through the C ABI: kr_hbm_copy copies
exactly (tail bytes included) and kr_hbm_stream writes, for every output
16-byte chunk, the XOR of the input chunks its header maps to it."""
from __future__ import annotations

import numpy as np
import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402


def expected_stream(src: np.ndarray, dst_bytes: int) -> np.ndarray:
    chunks = src.view(np.uint32).reshape(-1, 4)
    n_in, n_out = chunks.shape[0], dst_bytes // 16
    if n_in >= n_out:
        k = n_in // n_out
        out = np.bitwise_xor.reduce(chunks.reshape(n_out, k, 4), axis=1)
    else:
        out = chunks[np.arange(n_out) // (n_out // n_in)]
    return out.reshape(-1).view(np.uint8)


@pytest.mark.parametrize("src_bytes,dst_bytes", [(4096, 4096), (4096, 16384), (16384, 4096), (16, 16 << 12),
                                                 (16 << 8, 16), (1 << 20, 1 << 22), (48 << 10, 3 << 10)])
def test_stream_probe(src_bytes, dst_bytes):
    say(f"hbm_stream {src_bytes} -> {dst_bytes}")
    rng = np.random.default_rng(src_bytes ^ dst_bytes)
    host = rng.integers(0, 256, src_bytes, dtype=np.uint8)
    src = torch.from_numpy(host).cuda()
    dst = torch.zeros(dst_bytes, dtype=torch.uint8, device="cuda")
    kr.hbm_stream(dst, src)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), expected_stream(host, dst_bytes))


@pytest.mark.parametrize("nbytes", [16, 17, 4096 + 5, (1 << 20) + 15])
def test_copy_probe(nbytes):
    say(f"hbm_copy {nbytes}")
    host = np.random.default_rng(nbytes).integers(0, 256, nbytes, dtype=np.uint8)
    src = torch.from_numpy(host).cuda()
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    kr.hbm_copy(dst, src)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), host)
