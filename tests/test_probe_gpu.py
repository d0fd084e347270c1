"""The gather micro-benchmark reads exactly the rows it is given: its XOR of every 32-bit
word read equals the same XOR formed on the CPU (duplicates cancel in pairs on both sides;
indices outside the table are skipped)."""
import numpy as np
import pytest
import torch

from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu


def _expected(words, idx):
    rows = words.shape[0]
    ok = idx[(idx >= 0) & (idx < rows)]
    x = np.bitwise_xor.reduce(words[ok], axis=None) if ok.size else np.uint32(0)
    return int(np.uint32(x))


@pytest.mark.parametrize("row_bytes", [16, 48, 128, 256, 1024, 2048, 4096])
@pytest.mark.parametrize("n", [0, 1, 63, 1000, 70001])
def test_gather_probe_xor(row_bytes, n):
    G.note("gather probe row_bytes=%d n=%d" % (row_bytes, n))
    rng = np.random.Generator(np.random.PCG64(row_bytes * 7 + n))
    rows = 777
    words = rng.integers(0, 1 << 32, size=(rows, row_bytes // 4), dtype=np.uint64).astype(np.uint32)
    idx = rng.integers(-3, rows + 3, size=n).astype(np.int32)
    table = torch.from_numpy(words.view(np.int32)).to(G.DEV)
    out = ops.spmm_gather_probe(table, row_bytes, torch.from_numpy(idx).to(G.DEV))
    torch.cuda.synchronize()
    got = int(np.uint32(out.cpu().numpy().view(np.uint32)[0]))
    assert got == _expected(words, idx)
