"""GPU test of the memory-system probe rr_probe_row_gather: the rows it
reads follow the sequence its declaration defines (splitmix64 finaliser,
multiply-high reduction), checked through the per-workgroup word sums
against the same sums computed here from the host copy of the rows."""
import numpy as np
import pytest

from paper_2502_13245_amd import synth
from tests.gpu_common import flush_print

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

M64 = (1 << 64) - 1


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _expected(rows_padded, gathers, seed):
    n = rows_padded.shape[0]
    words = rows_padded.view(np.uint32).astype(np.uint64).sum(axis=1) % (1 << 32)
    idx = np.array([(_mix((seed + i + 0x9E3779B97F4A7C15) & M64) * n) >> 64 for i in range(gathers)],
                   dtype=np.int64)
    per = words[idx]
    parts = (gathers + 1023) // 1024
    return np.array([int(per[w * 1024:(w + 1) * 1024].sum()) % (1 << 32) for w in range(parts)],
                    dtype=np.int64)


@pytest.fixture(scope="module")
def rr():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_13245_amd import rr as _rr
    _rr.lib()
    return _rr


@pytest.mark.parametrize("d,gathers,seed", [(128, 5000, 7), (100, 3073, 2 ** 63 + 5), (7, 1024, 0), (128, 0, 1)])
def test_probe_reads_the_defined_rows(rr, d, gathers, seed):
    flush_print(f"probe d={d} gathers={gathers}")
    n = 1531
    w = synth.gaussian_mixture_int(n, 4, d, 5, 12.0, 11)
    ix = rr.Index.from_graph(w.base, synth.random_graph(n, 8, 3), 0).to_device("cuda:0")
    sink = rr.probe_row_gather(ix, gathers, seed)
    torch.cuda.synchronize()
    row_bytes = (d + 15) // 16 * 16
    padded = np.zeros((n, row_bytes), dtype=np.uint8)
    padded[:, :d] = w.base
    np.testing.assert_array_equal(sink.cpu().numpy(), _expected(padded, gathers, seed))


def test_probe_needs_a_device_index(rr):
    w = synth.gaussian_mixture_int(100, 4, 16, 5, 12.0, 11)
    ix = rr.Index.from_graph(w.base, synth.random_graph(100, 8, 3), 0)
    with pytest.raises(rr.RRError):
        rr.probe_row_gather(ix, 10)
