"""The reference stream of the rooflines writes every element of its write
stream (element i holds i, 1, 2, 3) and reads its read stream, for write- and
read-heavy mixes and sizes that leave partial rounds."""
import numpy as np
import pytest

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("read_elems,write_elems", [(1000, 2417), (5003, 1024), (777, 777), (1, 3 * 2 ** 20 + 5)])
def test_stream_probe_writes_its_whole_write_stream(read_elems, write_elems):
    import torch
    from paper_2501_13664_amd import api
    announce("stream probe: %d read, %d written (16-byte elements)" % (read_elems, write_elems))
    src = torch.randint(0, 1 << 30, (read_elems, 4), dtype=torch.int32, device="cuda")
    dst = torch.full((write_elems, 4), -1, dtype=torch.int32, device="cuda")
    api.stream_probe(src, 16 * read_elems, dst, 16 * write_elems)
    torch.cuda.synchronize()
    got = dst.cpu().numpy()
    want = np.stack([np.arange(write_elems), np.ones(write_elems), 2 * np.ones(write_elems),
                     3 * np.ones(write_elems)], axis=1).astype(np.int32)
    assert np.array_equal(got, want)
