"""Index life cycle on the device: the rotation sampled by the library, and
save / load through a versioned file (every array back bit for bit, searches
identical)."""
import sys

import numpy as np
import pytest
import torch

from paper_2409_09913_amd import erq, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_index_samples_its_rotation():
    ix = erq.Index(256, 4, 8, None, seed=12345)
    P = ix.rotation().cpu().numpy()
    np.testing.assert_array_equal(P, erq.sample_rotation(256, 12345))
    ix.close()


@pytest.mark.parametrize("keep_raw", [True, False])
def test_save_load_roundtrip(tmp_path, keep_raw):
    n, d, nl = 30000, 192, 48
    x = torch.from_numpy(synth.gmm(n, d, 16, 0.3, seed=71, dp=d)).to(DEV)
    q = torch.from_numpy(synth.gmm(200, d, 16, 0.3, seed=71, stream=synth.S_QUERY, dp=d)).to(DEV)
    cent, assign = erq.kmeans(x, nl, iters=3)
    ix = erq.Index(d, 5, nl, None, seed=9)
    ix.build(x, cent, assign, keep_raw=keep_raw)
    ix.set_tune(1, 3, 4, 0)
    path = str(tmp_path / "index.erq")
    ix.save(path)
    iy = erq.Index.load_file(path)
    assert iy.info() == ix.info()
    assert iy.get_tune() == ix.get_tune()
    for a, b in zip(ix.export(), iy.export()):
        assert torch.equal(a.cpu().view(torch.uint8), b.cpu().view(torch.uint8))
    np.testing.assert_array_equal(iy.rotation().cpu().numpy(), ix.rotation().cpu().numpy())
    rr = 20 if keep_raw else 0
    a = ix.search(q, 12, 10, rr)
    b = iy.search(q, 12, 10, rr)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
    if not keep_raw:
        with pytest.raises(erq.ErqError):
            iy.search(q, 12, 10, 20)
    say("  save/load identical, keep_raw", keep_raw)
    ix.close()
    iy.close()
