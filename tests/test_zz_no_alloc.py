"""rt_wedges_noalloc (GPU, through the C ABI): the allocation-free variant of
rt_wedges gives its neighbour array bit for bit, on consecutive calls that
shrink (the 200k-facet dense city, the 24k city, the 242-facet microcell: the
shared device scratch keeps the previous call's contents), clears its
non-finite flag between calls, and refuses scenes above its scratch size
before any device work."""
import ctypes
import sys

import numpy as np
import pytest

import paper_2208_10008_amd as R
from rtgen import workloads

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    R.load()
    yield
    torch.cuda.synchronize()


def test_noalloc_wedges_equal_rt_wedges_on_shrinking_calls():
    for w in (workloads.dense200k(), workloads.city24k(), workloads.microcell()):
        tris = torch.from_numpy(np.ascontiguousarray(w.tris)).cuda()
        want = R.rt_wedges(tris).cpu().numpy()
        got = torch.full((tris.shape[0], 3), 7, dtype=torch.int32, device="cuda")
        R.rt_wedges_noalloc(tris, got)
        got = got.cpu().numpy()
        log(f"{w.name}: {tris.shape[0]} facets, {int((want >= 0).sum())} wedge half-edges")
        assert np.array_equal(got, want), w.name


def test_noalloc_wedges_flag_and_size_limit():
    w = workloads.microcell()
    bad = w.tris.copy()
    bad[3, 4] = np.inf
    nbr = torch.empty((bad.shape[0], 3), dtype=torch.int32, device="cuda")
    with pytest.raises(R.RtError) as e:
        R.rt_wedges_noalloc(torch.from_numpy(bad).cuda(), nbr)
    assert e.value.code == R.RT_EINVAL
    tris = torch.from_numpy(w.tris).cuda()       # the flag left set above is cleared
    R.rt_wedges_noalloc(tris, nbr)
    assert torch.equal(nbr, R.rt_wedges(tris))
    lib = R.load()
    assert lib.rt_wedges_noalloc(tris.data_ptr(), 262145, nbr.data_ptr(), None) == R.RT_EINVAL
    assert b"262144" in lib.rt_last_error()
