"""The flush that keeps LDS uint32 sub-histograms from wrapping: a workgroup
must flush before the pairs it has counted since its last flush could reach
2^32 (the paper flushes its private uint32 histograms before they approach
their limit, Sec. 3.1).

2^21 points of one species, no box, in two tight clusters: every pair within
a cluster lands in bin 0 and every pair across them in bin 2, both fixed by
geometry (cluster width 1e-3, centres 2.5 apart, r_max = 4, 4 bins). With
one workgroup per CU each workgroup counts about 8.6e9 pairs of that one
histogram, so it must flush at least once on the uint32 bound; a wrapped
slot would lose a multiple of 2^32 from bin 0 or bin 2. The expected counts
come from the geometry, not from the kernel's own pair bookkeeping."""
import numpy as np
import pytest

import workloads
from gpu_util import run_gpu

pytestmark = pytest.mark.gpu

N = 1 << 21


def two_clusters():
    rng = np.random.Generator(np.random.PCG64(2121))
    na = N // 2 + 12345
    x = rng.uniform(0.0, 1e-3, size=(N, 3))
    x[na:, 0] += 2.5
    fr = workloads.Frame(np.ascontiguousarray(x), np.array([0, N], np.int64), workloads.BOX_NONE,
                         None, 4.0, 4, "two-clusters-2M")
    return fr, na, N - na


@pytest.fixture(scope="module")
def ctx():
    import paper_1808_01478_amd as dh
    c = dh.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_uint32_flush_bound(ctx, precision):
    fr, na, nb = two_clusters()
    # one 1024-thread workgroup per CU, four interleaved copies
    ctx.set_config(dict(r=4, copies=4, tj=256, noclamp=1, occ_cap=1, items_per_wg=8,
                        threads=1024, wide=60))
    try:
        print(f"\n[case] two clusters N={N} prec={precision} occ_cap=1", flush=True)
        h, oor = run_gpu(ctx, fr, precision)
        cfg = ctx.last_config()
    finally:
        ctx.set_config(None)
    pairs = N * (N - 1) // 2
    assert pairs / cfg["grid"] > 2**32, "each workgroup must count more than 2^32 pairs"
    want = np.zeros(4, np.uint64)
    want[0] = na * (na - 1) // 2 + nb * (nb - 1) // 2
    want[2] = na * nb
    assert np.array_equal(h[0], want), (h[0], want)
    assert int(oor[0]) == 0
