"""pcba_read_list_noalloc, the entry point for callers that cannot allocate
device memory, through the C ABI: on two calls in a row (the second on a
shorter list, so the shared static staging array still holds the first call's
larger contents) it returns exactly what pcba_read_list returns, and a list
whose staging exceeds the static array is rejected with PCBA_E_ARG."""
import ctypes

import numpy as np
import pytest

from paper_2003_01758_amd.instances import make_instance, truncate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    from paper_2003_01758_amd import pcba
    pcba.lib()
    return pcba


def test_noalloc_read_equals_read_list_twice(gpu):
    big = gpu.Problem(truncate(make_instance(1, 0), 60))
    small = gpu.Problem(make_instance(0, 2))
    big.step(14)
    small.step(3)
    nb, ns = big.result()["list_len"], small.result()["list_len"]
    print(f"[no-alloc] list lengths {nb} then {ns}", flush=True)
    assert nb > 0 and ns > 0
    assert nb * big.words > ns * small.words   # the second call stages less
    for p in (big, small):
        ids_a, pat_a = p.list()
        ids_b, pat_b = p.list_noalloc()
        assert np.array_equal(ids_a, ids_b)
        # bit for bit (NaN marks a retired inequality in both)
        assert np.array_equal(pat_a, pat_b, equal_nan=True)


def test_noalloc_read_rejects_staging_beyond_the_static_array(gpu):
    # the 4-D workload: 63,295 words per item and lists of thousands of boxes;
    # past about 130 boxes the staging exceeds 64 MiB
    p = gpu.Problem(make_instance(2, 0).with_options(max_boxes=1 << 16))
    limit = gpu.STATIC_SCRATCH_BYTES // (8 * p.words)
    r = p.result()
    for _ in range(60):
        r = p.step(1)
        if r["list_len"] > limit or r["outcome"] != gpu.RUNNING:
            break
    n = r["list_len"]
    print(f"[no-alloc] 4-D list of {n} boxes, static limit {limit}", flush=True)
    assert n > limit
    ids = np.empty((n, p.l), dtype=np.uint32)
    pat = np.empty((1, p.words), dtype=np.float64)
    rc = gpu.lib().pcba_read_list_noalloc(p.h, ids.ctypes.data, pat.ctypes.data, n, None)
    assert rc == gpu.E_ARG and b"static scratch" in gpu.lib().pcba_last_error()
