"""rbq_search_noalloc (the allocation-free search) against rbq_search through
the C ABI: identical ids and distances on two calls in a row, the second with
a smaller input, for both scan kernels; requests beyond the scratch size and
host pointers are rejected."""
import ctypes as C
import sys

import numpy as np
import pytest

from gpu_common import Built, make_case

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[{msg}]", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def built():
    return Built(make_case("ivf128"))


@pytest.mark.parametrize("kernel", ["popcnt", "mfma"])
def test_noalloc_equals_search_on_two_calls(built, kernel):
    import torch
    from paper_2405_12497_amd import rabitq as R
    kern = R.RBQ_SCAN_POPCNT if kernel == "popcnt" else R.RBQ_SCAN_MFMA
    b = built
    _say(f"no-alloc search, {kernel}")
    for q, k, nprobe in ((b.q, 10, 8), (b.q[3:8].contiguous(), 5, 4)):
        want_i, want_d, _ = b.idx.search(q, k, nprobe, scan_kernel=kern)
        got_i, got_d = R.rbq_search_noalloc(b.idx.h, q, k, nprobe, scan_kernel=kern)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got_i.cpu().numpy(), want_i.cpu().numpy())
        np.testing.assert_array_equal(got_d.cpu().numpy(), want_d.cpu().numpy())


def test_noalloc_rejects_oversized_and_host_requests(built):
    import torch
    from paper_2405_12497_amd import rabitq as R
    b = built
    _say("no-alloc rejections")
    big = b.q.repeat(100, 1).contiguous()           # 2400 queries x 64 lists: segments beyond 128 MiB
    with pytest.raises(R.RbqError) as e:
        R.rbq_search_noalloc(b.idx.h, big, 10, 64)
    assert e.value.status == R.RBQ_EINVAL
    assert "scratch" in R.rbq_last_error()
    # the index and the array still work afterwards
    want_i, _, _ = b.idx.search(b.q, 10, 8)
    got_i, _ = R.rbq_search_noalloc(b.idx.h, b.q, 10, 8)
    np.testing.assert_array_equal(got_i.cpu().numpy(), want_i.cpu().numpy())
    host_q = np.ascontiguousarray(b.case.queries)
    o = R.RbqSearchOpts(10, 8, 0, 0, None, 0, 0, 0)
    out_i = torch.empty((len(host_q), 10), dtype=torch.int64, device="cuda")
    out_d = torch.empty((len(host_q), 10), dtype=torch.float32, device="cuda")
    st = R.lib().rbq_search_noalloc(b.idx.h, host_q.ctypes.data_as(C.c_void_p), len(host_q), C.byref(o),
                                    C.c_void_p(out_i.data_ptr()), C.c_void_p(out_d.data_ptr()), None)
    assert st == R.RBQ_EINVAL
