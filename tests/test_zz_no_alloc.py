"""The allocation-free sample entry point against rp_sample (MI355X).

rp_sample_noalloc keeps Floyd's membership tables in a fixed device array
instead of the stream-ordered pool; its samples and substream advance must
equal rp_sample's bit for bit.  Two calls in a row, the second on a smaller
input, check that a call does not see the tables the previous call left in
the shared array.
"""
import numpy as np
import pytest

import paper_2605_05099_amd as rp
from tests.gpu_common import make_streams

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _pair(engine, m):
    return make_streams(engine, m), make_streams(engine, m)


def _same_call(A, B, m, n, k):
    a = torch.empty(m * k, dtype=torch.int32, device="cuda")
    b = torch.empty(m * k, dtype=torch.int32, device="cuda")
    rp.rp_sample(A, n, k, a)
    rp.rp_sample_noalloc(B, n, k, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b), (m, n, k)
    wa, pa = A.get()
    wb, pb = B.get()
    assert np.array_equal(wa, wb) and np.array_equal(pa, pb), (m, n, k)


@pytest.mark.parametrize("engine", ["philox4x32", "pcg64", "x256++"])
def test_noalloc_sample_matches_rp_sample(engine):
    # first call: 4096 substreams x 2048-entry tables = 32 MiB of the array
    A, B = _pair(engine, 4096)
    _same_call(A, B, 4096, 10**6, 1000)
    # second call, smaller: fewer substreams, smaller tables, other n
    C, D = _pair(engine, 67)
    _same_call(C, D, 67, 5000, 10)
    # the same sets continue (Floyd again, then the reservoir branch)
    _same_call(C, D, 67, 777, 300)
    _same_call(C, D, 67, 100, 80)


def test_noalloc_sample_size_limit():
    S = make_streams("philox4x32", 2**16)
    out = torch.empty(2**16 * 200, dtype=torch.int32, device="cuda")
    before = S.get()[0].copy()
    # 2^16 x 512 entries x 4 B = 128 MiB: above the fixed array
    with pytest.raises(rp.RpError) as ei:
        rp.rp_sample_noalloc(S, 10**6, 200, out)
    assert ei.value.code == rp.RP_EINVAL
    assert np.array_equal(S.get()[0], before)
    # 2^16 x 256 entries x 4 B = 64 MiB: exactly the array
    A = make_streams("philox4x32", 2**16)
    a = torch.empty(2**16 * 128, dtype=torch.int32, device="cuda")
    b = torch.empty(2**16 * 128, dtype=torch.int32, device="cuda")
    rp.rp_sample(A, 10**6, 128, a)
    rp.rp_sample_noalloc(S, 10**6, 128, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
