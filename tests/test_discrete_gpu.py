"""GPU batched permutations and samples against the oracle (MI355X).

Integer work: every instance must equal the oracle's bit for bit on the same
substream, and the substream states must equal the oracle's afterwards (so
successive calls continue each substream).
"""
import numpy as np
import pytest

import paper_2605_05099_amd as rp
from paper_2605_05099_amd import workloads
from tests.gpu_common import ENGINES, make_streams, oracle_stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _states_equal(S, engine, ost):
    words, phase = S.get()
    nw = rp.STATE_WORDS[rp.ENGINES[engine]]
    for i, o in enumerate(ost):
        assert [int(words[k, i]) for k in range(nw)] == o.state[:nw], (engine, i)
        assert int(phase[i]) == o.phase, (engine, i)


@pytest.mark.parametrize("engine", ENGINES)
def test_permutations_and_samples_match_oracle(engine):
    m = 67 if engine != "ranlux++" else 37
    S = make_streams(engine, m)
    ost = [oracle_stream(engine, i) for i in range(m)]
    # permutations of several sizes, then samples by both methods; every
    # call continues the substreams
    for n in (1, 2, 37, 512, 1000, 1024, 1025):   # rows in LDS up to 1024 entries, in HBM above
        out = torch.empty(m * n, dtype=torch.int32, device="cuda")
        rp.rp_permutations(S, n, out)
        got = out.cpu().numpy().view(np.uint32).reshape(m, n)
        for i, o in enumerate(ost):
            assert np.array_equal(got[i], o.permutation(n)), (engine, n, i)
    for n, k in ((1000, 10), (1000, 500), (1000, 501), (1000, 999), (5, 5), (2**31 + 7, 100)):
        out = torch.empty(m * k, dtype=torch.int32, device="cuda")
        rp.rp_sample(S, n, k, out)
        got = out.cpu().numpy().view(np.uint32).reshape(m, k)
        for i, o in enumerate(ost):
            assert np.array_equal(got[i], o.sample(n, k)), (engine, n, k, i)
    _states_equal(S, engine, ost)


def test_discrete_at_substream_workload_size():
    """2^16 substreams (the substream workload's count): permutations of 256
    and Floyd samples of 64 from 10^6; sampled substreams checked in full."""
    m = workloads.SUB_N
    S = make_streams("philox4x32", m)
    idx = workloads.sampled_substreams(m, k=64)
    perm = torch.empty(m * 256, dtype=torch.int32, device="cuda")
    rp.rp_permutations(S, 256, perm)
    smp = torch.empty(m * 64, dtype=torch.int32, device="cuda")
    rp.rp_sample(S, 10**6, 64, smp)
    P = perm.view(m, 256)[torch.as_tensor(idx, device="cuda")].cpu().numpy().view(np.uint32)
    Q = smp.view(m, 64)[torch.as_tensor(idx, device="cuda")].cpu().numpy().view(np.uint32)
    for r, i in enumerate(idx):
        o = oracle_stream("philox4x32", int(i))
        assert np.array_equal(P[r], o.permutation(256))
        assert np.array_equal(Q[r], o.sample(10**6, 64))


def test_discrete_errors_and_empty():
    S = make_streams("pcg64", 4)
    before = S.get()[0].copy()
    out = torch.empty(16, dtype=torch.int32, device="cuda")
    rp.rp_permutations(S, 0, out)
    rp.rp_sample(S, 10, 0, out)
    assert (S.get()[0] == before).all()
    with pytest.raises(rp.RpError) as ei:
        rp.rp_sample(S, 3, 4, out)
    assert ei.value.code == rp.RP_EINVAL
    with pytest.raises(rp.RpError) as ei:
        rp.rp_permutations(S, 4, 0)
    assert ei.value.code == rp.RP_ENULL
