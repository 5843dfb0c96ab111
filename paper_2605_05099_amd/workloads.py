"""Seeded synthetic workloads (inputs only; no sampling arithmetic of the method).

Both the GPU path and the test oracle take their inputs from here.  Parameters
are drawn with numpy.random.default_rng(<config index>), kept apart from the
seeds of the generators under test (12345 and 42).

  serial_stream   x256++ seeded with 12345, one stream, 10^6 values per output
  substreams      Philox4x32-10 (key = substream index) and PCG64 (increment
                  2 i + 1), base seed 42, 2^16 substreams x 2^14 values
  batched_sets    10^6 gamma sets: shape log-uniform on [0.01, 100], counts
                  geometric with mean 256 capped at 4096; beta sets with a, b
                  log-uniform on [0.1, 10] and their own counts
  per_element     [4096, 1024] binary32 shapes log-uniform on [0.05, 50] (gamma)
                  and (a, b) of the same shape and range (beta); upstream
                  gradients ~ N(0, 1)
  mvn             d in {64, 256, 512}, Sigma = Q diag(logspace(-2, 2, d)) Q^T with
                  Q from the QR factorization of a Gaussian matrix, mu ~ N(0, 1),
                  2^20 rows
  fused_moments   ranlux++ (substream i = base jumped by i 2^64 steps) and sfc64
                  (seed 42, spawn key [i]) with 2^18 substreams x 2^16 normals
"""
import numpy as np

SERIAL_SEED = 12345
BASE_SEED = 42
SERIAL_N = 10**6
SUB_N = 2**16
SUB_PER = 2**14
MVN_N = 2**20
MVN_DIMS = (64, 256, 512)
MOM_N = 2**18
MOM_PER = 2**16
PER_ELEMENT_SHAPE = (4096, 1024)


def sampled_substreams(n=SUB_N, k=256, seed=2):
    """k random substream indices plus the first and last."""
    rng = np.random.default_rng(seed)
    idx = set(int(i) for i in rng.choice(n, size=min(k, n), replace=False))
    idx.update({0, n - 1})
    return np.array(sorted(idx), dtype=np.int64)


def batched_sets(n_sets=10**6, seed=3, cap=4096, mean=256):
    rng = np.random.default_rng(seed)
    alpha = np.exp(rng.uniform(np.log(0.01), np.log(100.0), n_sets))
    count = np.minimum(rng.geometric(1.0 / mean, n_sets), cap).astype(np.int64)
    a = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n_sets))
    b = np.exp(rng.uniform(np.log(0.1), np.log(10.0), n_sets))
    count_beta = np.minimum(rng.geometric(1.0 / mean, n_sets), cap).astype(np.int64)
    return dict(alpha=alpha, count=count, a=a, b=b, count_beta=count_beta)


def per_element(shape=(4096, 1024), seed=4):
    rng = np.random.default_rng(seed)
    lo, hi = np.log(0.05), np.log(50.0)
    alpha = np.exp(rng.uniform(lo, hi, shape)).astype(np.float32)
    a = np.exp(rng.uniform(lo, hi, shape)).astype(np.float32)
    b = np.exp(rng.uniform(lo, hi, shape)).astype(np.float32)
    gz = rng.standard_normal(shape).astype(np.float32)
    gza = rng.standard_normal(shape).astype(np.float32)
    return dict(alpha=alpha, a=a, b=b, gz=gz, gz_beta=gza)


def mvn(d, seed=5):
    rng = np.random.default_rng(seed * 1000 + d)
    q, r = np.linalg.qr(rng.standard_normal((d, d)))
    q = q * np.sign(np.diag(r))
    sigma = q @ np.diag(np.logspace(-2, 2, d)) @ q.T
    sigma = (sigma + sigma.T) / 2
    mu = rng.standard_normal(d)
    return dict(sigma=sigma, mu=mu)
