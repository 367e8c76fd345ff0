"""Row orders chosen to defeat the sampled starting bounds, as databases grown
by online inserts can be (Sec. 1.2: vectors arrive in their own order, not a
random one).  Whatever the order, the fused and the batched scan + top-k must
equal the oracle: a query whose bound fails, or whose keys overflow a
barrier-free tile's segments, is recomputed exactly on the whole GPU.

Orders (of the rows of a random code matrix, by the d of query 0):
  sorted   nearest rows first, so that one tile holds all of query 0's
           candidates (segment overflow in the barrier-free matrix-core tiles);
  sampled  the nearest rows placed one per 32-row block inside the chunks the
           sample reads (chunks of 1024 rows at a stride of N / nsc, nsc =
           N / 32768 clamped to [16, 256]), so that the sample's r-th smallest
           group minimum admits fewer than k rows and the bound fails.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def bolt():
    import paper_1706_10283_amd.bolt as b
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return b


def _d0(codes, luts, M, metric):
    s = oracle.scan(codes, luts[:1])[0].astype(np.int64)
    return 255 * M - s if metric == "dot" else s


def _ordered(codes, luts, M, metric, order):
    N = codes.shape[0]
    near = np.lexsort((np.arange(N), _d0(codes, luts, M, metric)))
    if order == "sorted":
        return np.ascontiguousarray(codes[near])
    nsc = min(max(N // 32 // 1024, 16), 256)
    stride = N // nsc
    slots = np.array([c * stride + 32 * j for c in range(nsc) for j in range(32)], dtype=np.int64)
    perm = np.full(N, -1, dtype=np.int64)
    perm[slots] = near[:slots.size]
    rest = np.setdiff1d(np.arange(N), near[:slots.size], assume_unique=True)
    perm[perm < 0] = rest
    return np.ascontiguousarray(codes[perm])


# (M, Q, N, k, metric, order): whole databases of 2^16 rows or more (sampled
# bounds by default) on the one-query, few-query and matrix-core kernels
CASES = [
    (32, 40, 600_000, 100, "l2", "sorted"), (16, 33, 530_000, 128, "dot", "sorted"),
    (32, 12, 600_000, 100, "dot", "sorted"), (32, 1, 600_000, 100, "l2", "sorted"),
    (32, 40, 600_000, 100, "l2", "sampled"), (64, 9, 540_000, 100, "dot", "sampled"),
    (16, 1, 600_000, 100, "l2", "sampled"), (32, 3, 560_000, 64, "dot", "sampled"),
]


@pytest.mark.parametrize("M,Q,N,k,metric,order", CASES)
def test_adversarial_order_fused(bolt, M, Q, N, k, metric, order):
    seed = 23 * M + 5 * Q + N + k
    print("[case] adversarial fused", order, metric, "seed", seed, "M", M, "Q", Q, "N", N, "k", k, flush=True)
    codes = synth.random_codes(seed, N, M)
    luts = synth.random_luts(seed + 1, Q, M)
    codes = _ordered(codes, luts, M, metric, order)
    vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
    v, i = bolt.bolt_scan_topk(torch.from_numpy(codes).to(DEV), torch.from_numpy(luts).to(DEV), metric, k)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), vr)
    assert np.array_equal(i.cpu().numpy(), ir)


def test_adversarial_order_batched(bolt):
    """The same orders inside one batched launch, beside a randomly ordered
    database: every database equals the oracle."""
    specs = [(32, 40, 600_000, 100, "l2", "sorted"), (32, 20, 560_000, 100, "dot", "sampled"),
             (16, 48, 530_000, 64, "l2", "random")]
    host, dev = [], []
    for j, (M, Q, N, k, metric, order) in enumerate(specs):
        seed = 4100 + 17 * j
        print("[case] adversarial batched db", j, order, metric, "M", M, "Q", Q, "N", N, "k", k, flush=True)
        codes = synth.random_codes(seed, N, M)
        luts = synth.random_luts(seed + 1, Q, M)
        if order != "random":
            codes = _ordered(codes, luts, M, metric, order)
        host.append((codes, luts, k, metric))
        dev.append({"codes": torch.from_numpy(codes).to(DEV), "luts": torch.from_numpy(luts).to(DEV),
                    "k": k, "metric": metric})
    plan = bolt.BatchPlan(dev)
    plan.run()
    torch.cuda.synchronize()
    res = [(v.cpu().numpy(), i.cpu().numpy()) for v, i in plan.results()]
    plan.close()
    for (codes, luts, k, metric), (v, i) in zip(host, res):
        vr, ir = oracle.topk(oracle.scan(codes, luts), k, metric == "dot")
        assert np.array_equal(v, vr)
        assert np.array_equal(i, ir)
