"""Codebook learning on the GPU (bolt_kmeans) against the oracle's k-means,
through the C ABI.  The assignment uses the oracle's fp64 operations in its
order, so on integer-valued data (the Gaussian-mixture workloads: every fp64
sum is exact) the centroids must be identical bit for bit; on N(0, 1) data
the parallel fp64 sums may round differently, within the last bit of the
fp32 mean.  The paper prints no trained codebooks; the oracle's k-means is
pinned to scikit-learn's Lloyd iterations (test_oracle_pins.py), and these
tests bind the GPU to it and to the invariants (non-increasing
objective)."""
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


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.mark.parametrize("J,M,iters", [(128, 32, 10), (128, 16, 6), (64, 64, 4), (32, 8, 10)])
def test_kmeans_mixture_bit_exact(bolt, J, M, iters):
    n = 20_000
    _say("kmeans mixture", "n", n, "J", J, "M", M, "iters", iters)
    X = synth.gmm_rows(synth.seed_for(4, 0), synth.seed_for(4, 3) + J, 0, n, J)
    init = synth.permutation_prefix(synth.seed_for(4, 4) + M, n, 16)
    C_ref, obj_ref = oracle.kmeans(X, M, iters, init)
    C, obj = bolt.bolt_kmeans(torch.from_numpy(X).to(DEV), M, iters, init)
    assert np.array_equal(C.cpu().numpy().view(np.uint32), C_ref.view(np.uint32))
    np.testing.assert_allclose(obj, obj_ref, rtol=1e-12)
    assert (np.diff(obj) <= 1e-9 * obj[0]).all()


def test_kmeans_empty_clusters_keep_centroid(bolt):
    """Seeds on duplicated rows: the later copy loses every tie, so its cluster
    starts empty and keeps its centroid; both sides must agree bit for bit."""
    n, J, M = 5000, 32, 8
    X = synth.gmm_rows(synth.seed_for(4, 0), 99, 0, n, J)
    init = synth.permutation_prefix(123, n, 16)
    init[9] = init[3]
    init[15] = init[0]
    C_ref, obj_ref = oracle.kmeans(X, M, 5, init)
    C, obj = bolt.bolt_kmeans(torch.from_numpy(X).to(DEV), M, 5, init)
    assert np.array_equal(C.cpu().numpy().view(np.uint32), C_ref.view(np.uint32))
    np.testing.assert_allclose(obj, obj_ref, rtol=1e-12)


def test_kmeans_normal_data_within_last_bit(bolt):
    n, J, M, iters = 6000, 32, 8, 3
    _say("kmeans normal", "n", n, "J", J, "M", M, "iters", iters)
    X = synth.normal(311, (n, J))
    init = synth.permutation_prefix(312, n, 16)
    C_ref, obj_ref = oracle.kmeans(X, M, iters, init)
    C, obj = bolt.bolt_kmeans(torch.from_numpy(X).to(DEV), M, iters, init)
    np.testing.assert_array_max_ulp(C.cpu().numpy(), C_ref, maxulp=2)
    np.testing.assert_allclose(obj, obj_ref, rtol=1e-9)


def test_kmeans_errors(bolt):
    X = torch.zeros((10, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(bolt.BoltError):
        bolt.bolt_kmeans(X, 4, 2, np.arange(16))          # fewer than 16 rows
    X = torch.zeros((100, 8), dtype=torch.float32, device=DEV)
    with pytest.raises(bolt.BoltError):
        bolt.bolt_kmeans(X, 4, 2, np.arange(16) + 90)     # seed row out of range
    with pytest.raises(bolt.BoltError):
        bolt.bolt_kmeans(X, 3, 2, np.arange(16))          # odd M


@pytest.mark.parametrize("metric", ["l2", "dot", "l1", "cosine", "lp3"])
@pytest.mark.parametrize("nq,n,J,M", [(200, 3000, 64, 16), (1000, 20_000, 128, 32), (7, 60, 16, 4),
                                      (1024, 5000, 32, 8)])
def test_quantizer_search_matches_oracle(bolt, metric, nq, n, J, M):
    """The alpha grid search on the GPU (Sec. 3.2) against the oracle's: the
    same chosen alpha, a and offsets bit for bit (the fp64 operations that
    decide them are the definition's in its order), losses within the
    rounding of their parallel sums.  L_p tables use repeated products on
    the GPU and pow in the oracle: a and offsets within a few fp32 ulp."""
    _say("quantizer search", metric, "nq", nq, "n", n, "J", J, "M", M)
    seed = nq + n + J + M
    X = synth.gmm_rows(synth.seed_for(4, 0), seed, 0, n, J)
    if metric == "cosine":
        X = oracle.normalize_rows(X)
    C, _ = oracle.kmeans(X, M, 3, synth.permutation_prefix(seed + 1, n, 16))
    codes = oracle.encode(X, C, M)
    Qt = synth.gmm_rows(synth.seed_for(4, 0), seed + 2, 0, nq, J)
    a_ref, off_ref, best_ref, loss_ref = oracle.learn_quantizer(Qt, codes, C, metric)
    a, offs, best, losses = bolt.bolt_learn_quantizer(torch.from_numpy(Qt).to(DEV), torch.from_numpy(codes).to(DEV),
                                                      torch.from_numpy(C).to(DEV), metric)
    offs = offs.cpu().numpy()
    assert best == best_ref
    np.testing.assert_allclose(losses, loss_ref, rtol=1e-10)
    if metric == "lp3":
        np.testing.assert_array_max_ulp(np.float32(a), np.float32(a_ref), maxulp=4)
        np.testing.assert_allclose(offs, off_ref, rtol=1e-6, atol=1e-3)
    else:
        assert np.float32(a).view(np.uint32) == np.float32(a_ref).view(np.uint32)
        assert np.array_equal(offs.view(np.uint32), off_ref.view(np.uint32))


def test_quantizer_search_ties_and_limits(bolt):
    """Constant tables (every alpha gives the same loss: the smallest alpha
    wins) and the size limit of 1024 training queries."""
    J, M, n = 16, 4, 100
    C = np.ones((M, 16, J // M), dtype=np.float32)
    codes = np.zeros((n, M // 2), dtype=np.uint8)
    Qt = np.ones((30, J), dtype=np.float32)
    a_ref, off_ref, best_ref, _ = oracle.learn_quantizer(Qt, codes, C, "l2")
    a, offs, best, _ = bolt.bolt_learn_quantizer(torch.from_numpy(Qt).to(DEV), torch.from_numpy(codes).to(DEV),
                                                 torch.from_numpy(C).to(DEV), "l2")
    assert best == best_ref == 0
    assert np.float32(a) == np.float32(a_ref) and np.array_equal(offs.cpu().numpy(), off_ref)
    with pytest.raises(bolt.BoltError):
        bolt.bolt_learn_quantizer(torch.zeros((1025, J), device=DEV), torch.from_numpy(codes).to(DEV),
                                  torch.from_numpy(C).to(DEV), "l2")
