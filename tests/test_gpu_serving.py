"""The continuous-batching server on the GPU: every query result equals the
same query run alone against the snapshot it was admitted at, inserts land
as bolt_encode of their payload, and the FIFO baseline agrees."""
import numpy as np
import pytest
import torch

import synth
import synth.device as sdev

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.fixture(scope="module")
def env():
    import paper_1706_10283_amd.bolt as B
    from paper_1706_10283_amd import workloads as W
    J, M = 64, 16
    C, quant = W.train(7000, 7003, 7004, 7005, J, M, n_train=5000, iters=4, n_lut_train=300)
    dbs = [W.build_db(7000, 7010 + i, 40_000 + 7_777 * i, J, M, C, quant, capacity=120_000) for i in range(3)]
    qpool = sdev.gmm_rows(7000, 7020, 0, 512, J).cpu().numpy()
    ipool = sdev.gmm_rows(7000, 7021, 0, 20_000, J).cpu().pin_memory()
    return B, W, dbs, qpool, ipool


@pytest.mark.parametrize("mode,rate", [("continuous", 0.0), ("continuous", 3000.0), ("fifo", 0.0)])
def test_serving_results_equal_alone(env, mode, rate):
    B, W, dbs, qpool, ipool = env
    from paper_1706_10283_amd.serve import GpuExecutor, Server, make_requests, summarize
    print("[case] serving", mode, rate, flush=True)
    before = [db.n_rows for db in dbs]
    reqs = make_requests(60, len(dbs), 64, rate, seed=11, query_pool=qpool, insert_pool=ipool,
                         frac_insert=0.15, batch_hi=32, ins_lo=1e3, ins_hi=2e4, k=50)
    srv = Server(GpuExecutor(dbs), dbs, budget_bytes=2 << 30, mode=mode)
    # each run starts from the same committed rows (earlier parametrizations appended inserts)
    srv.committed = list(before)
    srv.reserved = list(before)
    wall = srv.run(reqs, realtime=rate > 0)
    torch.cuda.synchronize()
    print(summarize(reqs, wall), flush=True)
    assert all(r.status == "done" for r in reqs), [(r.rid, r.status, r.error) for r in reqs if r.status != "done"]
    for r in reqs:
        db = dbs[r.db]
        if r.kind == "query":
            qd = torch.from_numpy(np.ascontiguousarray(r.Qv)).to(DEV)
            v, i = B.bolt_scan_topk(db.codes[:r.watermark], db.luts(qd, r.metric), r.metric, r.k)
            assert np.array_equal(v.cpu().numpy(), r.vals)
            assert np.array_equal(i.cpu().numpy(), r.idx)
        else:
            a, b = r.rows
            xd = r.X.to(DEV) if isinstance(r.X, torch.Tensor) else torch.from_numpy(r.X).to(DEV)
            ref = B.bolt_encode(xd, db.centroids, db.M)
            assert torch.equal(ref, db.codes[a:b])
