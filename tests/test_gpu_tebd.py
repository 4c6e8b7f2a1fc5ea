"""The TEBD compression shapes of Sec. III as one uneven batch: product
updates ((chi K) x (chi d), ratio 1/min(K, d)) and block updates ((chi d)^2,
ratio 1/d), chi = 100, K = 2, d = 5, FP64.  Every problem is checked against
properties that hold at any size; two of each shape against the oracle at
the FP64 parity bar."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


def test_tebd_product_and_block_updates_one_plan():
    import paper_1710_01463_amd as P
    probs = wl.tebd_product(12).problems + wl.tebd_block(6).problems
    mats = [pr.matrix() for pr in probs]
    As = [torch.from_numpy(A).cuda() for A in mats]
    plan = P.Plan([dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in probs],
                  torch.float64, "f64", graph=True)
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    w = w.cpu().numpy()
    kk = kk.cpu().numpy()
    for b, (A, (U, S, VT)) in enumerate(zip(As, outs)):
        k = probs[b].k
        assert kk[b] == k
        I = torch.eye(k, dtype=torch.float64, device="cuda")
        assert float((U.T @ U - I).abs().max()) < 1e-12
        assert float((VT @ VT.T - I).abs().max()) < 1e-12
        R = A - (U * S) @ VT
        a2 = float((A * A).sum())
        assert abs(float((R * R).sum()) - w[b]) <= 1e-12 * a2
    for b in (0, 7, 12, 17):
        pr = probs[b]
        ref = oracle.rsvd(mats[b], pr.k, pr.p, pr.q, pr.seed)
        S = outs[b][1].cpu().numpy()
        bar = np.where(ref.S >= 1e-5 * ref.S[0], 1e-10 * ref.S, 1e-15 * ref.S[0])
        assert np.all(np.abs(S - ref.S) <= bar), b
        assert np.max(np.abs(outs[b][0].cpu().numpy()[:, :20] - ref.U[:, :20])) < 1e-8
        assert abs(w[b] - ref.w) <= 1e-10 * ref.w + 1e-13 * np.sum(mats[b] ** 2)
    plan.close()
