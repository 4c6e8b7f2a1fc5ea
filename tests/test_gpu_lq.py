"""Small SVD on the triangular factor of B (plans without a saved forward,
n >= 4 l): B^T = Q_B R by Cholesky QR twice, Jacobi on R^T, V^T = W Q_B^T.
Mixed batches (problems with and without it) against the FP64 oracle, FP32
storage, a non-finite input, and post-selection on such a plan."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu

SHAPES = [  # m, n, k, p, q, alpha   (n / l: 18, 4.3, 2.7 (plain path), 4.5)
    (300, 900, 40, 10, 2, 0.05),
    (256, 256, 44, 16, 1, 0.03),
    (200, 300, 100, 10, 2, 0.04),
    (500, 180, 30, 10, 2, 0.1),
]


def problems(dtype):
    out = []
    for i, (m, n, k, p, q, alpha) in enumerate(SHAPES):
        A = wl.make_matrix(m, n, np.exp(-alpha * np.arange(1, min(m, n) + 1)), 60 + i).astype(dtype)
        out.append((A, dict(m=m, n=n, k=k, p=p, q=q, seed=90 + i)))
    return out


def run(P, probs, tdt, prec):
    plan = P.Plan([pr for _, pr in probs], tdt, prec, graph=True)
    As = [torch.from_numpy(A).cuda() for A, _ in probs]
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    return plan, As, outs, w.cpu().numpy(), kk.cpu().numpy(), info.cpu().numpy()


def test_lq_mixed_batch_f64_matches_oracle():
    import paper_1710_01463_amd as P
    probs = problems(np.float64)
    plan, As, outs, w, kk, info = run(P, probs, torch.float64, "f64")
    assert np.all(info == 0)
    for b, ((A, pr), (U, S, VT)) in enumerate(zip(probs, outs)):
        ref = oracle.rsvd(A, pr["k"], pr["p"], pr["q"], pr["seed"])
        s = S.cpu().numpy()
        bar = np.where(ref.S >= 1e-5 * ref.S[0], 1e-10 * ref.S, 1e-15 * ref.S[0])
        assert np.all(np.abs(s - ref.S) <= bar), b
        assert np.max(np.abs(U.cpu().numpy()[:, :10] - ref.U[:, :10])) < 1e-8, b
        assert np.max(np.abs(VT.cpu().numpy()[:10] - ref.VT[:10])) < 1e-8, b
        assert abs(w[b] - ref.w) <= 1e-10 * ref.w + 1e-13 * np.sum(A * A), b
        k = pr["k"]
        I = torch.eye(k, dtype=torch.float64, device="cuda")
        assert float((VT @ VT.T - I).abs().max()) < 1e-12
    plan.close()


def test_lq_f32_storage():
    import paper_1710_01463_amd as P
    probs = problems(np.float32)
    plan, As, outs, w, kk, info = run(P, probs, torch.float32, "f32")
    assert np.all(info == 0)
    for b, ((A, pr), (U, S, VT)) in enumerate(zip(probs, outs)):
        ref = oracle.rsvd(A.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["seed"])
        err = np.max(np.abs(S.double().cpu().numpy() - ref.S)) / ref.S[0]
        assert err <= 1e-6, (b, err)
        k = pr["k"]
        I = torch.eye(k, dtype=torch.float64, device="cuda")
        assert float((VT.double() @ VT.double().T - I).abs().max()) < 1e-5
    plan.close()


def test_lq_nonfinite_input_gives_zero_outputs():
    import paper_1710_01463_amd as P
    probs = problems(np.float64)
    probs[0][0][5, 7] = np.nan
    plan, As, outs, w, kk, info = run(P, probs, torch.float64, "f64")
    assert info[0] == -4 and kk[0] == 0
    U, S, VT = outs[0]
    assert bool(torch.all(S == 0)) and bool(torch.all(U == 0)) and bool(torch.all(VT == 0))
    assert np.all(info[1:] == 0)
    plan.close()


def test_lq_postselect():
    import paper_1710_01463_amd as P
    probs = problems(np.float64)
    plan, As, outs, w, kk, info = run(P, probs, torch.float64, "f64")
    S0 = [o[1].cpu().numpy().copy() for o in outs]
    chi = 90
    chi_s = plan.postselect(chi).cpu().numpy()
    assert list(chi_s) == oracle.postselect(S0, kk, chi)
    for b, (U, S, VT) in enumerate(outs):
        cs = int(chi_s[b])
        assert bool(torch.all(VT[cs:] == 0)) and bool(torch.all(U[:, cs:] == 0))
    plan.close()
