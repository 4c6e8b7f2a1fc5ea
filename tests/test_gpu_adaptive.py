"""Fixed-error RSVD with an adaptive rank (rsvd_truncate_adaptive) against the
oracle's loop: the same ranks are tried (same number of attempts), the same
k_kept (up to one where the discarded weight sits on the threshold), the FP64
singular values within the parity bar, the error target met whenever the cut
binds, and zero triplets beyond k_kept."""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1710_01463_amd as P
    assert torch.cuda.is_available()
    return P


CASES = [  # m, n, alpha, k0, k_max, p, q, delta
    (200, 150, 0.05, 8, 150, 10, 2, 1e-6),
    (96, 300, 0.12, 4, 64, 8, 1, 1e-8),
    (256, 256, 0.03, 16, 256, 16, 2, 1e-4),
    (180, 120, 0.02, 4, 24, 10, 2, 1e-6),  # capped before the target
]


@pytest.mark.parametrize("case", CASES)
def test_adaptive_f64_matches_oracle(P, case):
    m, n, alpha, k0, kmax, p, q, delta = case
    A = wl.make_matrix(m, n, np.exp(-alpha * np.arange(1, min(m, n) + 1)), 40 + m)
    U, S, VT, w, kk, att = P.rsvd_truncate_adaptive(torch.from_numpy(A).cuda(), k0, kmax, delta, p, q, seed=5)
    ref, ratt = oracle.rsvd_adaptive(A, k0, kmax, p, q, 5, delta)
    kk = int(kk.item())
    w = float(w.item())
    a2 = float(np.sum(A * A))
    kcap = min(kmax, m, n)
    assert att == ratt
    on_threshold = abs(ref.w / a2 - delta) < 1e-9 * max(delta, 1e-12) + 1e-12
    assert kk == ref.k_kept or (on_threshold and abs(kk - ref.k_kept) <= 1)
    s = S.cpu().numpy()
    r = min(kk, ref.k_kept)
    bar = np.where(ref.S[:r] >= 1e-5 * ref.S[0], 1e-10 * ref.S[:r], 1e-15 * ref.S[0])
    assert np.all(np.abs(s[:r] - ref.S[:r]) <= bar)
    assert np.all(s[kk:] == 0) and bool(torch.all(U[:, kk:] == 0)) and bool(torch.all(VT[kk:] == 0))
    assert S.shape[0] == kcap
    Ud, Vd = U.double()[:, :kk], VT.double()[:kk]
    R = torch.from_numpy(A).cuda() - (Ud * S.double()[:kk]) @ Vd
    assert abs(float((R * R).sum()) - w) <= 1e-12 * a2
    if kk < kcap:
        assert w <= delta * a2 * (1 + 1e-9)


def test_adaptive_exact_low_rank(P):
    rng = np.random.default_rng(3)
    m, n, r = 90, 70, 21
    U0, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V0, _ = np.linalg.qr(rng.standard_normal((n, r)))
    A = (U0 * np.linspace(3.0, 1.0, r)) @ V0.T
    for k0, expect in [(4, 4), (6, 3), (22, 1), (21, 2)]:
        U, S, VT, w, kk, att = P.rsvd_truncate_adaptive(torch.from_numpy(A).cuda(), k0, 70, 1e-12, 5, 1, seed=11)
        assert att == expect and int(kk.item()) == r
        rec = (U.double()[:, :r] * S.double()[:r]) @ VT.double()[:r]
        assert float((rec - torch.from_numpy(A).cuda()).abs().max()) < 1e-12


def test_adaptive_f32_storage(P):
    m, n = 160, 140
    A = wl.make_matrix(m, n, np.exp(-0.06 * np.arange(1, 141)), 77).astype(np.float32)
    U, S, VT, w, kk, att = P.rsvd_truncate_adaptive(torch.from_numpy(A).cuda(), 8, 140, 1e-5, 10, 2, seed=9,
                                                    prec="f32")
    ref, ratt = oracle.rsvd_adaptive(A.astype(np.float64), 8, 140, 10, 2, 9, 1e-5)
    assert att == ratt and abs(int(kk.item()) - ref.k_kept) <= 1
    r = min(int(kk.item()), ref.k_kept)
    assert np.max(np.abs(S.double().cpu().numpy()[:r] - ref.S[:r])) / ref.S[0] <= 1e-6


def test_adaptive_rejects_bad_arguments(P):
    A = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    from paper_1710_01463_amd._lib import RsvdError
    with pytest.raises(RsvdError):
        P.rsvd_truncate_adaptive(A, 4, 8, 0.0)
    with pytest.raises(RsvdError):
        P.rsvd_truncate_adaptive(A, 5, 4, 1e-3)
