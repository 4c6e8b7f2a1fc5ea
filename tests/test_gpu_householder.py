"""GPU parity of the blocked Householder fallback (RSVD_PLAN_BLOCKED_QR).

Steep exponential spectra make the sketch bases so ill-conditioned that the
Cholesky QR breaks down at every stage and every basis goes through the
Householder fallback.  The blocked form (16-column panels in compact WY form,
trailing updates as FP64 MFMA products over 64-column tiles) is forced on
small problems here and compared with the FP64 oracle (bars as in the other
FP64 parity tests) and with the one-workgroup form on the same plan inputs.
Shapes cover a last panel narrower than 16 columns, a single partial panel,
bases of up to 2048 rows (the three register layouts of the panel kernel:
<= 512, <= 1024, <= 2048 rows), tall and wide problems, and batches that mix
problems that break down with problems that do not.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import paper_1710_01463_amd as P
    assert torch.cuda.is_available()
    return P


def run(P, mats, probs, blocked):
    plan = P.Plan(probs, torch.float64, "f64", graph=True, blocked_qr=blocked)
    outs, w, kk, info = plan.execute([torch.from_numpy(A).cuda() for A in mats])
    torch.cuda.synchronize()
    res = [(o[0].cpu().numpy(), o[1].cpu().numpy(), o[2].cpu().numpy()) for o in outs]
    r = (res, w.cpu().numpy(), kk.cpu().numpy(), info.cpu().numpy())
    plan.close()
    return r


def check_vs_oracle(A, pr, U, S, VT, w, kk):
    ref = oracle.rsvd(A, pr["k"], pr["p"], pr["q"], pr["seed"], pr.get("delta", 0.0))
    assert kk == ref.k_kept, (kk, ref.k_kept)
    kept = ref.k_kept
    bar = np.where(ref.S[:kept] >= 1e-5 * ref.S[0], 1e-10 * ref.S[:kept], 1e-15 * ref.S[0])
    assert np.all(np.abs(S[:kept] - ref.S[:kept]) <= bar)
    assert np.all(S[kept:] == 0)
    Uk = U[:, :kept]
    assert np.max(np.abs(Uk.T @ Uk - np.eye(kept))) < 1e-12
    Vk = VT[:kept]
    assert np.max(np.abs(Vk @ Vk.T - np.eye(kept))) < 1e-12
    tot = np.sum(A * A)
    assert abs(w - ref.w) <= 1e-10 * ref.w + 1e-13 * tot
    return ref


def steep(m, n, k, p, q, alpha, seed, delta=1e-12):
    r = min(m, n)
    A = wl.make_matrix(m, n, wl.spectrum_exp(r, alpha), seed=seed)
    return A, dict(m=m, n=n, k=k, p=p, q=q, seed=seed + 11, delta=delta)


@pytest.mark.parametrize("shape", [
    (160, 160, 120, 16, 2, 0.6),   # l = 136: eight full panels and one of 8 columns
    (300, 90, 40, 10, 1, 0.6),     # tall, l = 50 (last panel 2 columns)
    (90, 300, 8, 4, 2, 3.0),       # wide, l = 12: one partial panel
    (700, 500, 150, 16, 2, 0.25),  # rows up to 700: the <= 1024-row panel layout
    (1800, 260, 200, 16, 1, 0.25), # rows up to 1800: the <= 2048-row panel layout
])
def test_blocked_householder_matches_oracle(lib, shape):
    """kappa of every basis is far beyond the Cholesky QR's reach
    (sigma_1 / sigma_l = exp(alpha (l - 1)) >= e^29)."""
    m, n, k, p, q, alpha = shape
    A, pr = steep(m, n, k, p, q, alpha, 900 + m)
    res, w, kk, info = run(lib, [A], [pr], True)
    assert info[0] == 0
    U, S, VT = res[0]
    check_vs_oracle(A, pr, U, S, VT, w[0], kk[0])


def test_blocked_equals_one_workgroup_form(lib):
    """Both forms of the fallback on the same uneven batch: the same kept
    count, singular values to rounding, and the same leading vectors."""
    mats, probs = zip(*[steep(200, 170, 100, 16, 2, 0.5, 40),
                        steep(90, 260, 40, 8, 1, 0.9, 41),
                        steep(333, 333, 160, 16, 2, 0.3, 42)])
    rb, wb, kb, ib = run(lib, mats, probs, True)
    ru, wu, ku, iu = run(lib, mats, probs, False)
    assert np.all(ib == 0) and np.all(iu == 0)
    assert np.array_equal(kb, ku)
    for (Ub, Sb, VTb), (Uu, Su, VTu), kk in zip(rb, ru, kb):
        assert np.max(np.abs(Sb - Su)) <= 1e-12 * Su[0]
        # the leading, well-separated vectors agree up to rounding (same canonical signs)
        assert np.max(np.abs(Ub[:, :8] - Uu[:, :8])) < 1e-9
        assert np.max(np.abs(VTb[:8] - VTu[:8])) < 1e-9


def test_blocked_mixed_batch(lib):
    """A batch in which some problems break down (steep spectra) and others do
    not (a power law): the blocked launches skip the unflagged problems, and
    every problem matches the oracle."""
    mats, probs = [], []
    for b, (m, n) in enumerate([(260, 200), (128, 128), (400, 150), (96, 333)]):
        if b % 2 == 0:
            A, pr = steep(m, n, 60, 10, 2, 0.7, 70 + b)
        else:
            A = wl.make_matrix(m, n, wl.spectrum_power(min(m, n), 1.5), seed=70 + b)
            pr = dict(m=m, n=n, k=48, p=10, q=2, seed=80 + b)
        mats.append(A)
        probs.append(pr)
    res, w, kk, info = run(lib, mats, probs, True)
    assert np.all(info == 0)
    for (U, S, VT), A, pr, wb, kb in zip(res, mats, probs, w, kk):
        check_vs_oracle(A, pr, U, S, VT, wb, kb)


def test_blocked_f32_storage_and_lq_path(lib):
    """FP32 storage with FP32 sketch products (the fallback copies the FP32
    basis in) on a problem with n >= 4 l (the triangular-factor small SVD, whose
    own Cholesky QR of B^T also falls back)."""
    A, pr = steep(120, 700, 24, 8, 2, 0.8, 55)
    A32 = A.astype(np.float32)
    plan = lib.Plan([pr], torch.float32, "f32", graph=True, blocked_qr=True)
    outs, w, kk, info = plan.execute([torch.from_numpy(A32).cuda()])
    torch.cuda.synchronize()
    assert int(info[0]) == 0
    ref = oracle.rsvd(A32.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["seed"], pr["delta"])
    S = outs[0][1].double().cpu().numpy()
    kept = min(int(kk[0]), ref.k_kept)
    assert np.max(np.abs(S[:kept] - ref.S[:kept])) <= 2 * 2.0 ** -24 * ref.S[0]
    U = outs[0][0].double().cpu().numpy()[:, :int(kk[0])]
    assert np.max(np.abs(U.T @ U - np.eye(U.shape[1]))) < 1e-5
    plan.close()
