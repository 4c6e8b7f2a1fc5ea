"""GPU parity of the mixed-precision paths and of uneven batches.

Tolerances on singular values are relative to sigma_1:
  FP32 sketch/power products:  <= 1e-6 before refinement, <= 1e-8 after on
  decaying spectra.  On nearly flat spectra (the exponential ones with small
  alpha) the power steps do not damp the directions the FP32 rounding of the
  products perturbs, and the singular values of B = Q^T A depend on the
  sampled subspace at first order: |d sigma_i| ~ u32 sigma_i (u32 = 2^-24),
  which no FP64 pass over the same subspace removes; the bar there is
  2 u32 sigma_1.
  BF16 sketch/power products:  <= 1e-3 before refinement; after the FP64
  refinement pass of B the same first-order mechanism leaves about 1e-6
  sigma_1 at the last kept index (the leading quarter of the kept values
  sits near 5e-8), so the bar is 2e-5 and 1e-8 is not reached.
The FP64 oracle runs on the exact FP32-stored matrix, upcast.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as wl

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def lib():
    import paper_1710_01463_amd as P
    assert torch.cuda.is_available()
    return P


def run_plan(P, mats, probs, dtype, prec, refine=True):
    plan = P.Plan(probs, dtype, prec, refine=refine)
    outs, w, kk, info = plan.execute([torch.from_numpy(np.ascontiguousarray(A)).to(dtype).cuda()
                                      for A in mats])
    torch.cuda.synchronize()
    res = [(o[0].double().cpu().numpy(), o[1].double().cpu().numpy(), o[2].double().cpu().numpy())
           for o in outs]
    return res, w.cpu().numpy(), kk.cpu().numpy(), info.cpu().numpy()


def case(m, n, k, p, q, s, seed):
    A = wl.make_matrix(m, n, s, seed=seed).astype(np.float32)
    return A, dict(m=m, n=n, k=k, p=p, q=q, seed=seed + 7)


@pytest.mark.parametrize("refine,tol", [(True, 1e-8), (False, 1e-6)])
def test_f32_sketch_power_law(lib, refine, tol):
    """C2-like critical spectrum (s_i = i^-1.5), FP32 storage and FP32 products."""
    mats, probs = zip(*[case(256, 256, 96, 16, 2, wl.spectrum_power(256, 1.5), 300 + b) for b in range(3)])
    res, w, kk, info = run_plan(lib, mats, probs, torch.float32, "f32", refine)
    assert np.all(info == 0)
    for (U, S, VT), A, pr in zip(res, mats, probs):
        ref = oracle.rsvd(A.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["seed"])
        err = np.max(np.abs(S - ref.S)) / ref.S[0]
        assert err <= tol, err
        k = len(S)
        assert np.linalg.norm(U.T @ U - np.eye(k)) < 1e-5
        assert np.linalg.norm(VT @ VT.T - np.eye(k)) < 1e-5


@pytest.mark.parametrize("refine,tol", [(True, 2e-5), (False, 1e-3)])
def test_bf16_sketch_noisy_power_law(lib, refine, tol):
    """C3-like spectrum (|i^-1.2 (1 + 0.05 xi)|), BF16 products with FP32 accumulate."""
    s = wl.spectrum_noisy_power(384, 1.2, 0.05, 11)
    mats, probs = zip(*[case(384, 384, 32, 16, 3, s, 400 + b) for b in range(2)])
    res, w, kk, info = run_plan(lib, mats, probs, torch.float32, "bf16", refine)
    assert np.all(info == 0)
    for (U, S, VT), A, pr in zip(res, mats, probs):
        ref = oracle.rsvd(A.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["seed"])
        err = np.max(np.abs(S - ref.S)) / ref.S[0]
        assert err <= tol, err


def test_f32_with_degenerate_pairs(lib):
    """C5-like spectrum with three near-degenerate pairs (relative gap 1e-6)."""
    s = wl.spectrum_power_with_pairs(200, 1.5)
    mats, probs = zip(*[case(200, 200, 64, 16, 2, s, 500)])
    res, w, kk, info = run_plan(lib, mats, probs, torch.float32, "f32")
    U, S, VT = res[0]
    ref = oracle.rsvd(mats[0].astype(np.float64), 64, 16, 2, probs[0]["seed"])
    assert np.max(np.abs(S - ref.S)) / ref.S[0] <= 1e-8
    # the pairs: compare the 2-dimensional projectors, not the vectors
    for i in (8, 40):
        a = U[:, i - 1:i + 1]
        b = ref.U[:, i - 1:i + 1]
        assert np.linalg.norm(a @ a.T - b @ b.T, 2) < 1e-5


def c4_like(count, seed, max_dim):
    """Uneven batch drawn like the symmetry-sector workload, scaled down so the
    oracle stays fast: m, n uniform in [32, max_dim], k = min(m, n)/4 rounded
    to 8 (at least 8), s_i = exp(-alpha i), alpha in [0.005, 0.1], delta = 1e-10."""
    rng = np.random.default_rng(seed)
    mats, probs = [], []
    for b in range(count):
        m = int(rng.integers(32, max_dim, endpoint=True))
        n = int(rng.integers(32, max_dim, endpoint=True))
        alpha = float(rng.uniform(0.005, 0.1))
        r = min(m, n)
        k = max(8, 8 * int(np.floor(r / 32 + 0.5)))
        s = wl.spectrum_exp(r, alpha)
        mats.append(wl.make_matrix(m, n, s, seed=6000 + b).astype(np.float32))
        probs.append(dict(m=m, n=n, k=k, p=16, q=2, seed=7000 + b, delta=1e-10))
    return mats, probs


def test_uneven_batch_f32(lib):
    """FP32 sketch on the uneven exponential-spectrum batch.  Where alpha is
    small the spectrum is nearly flat over the sketched range and the RSVD's
    singular values depend on the sampled subspace at first order, so the FP32
    rounding of that subspace reaches them at about u32 sigma_i: bar 2 u32
    sigma_1 (the 1e-8 bar holds on the decaying spectra above)."""
    mats, probs = c4_like(24, 4, 320)
    res, w, kk, info = run_plan(lib, mats, probs, torch.float32, "f32")
    assert np.all(info == 0), info
    for i, ((U, S, VT), A, pr) in enumerate(zip(res, mats, probs)):
        A64 = A.astype(np.float64)
        ref = oracle.rsvd(A64, pr["k"], pr["p"], pr["q"], pr["seed"], pr["delta"])
        tot = np.sum(A64 ** 2)
        # k_kept is an integer decided by FP64 sums on both sides; equal unless
        # the relative discarded weight sits on the threshold
        if kk[i] != ref.k_kept:
            assert abs(ref.w / tot - 1e-10) < 1e-11, (i, kk[i], ref.k_kept)
            continue
        kept = ref.k_kept
        err = np.max(np.abs(S[:kept] - ref.S[:kept])) / ref.S[0]
        print(f"problem {i}: {pr['m']}x{pr['n']} k={pr['k']} kept={kept} max|dS|/s1={err:.2e}")
        assert err <= 2 * 2.0 ** -24, (i, err)
        assert np.all(S[kept:] == 0)
        assert abs(w[i] - ref.w) <= 1e-8 * tot, (i, w[i], ref.w)
        assert np.linalg.norm(U[:, :kept].T @ U[:, :kept] - np.eye(kept)) < 1e-5


def test_uneven_batch_f64_matches_one_at_a_time(lib):
    """One plan over an uneven batch gives bit-identical results to one call
    per problem (the test matrix depends on the seed only)."""
    mats, probs = c4_like(12, 5, 200)
    mats = [A.astype(np.float64) for A in mats]
    res, w, kk, info = run_plan(lib, mats, probs, torch.float64, "f64")
    for i, ((U, S, VT), A, pr) in enumerate(zip(res, mats, probs)):
        U1, S1, VT1, w1, k1 = lib.rsvd_truncate(torch.from_numpy(A).cuda(), pr["k"], pr["p"], pr["q"],
                                                pr["seed"], pr["delta"])
        assert np.array_equal(S, S1.cpu().numpy())
        assert np.array_equal(U, U1.cpu().numpy())
        assert int(k1.item()) == kk[i]


def test_householder_fallback_on_steep_spectrum(lib):
    """kappa(Y) far beyond 1e8 (exponential tail down to 1e-40): Cholesky QR
    breaks down, the Householder fallback keeps Q orthonormal, and the kept
    triplets match the oracle."""
    m = n = 160
    s = wl.spectrum_exp(160, 0.6)
    A = wl.make_matrix(m, n, s, seed=77)
    ref = oracle.rsvd(A, 120, 16, 2, 5, 1e-12)
    res, w, kk, info = run_plan(lib, [A], [dict(m=m, n=n, k=120, p=16, q=2, seed=5, delta=1e-12)],
                                torch.float64, "f64")
    U, S, VT = res[0]
    assert info[0] == 0 and kk[0] == ref.k_kept
    kept = ref.k_kept
    assert np.all(np.abs(S[:kept] - ref.S[:kept]) <= np.maximum(1e-10 * ref.S[:kept], 1e-15 * ref.S[0]))
    assert np.linalg.norm(U[:, :kept].T @ U[:, :kept] - np.eye(kept)) < 1e-12


def test_fp64_final_power_step(lib):
    """RSVD_PLAN_FP64_FINAL: the last power step (A^T Q, A Z and their Cholesky
    QRs) in FP64 from the stored A.  Bars from the first-order model of the
    mixed-precision error (written before this test was first run): each FP64
    power step shrinks the sketch precision's subspace error by about
    (sigma_{l+1} / sigma_k)^2, so on the BF16 noisy power law (C3-like, k = 32,
    p = 16, q = 3) the error must not grow (the model predicts about half), and
    on the nearly flat exponential spectra of the uneven FP32 batch it stays
    within 2 u32 sigma_1 (the FP32 outputs' own rounding plus the sketch term).  FP64 plans ignore
    the flag; plans with differing q, or q = 0, are rejected."""
    s = wl.spectrum_noisy_power(384, 1.2, 0.05, 11)
    mats, probs = zip(*[case(384, 384, 32, 16, 3, s, 400 + b) for b in range(2)])
    plain, _, _, info_p = run_plan(lib, mats, probs, torch.float32, "bf16")
    plan = lib.Plan(probs, torch.float32, "bf16", fp64_final=True)
    outs, w, kk, info = plan.execute([torch.from_numpy(np.ascontiguousarray(A)).cuda() for A in mats])
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and np.all(info_p == 0)
    for (Up, Sp, VTp), o, A, pr in zip(plain, outs, mats, probs):
        ref = oracle.rsvd(A.astype(np.float64), pr["k"], pr["p"], pr["q"], pr["seed"])
        e_plain = np.max(np.abs(Sp - ref.S)) / ref.S[0]
        e_final = np.max(np.abs(o[1].double().cpu().numpy() - ref.S)) / ref.S[0]
        print(f"BF16 max|dS|/s1: {e_plain:.2e} plain, {e_final:.2e} with the FP64 final power step")
        assert e_final <= 1.05 * e_plain and e_final <= 2e-5
    plan.close()
    mats, probs = c4_like(12, 4, 320)
    probs = [dict(pr, q=2) for pr in probs]
    res, w, kk, info = run_plan(lib, mats, probs, torch.float32, "f32")
    plan = lib.Plan(probs, torch.float32, "f32", fp64_final=True)
    outs, w2, kk2, info2 = plan.execute([torch.from_numpy(np.ascontiguousarray(A)).cuda() for A in mats])
    torch.cuda.synchronize()
    assert np.all(info2.cpu().numpy() == 0)
    kk2 = kk2.cpu().numpy()
    for i, (o, A, pr) in enumerate(zip(outs, mats, probs)):
        A64 = A.astype(np.float64)
        ref = oracle.rsvd(A64, pr["k"], pr["p"], pr["q"], pr["seed"], pr["delta"])
        if kk2[i] != ref.k_kept:
            assert abs(ref.w / np.sum(A64 ** 2) - 1e-10) < 1e-11
            continue
        S = o[1].double().cpu().numpy()
        kept = ref.k_kept
        e_final = np.max(np.abs(S[:kept] - ref.S[:kept])) / ref.S[0]
        e_plain = np.max(np.abs(res[i][1][:kept] - ref.S[:kept])) / ref.S[0]
        print(f"FP32 flat problem {i}: {e_plain:.2e} plain, {e_final:.2e} with the FP64 final power step")
        assert e_final <= 2 * 2.0 ** -24
    plan.close()
    # rejected forms
    with pytest.raises(RuntimeError):
        lib.Plan([dict(m=64, n=64, k=8, p=4, q=0, seed=1)], torch.float32, "f32", fp64_final=True)
    with pytest.raises(RuntimeError):
        lib.Plan([dict(m=64, n=64, k=8, p=4, q=1, seed=1), dict(m=64, n=64, k=8, p=4, q=2, seed=2)],
                 torch.float32, "f32", fp64_final=True)
