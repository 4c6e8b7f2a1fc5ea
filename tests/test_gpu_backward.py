"""GPU parity of the hand-written adjoint (rsvd_plan_backward) against the
oracle's FP64 adjoint on the same seeds, the same test matrices and the same
cotangents; against central finite differences of the GPU forward; and, at
full sketch width, against the full-SVD reference gradient.

Tolerances (max-norm relative to max |dA|): FP64 1e-9.  The adjoint divides
by s_j^2 - s_i^2 and by the pivots of every R, so forward rounding differences
of order 1e-15 grow by the conditioning of those quantities; the spectra here
keep that growth below 1e4.  FP32 storage with FP32 sketch products: 2e-5
(measured 4e-7 on the case below: the forward's bases differ from the FP64
ones at the FP32 rounding level, which the adjoint's divisions by singular
value gaps amplify by less than 1e2 on this spectrum).
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


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_backward(P, mats, probs, cots, dtype=torch.float64, prec="f64", broad=0.0):
    plan = P.Plan(probs, dtype, prec, graph=False, save=True)
    As = [torch.from_numpy(np.ascontiguousarray(A)).to(dtype).cuda() for A in mats]
    outs, w, kk, info = plan.execute(As)
    dU = [torch.from_numpy(c[0]).to(dtype).cuda() for c in cots]
    dS = [torch.from_numpy(c[1]).to(dtype).cuda() for c in cots]
    dVT = [torch.from_numpy(c[2]).to(dtype).cuda() for c in cots]
    dA = plan.backward(dU, dS, dVT, broad)
    torch.cuda.synchronize()
    res = [g.double().cpu().numpy() for g in dA]
    fw = [(o[0].double().cpu().numpy(), o[1].double().cpu().numpy(), o[2].double().cpu().numpy()) for o in outs]
    info = info.cpu().numpy()
    plan.close()
    return res, fw, info


def case(m, n, k, p, q, alpha, seed):
    A = wl.make_matrix(m, n, wl.spectrum_exp(min(m, n), alpha), seed=seed)
    kk = min(k, m, n)
    return A, dict(m=m, n=n, k=k, p=p, q=q, seed=seed + 17), wl.cotangents(m, n, kk, seed + 29)


SHAPES = [(150, 100, 20, 8, 2), (90, 170, 24, 6, 1), (64, 64, 16, 0, 0), (200, 131, 40, 16, 3),
          (33, 47, 9, 5, 2)]


@pytest.mark.parametrize("m,n,k,p,q", SHAPES)
def test_backward_f64_matches_oracle(lib, m, n, k, p, q):
    A, pr, cot = case(m, n, k, p, q, 0.1, m + 3 * n)
    print(f"case m={m} n={n} k={k} p={p} q={q}", flush=True)
    got, _, info = gpu_backward(lib, [A], [pr], [cot])
    assert info[0] == 0
    ref = oracle.rsvd_backward(A, k, p, q, pr["seed"], *cot)
    err = relerr(got[0], ref)
    print(f"max|dA - ref| / max|ref| = {err:.2e}")
    assert err <= 1e-9, err


def test_backward_uneven_batch_f64(lib):
    """One plan over problems with different shapes and power-iteration counts
    (q = 0..3): the reverse stage loop must pick each problem's own stages."""
    shapes = [(120, 80, 16, 8, 0), (70, 140, 12, 4, 3), (96, 96, 24, 8, 1), (50, 61, 10, 6, 2),
              (130, 45, 8, 8, 2)]
    cases = [case(*s, 0.12, 500 + i) for i, s in enumerate(shapes)]
    mats, probs, cots = zip(*cases)
    got, _, info = gpu_backward(lib, mats, probs, cots)
    assert np.all(info == 0)
    for i, (A, pr, cot) in enumerate(cases):
        ref = oracle.rsvd_backward(A, pr["k"], pr["p"], pr["q"], pr["seed"], *cot)
        err = relerr(got[i], ref)
        print(f"problem {i} {shapes[i]}: {err:.2e}")
        assert err <= 1e-9, (i, err)


def test_backward_with_truncation_and_broadening(lib):
    """delta_trunc drops trailing triplets (their cotangents are ignored) and a
    Lorentzian broadening replaces 1/(s_j^2 - s_i^2)."""
    A, pr, cot = case(110, 90, 40, 10, 2, 0.25, 77)
    pr["delta"] = 1e-6
    for broad in (0.0, 1e-6):
        got, fw, info = gpu_backward(lib, [A], [pr], [cot], broad=broad)
        ref_f = oracle.rsvd(A, 40, 10, 2, pr["seed"], 1e-6)
        assert ref_f.k_kept < 40
        assert np.count_nonzero(fw[0][1]) == ref_f.k_kept
        ref = oracle.rsvd_backward(A, 40, 10, 2, pr["seed"], *cot, delta=1e-6, broad=broad)
        err = relerr(got[0], ref)
        print(f"broad={broad}: k_kept={ref_f.k_kept} err={err:.2e}")
        assert err <= 1e-9, (broad, err)


def test_backward_matches_gpu_finite_differences(lib):
    """Central differences of the GPU forward itself (h = 1e-6, FP64)."""
    m, n, k, p, q = 80, 72, 12, 6, 2
    A, pr, cot = case(m, n, k, p, q, 0.15, 9)
    got, _, _ = gpu_backward(lib, [A], [pr], [cot])
    dU, dS, dVT = cot
    rng = np.random.default_rng(5)
    At = torch.from_numpy(A).cuda()
    for t in range(3):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        Et = torch.from_numpy(E).cuda()
        vals = []
        for sgn in (1.0, -1.0):
            U, S, VT, w, kk = lib.rsvd_truncate(At + sgn * 1e-6 * Et, k, p, q, pr["seed"])
            vals.append(np.sum(dU * U.cpu().numpy()) + np.sum(dS * S.cpu().numpy()) +
                        np.sum(dVT * VT.cpu().numpy()))
        fd = (vals[0] - vals[1]) / 2e-6
        an = float(np.sum(got[0] * E))
        print(f"direction {t}: fd={fd:.10e} adjoint={an:.10e}")
        assert abs(fd - an) <= 2e-6 * max(abs(fd), np.linalg.norm(got[0])), (t, fd, an)


@pytest.mark.parametrize("m,n,k", [(96, 80, 20), (70, 100, 16)])
def test_full_width_equals_full_svd_reference_gradient(lib, m, n, k):
    """With l = min(m, n) the RSVD is the exact truncated SVD; its gradient
    through every QR and GEMM of the GPU path equals the oracle's SVD adjoint
    of A (an independent formula)."""
    A, pr, cot = case(m, n, k, 200, 2, 0.2, 31)
    got, _, info = gpu_backward(lib, [A], [pr], [cot])
    ref = oracle.fullsvd_backward(A, k, *cot)
    err = relerr(got[0], ref)
    print(f"full width: {err:.2e}")
    assert err <= 1e-8, err


def test_near_degenerate_pairs_with_invariant_loss(lib):
    """C5-like spectrum (power law with three pairs at relative gap 1e-6).  A
    loss that depends on the kept subspace only through U U^T and on S,
    L = tr(U^T G U) + sum(S), has a finite gradient however close the pair;
    cotangents dU = 2 G U are formed from each side's own U."""
    m = n = 160
    s = wl.spectrum_power_with_pairs(160, 1.5, pairs=(8, 40, 100))
    A = wl.make_matrix(m, n, s, seed=41)
    k, p, q, seed = 48, 16, 2, 12
    rng = np.random.default_rng(3)
    G = rng.standard_normal((m, m))
    G = G + G.T
    ref_f = oracle.rsvd(A, k, p, q, seed)
    cot_ref = (2 * G @ ref_f.U, np.ones(k), np.zeros((k, n)))
    ref = oracle.rsvd_backward(A, k, p, q, seed, *cot_ref)
    P = lib
    plan = P.Plan([dict(m=m, n=n, k=k, p=p, q=q, seed=seed)], torch.float64, "f64", graph=False, save=True)
    outs, _, _, info = plan.execute([torch.from_numpy(A).cuda()])
    U = outs[0][0]
    Gt = torch.from_numpy(G).cuda()
    dA = plan.backward([2 * Gt @ U], [torch.ones(k, dtype=torch.float64, device="cuda")],
                       [torch.zeros((k, n), dtype=torch.float64, device="cuda")])
    torch.cuda.synchronize()
    err = relerr(dA[0].cpu().numpy(), ref)
    print(f"invariant loss across pairs: {err:.2e}")
    assert err <= 1e-7, err


def test_backward_f32_sketch(lib):
    """FP32 storage and FP32 sketch products; the adjoint's products run in
    FP64 on the FP32-stored A.  Oracle on the upcast A."""
    m, n, k, p, q = 256, 192, 32, 16, 2
    A, pr, cot = case(m, n, k, p, q, 0.05, 13)
    A = A.astype(np.float32).astype(np.float64)
    got, _, info = gpu_backward(lib, [A], [pr], [cot], dtype=torch.float32, prec="f32")
    assert info[0] == 0
    ref = oracle.rsvd_backward(A, k, p, q, pr["seed"], *cot)
    err = relerr(got[0], ref)
    print(f"f32: {err:.2e}")
    assert err <= 2e-5, err


def test_autograd_function_batch(lib):
    """torch.autograd through RSVDFunction gives the oracle's gradient of a
    scalar loss built from the outputs (cotangents reach the library through
    autograd)."""
    P = lib
    shapes = [(100, 90), (64, 120)]
    mats = [wl.make_matrix(m, n, wl.spectrum_exp(min(m, n), 0.1), seed=60 + i) for i, (m, n) in enumerate(shapes)]
    k, p, q = 12, 8, 2
    As = [torch.from_numpy(A).cuda().requires_grad_(True) for A in mats]
    outs = P.rsvd_batch(As, k, p, q, seeds=[5, 6])
    cots = [wl.cotangents(m, n, k, 70 + i) for i, (m, n) in enumerate(shapes)]
    loss = 0
    for (U, S, VT), (dU, dS, dVT) in zip(outs, cots):
        loss = loss + (U * torch.from_numpy(dU).cuda()).sum() + (S * torch.from_numpy(dS).cuda()).sum() + \
            (VT * torch.from_numpy(dVT).cuda()).sum()
    grads = torch.autograd.grad(loss, As)
    for i, g in enumerate(grads):
        ref = oracle.rsvd_backward(mats[i], k, p, q, 5 + i, *cots[i])
        err = relerr(g.cpu().numpy(), ref)
        print(f"autograd problem {i}: {err:.2e}")
        assert err <= 1e-9, (i, err)


def test_backward_needs_a_saving_plan(lib):
    P = lib
    plan = P.Plan([dict(m=40, n=30, k=5, p=4, q=1, seed=1)], torch.float64, "f64", graph=False, save=False)
    A = torch.from_numpy(wl.make_matrix(40, 30, wl.spectrum_exp(30, 0.2), seed=1)).cuda()
    plan.execute([A])
    z = [torch.zeros_like(t) for t in plan.outputs[0]]
    with pytest.raises(P._lib.RsvdError):
        plan.backward([z[0]], [z[1]], [z[2]])
    plan.close()
