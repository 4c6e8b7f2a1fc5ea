"""Sector post-selection on the GPU (rsvd_plan_postselect) against the oracle.

The sectors of a block-diagonal matrix are the problems of one plan, each run
with its own rank guess chi'_s = chi / N + c.  After post-selection the number
kept per sector must equal the oracle's selection applied to the same singular
values (an integer decision taken on the GPU's FP64 or FP32 values on both
sides: bit-exact), the dropped triplets must be zero-filled, k_kept lowered,
and each sector's discarded weight must still be its squared Frobenius error.
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


def sector_matrix(m, n, alpha, seed, dtype):
    rng = np.random.default_rng(seed)
    r = min(m, n)
    s = np.exp(-alpha * np.arange(1, r + 1))
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    return ((U * s) @ V.T).astype(dtype)


def run_sectors(P, sizes, chi, c, dtype, np_dtype, dup=None):
    """One plan over the sectors; dup = (i, j) makes sector j a copy of sector i
    (same matrix and seed), so their values tie exactly."""
    nsec = len(sizes)
    kprime = chi // nsec + c
    mats, probs = [], []
    for b in range(nsec):
        src = dup[0] if dup and b == dup[1] else b
        m, n, alpha = sizes[src]
        mats.append(sector_matrix(m, n, alpha, 500 + src, np_dtype))
        probs.append(dict(m=m, n=n, k=kprime, p=8, q=2, seed=77 + src))
    As = [torch.from_numpy(A).cuda() for A in mats]
    plan = P.Plan(probs, dtype, "f64" if dtype == torch.float64 else "f32", graph=True)
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    S0 = [o[1].double().cpu().numpy().copy() for o in outs]
    kk0 = kk.cpu().numpy().copy()
    w0 = w.cpu().numpy().copy()
    chi_s = plan.postselect(chi).cpu().numpy()
    torch.cuda.synchronize()
    return plan, As, outs, w, kk, S0, kk0, w0, chi_s


def check_after(As, outs, w, kk, S0, kk0, w0, chi_s, exp, rel):
    assert list(chi_s) == exp
    kk1 = kk.cpu().numpy()
    w1 = w.cpu().numpy()
    for b, (A, (U, S, VT)) in enumerate(zip(As, outs)):
        cs = int(chi_s[b])
        assert kk1[b] == cs
        s = S.double().cpu().numpy()
        assert np.array_equal(s[:cs], S0[b][:cs]) and np.all(s[cs:] == 0)
        assert bool(torch.all(U[:, cs:] == 0)) and bool(torch.all(VT[cs:] == 0))
        dropped = np.sum(S0[b][cs:kk0[b]] ** 2)
        a2 = float((A.double() ** 2).sum())
        assert abs(w1[b] - (w0[b] + dropped)) <= 1e-12 * a2
        Ud, Vd = U.double()[:, :cs], VT.double()[:cs]
        R = A.double() - (Ud * torch.from_numpy(s[:cs]).cuda()) @ Vd
        assert abs(float((R * R).sum()) - w1[b]) <= rel * a2


SIZES = [(120, 90, 0.05), (64, 200, 0.08), (150, 150, 0.03), (40, 33, 0.2), (96, 128, 0.06), (200, 70, 0.04)]


@pytest.mark.parametrize("chi", [60, 150, 1000])
def test_postselect_f64_matches_oracle(lib, chi):
    plan, As, outs, w, kk, S0, kk0, w0, chi_s = run_sectors(lib, SIZES, chi, 6, torch.float64, np.float64)
    exp = oracle.postselect(S0, kk0, chi)
    check_after(As, outs, w, kk, S0, kk0, w0, chi_s, exp, 1e-12)
    assert sum(exp) == min(chi, int(kk0.sum()))
    plan.close()


def test_postselect_f32_matches_oracle(lib):
    chi = 100
    plan, As, outs, w, kk, S0, kk0, w0, chi_s = run_sectors(lib, SIZES, chi, 4, torch.float32, np.float32)
    check_after(As, outs, w, kk, S0, kk0, w0, chi_s, oracle.postselect(S0, kk0, chi), 1e-5)
    plan.close()


def test_postselect_exact_ties_go_to_the_lower_sector(lib):
    """Sectors 1 and 4 are the same matrix with the same seed: every value of
    sector 4 ties with one of sector 1; the oracle's order decides."""
    sizes = list(SIZES)
    for chi in (41, 77):
        plan, As, outs, w, kk, S0, kk0, w0, chi_s = run_sectors(lib, sizes, chi, 5, torch.float64, np.float64,
                                                                dup=(1, 4))
        assert np.array_equal(S0[1], S0[4])
        exp = oracle.postselect(S0, kk0, chi)
        check_after(As, outs, w, kk, S0, kk0, w0, chi_s, exp, 1e-12)
        plan.close()


def test_postselect_edge_cases(lib):
    # chi = 0 drops everything: w becomes ||A||^2
    plan, As, outs, w, kk, S0, kk0, w0, chi_s = run_sectors(lib, SIZES[:3], 0, 4, torch.float64, np.float64)
    check_after(As, outs, w, kk, S0, kk0, w0, chi_s, [0, 0, 0], 1e-12)
    for b, A in enumerate(As):
        a2 = float((A.double() ** 2).sum())
        assert abs(float(w[b]) - a2) <= 1e-12 * a2
    plan.close()
    # chi above the number of candidates keeps everything
    plan, As, outs, w, kk, S0, kk0, w0, chi_s = run_sectors(lib, SIZES[:3], 10 ** 6, 4, torch.float64, np.float64)
    check_after(As, outs, w, kk, S0, kk0, w0, chi_s, [int(x) for x in kk0], 1e-12)
    plan.close()


def test_postselect_many_sectors_c2_shape(lib):
    """The 32-problem C2 batch as one sector group (8192 candidates), half kept."""
    W = wl.c2(32)
    mats = [pr.matrix() for pr in W.problems[:32]]
    As = [torch.from_numpy(A).cuda() for A in mats]
    plan = lib.Plan([dict(m=pr.m, n=pr.n, k=pr.k, p=pr.p, q=pr.q, seed=pr.seed) for pr in W.problems],
                    torch.float64, "f64", graph=True)
    outs, w, kk, info = plan.execute(As)
    torch.cuda.synchronize()
    S0 = [o[1].cpu().numpy().copy() for o in outs]
    kk0 = kk.cpu().numpy().copy()
    w0 = w.cpu().numpy().copy()
    chi = 4096
    chi_s = plan.postselect(chi).cpu().numpy()
    exp = oracle.postselect(S0, kk0, chi)
    check_after(As, outs, w, kk, S0, kk0, w0, chi_s, exp, 1e-12)
    plan.close()
