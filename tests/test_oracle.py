"""Pins of the FP64 CPU oracle against facts fixed outside the oracle itself:
published known-answer vectors, closed forms, library routines (numpy/LAPACK),
invariants of the SVD (Eckart-Young-Mirsky), and the Halko-Martinsson-Tropp
expected-error bounds for the randomized range finder.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads as wl
from conftest import load_kat

EPS = 2.0 ** -53


# ---------------------------------------------------------------- Philox / Omega
@pytest.mark.parametrize("row", load_kat())
def test_philox_known_answers(row):
    ctr, key, expect = row
    got = oracle.philox4x32_10(ctr, key)
    assert tuple(int(x) for x in got) == expect


def test_gaussian_moments_and_ks():
    om = oracle.gaussian(12345, 400, 250)
    x = om.ravel()
    assert abs(x.mean()) < 5.0 / math.sqrt(x.size)
    assert abs(x.var() - 1.0) < 5.0 * math.sqrt(2.0 / x.size)
    assert stats.kstest(x, "norm").pvalue > 1e-3


def test_gaussian_box_muller_pairs():
    """Each (even, odd) pair of a column is one Box-Muller draw: its angle is
    uniform on (-pi, pi] and its squared radius is exponential with mean 2."""
    om = oracle.gaussian(777, 600, 120)
    a, b = om[0::2, :].ravel(), om[1::2, :].ravel()
    ang = np.arctan2(b, a)
    assert stats.kstest(ang, stats.uniform(loc=-np.pi, scale=2 * np.pi).cdf).pvalue > 1e-3
    r2 = a * a + b * b
    assert stats.kstest(r2, stats.expon(scale=2.0).cdf).pvalue > 1e-3


def test_gaussian_independence_and_layout():
    om = oracle.gaussian(99, 512, 64)
    c = np.corrcoef(om.T)
    off = c[~np.eye(64, dtype=bool)]
    assert np.max(np.abs(off)) < 6.0 / math.sqrt(512)
    # stateless: any sub-block equals the corresponding block of a larger draw
    small = oracle.gaussian(99, 37, 11)
    assert np.array_equal(small, om[:37, :11])
    # different seeds differ; seed high word matters
    assert not np.array_equal(oracle.gaussian(99 + (1 << 32), 8, 8), om[:8, :8])


# ---------------------------------------------------------------- Householder QR
@pytest.mark.parametrize("shape", [(1, 1), (7, 3), (64, 64), (130, 37)])
def test_hqr_against_lapack(shape):
    rng = np.random.default_rng(1)
    Y = rng.standard_normal(shape)
    Q, R = oracle.hqr(Y)
    m, l = shape
    assert np.allclose(np.triu(R), R)
    assert np.all(np.diag(R) >= 0)
    assert np.linalg.norm(Q.T @ Q - np.eye(l)) < 50 * m * EPS
    assert np.linalg.norm(Q @ R - Y) < 50 * m * EPS * np.linalg.norm(Y)
    Ql, Rl = np.linalg.qr(Y)
    d = np.sign(np.diag(Rl))
    assert np.allclose(Q, Ql * d, atol=1e-12)
    assert np.allclose(R, Rl * d[:, None], atol=1e-12)


def test_hqr_rank_deficient_is_orthonormal():
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 10))
    Q, R = oracle.hqr(Y)
    assert np.linalg.norm(Q.T @ Q - np.eye(10)) < 1e-13
    assert np.linalg.norm(Q @ R - Y) < 1e-12 * np.linalg.norm(Y)


# ---------------------------------------------------------------- Jacobi SVD
def test_jacobi_2x2_closed_form():
    a, b, c, d = 3.0, -1.25, 0.5, 2.0
    G, J, st, _ = oracle.jacobi_cols(np.array([[a, b], [c, d]]))
    assert st == 0
    s = np.sort(np.linalg.norm(G, axis=0))[::-1]
    S = a * a + b * b + c * c + d * d
    D = abs(a * d - b * c)
    s1 = math.sqrt((S + math.sqrt(S * S - 4 * D * D)) / 2)
    s2 = D / s1
    assert abs(s[0] - s1) < 4 * EPS * s1
    assert abs(s[1] - s2) < 8 * EPS * s1


def test_jacobi_rank_one_diag_perm():
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(9), rng.standard_normal(5)
    G, J, st, _ = oracle.jacobi_cols(np.outer(x, y))
    s = np.sort(np.linalg.norm(G, axis=0))[::-1]
    assert abs(s[0] - np.linalg.norm(x) * np.linalg.norm(y)) < 1e-14 * s[0]
    assert np.all(s[1:] < 1e-14 * s[0])
    D = np.diag([3.0, 1.0, 2.0, 0.5])
    G, J, st, sw = oracle.jacobi_cols(D)
    assert st == 0 and sw == 1  # already orthogonal: first sweep rotates nothing
    assert np.array_equal(G, D)
    P = np.eye(6)[[3, 0, 5, 1, 4, 2]] * 2.5
    G, J, st, _ = oracle.jacobi_cols(P)
    assert np.allclose(np.linalg.norm(G, axis=0), 2.5, rtol=0, atol=1e-15)


def test_jacobi_against_lapack_and_invariants():
    rng = np.random.default_rng(4)
    M = rng.standard_normal((50, 30))
    G, J, st, _ = oracle.jacobi_cols(M)
    assert st == 0
    assert np.linalg.norm(J.T @ J - np.eye(30)) < 1e-13
    assert np.linalg.norm(M @ J - G) < 1e-13 * np.linalg.norm(M)
    gram = G.T @ G
    off = gram - np.diag(np.diag(gram))
    assert np.max(np.abs(off)) < 1e-13 * np.max(np.diag(gram))
    s = np.sort(np.linalg.norm(G, axis=0))[::-1]
    assert np.allclose(s, np.linalg.svd(M, compute_uv=False), rtol=1e-13, atol=0)


# ---------------------------------------------------------------- full SVD + truncation
@pytest.mark.parametrize("m,n", [(40, 40), (60, 25), (25, 60)])
def test_fullsvd_known_spectrum_and_eckart_young(m, n):
    r = min(m, n)
    s = wl.spectrum_exp(r, 0.3)
    A = wl.make_matrix(m, n, s, seed=5)
    k = r // 3
    res = oracle.fullsvd(A, k)
    assert res.status == 0 and res.k_kept == k
    assert np.max(np.abs(res.sig_all - s)) < 10 * r * EPS * s[0]
    # Eckart-Young-Mirsky: discarded weight is the tail sum and equals the error
    err2 = np.linalg.norm(A - (res.U * res.S) @ res.VT) ** 2
    assert abs(res.w - np.sum(s[k:] ** 2)) < 1e-12 * np.sum(s ** 2)
    assert abs(err2 - res.w) < 1e-12 * np.sum(s ** 2)
    assert np.linalg.norm(res.U.T @ res.U - np.eye(k)) < 1e-13
    assert np.linalg.norm(res.VT @ res.VT.T - np.eye(k)) < 1e-13
    # canonical signs: largest |entry| of each left vector is positive
    idx = np.argmax(np.abs(res.U), axis=0)
    assert np.all(res.U[idx, np.arange(k)] > 0)
    # against LAPACK gesdd (library routine independent of the oracle)
    Ul, sl, Vl = np.linalg.svd(A, full_matrices=False)
    assert np.allclose(res.sig_all, sl, rtol=0, atol=1e-13 * sl[0])
    for j in range(k):
        c = abs(res.U[:, j] @ Ul[:, j])
        assert abs(c - 1.0) < 1e-9


def test_truncation_rule_on_diagonal():
    s = np.array([4.0, 2.0, 1.0, 0.5, 0.25, 0.125])
    A = np.zeros((6, 6))
    A[np.arange(6), np.arange(6)] = s
    tot = np.sum(s ** 2)
    # smallest k' with tail(k') <= delta * ||A||^2
    for delta, expect in [(0.0, 5), (0.2, 2), (0.05, 3), (1.0, 1), (1e-12, 5)]:
        res = oracle.fullsvd(A, 5, delta)
        assert res.k_kept == expect, (delta, res.k_kept)
        assert res.w == pytest.approx(np.sum(s[expect:] ** 2), rel=1e-15)
        assert np.all(res.S[expect:] == 0) and np.all(res.U[:, expect:] == 0)
        assert res.w <= delta * tot or delta == 0.0 or expect == 5
    r = oracle.rsvd(A, 5, 1, 1, 3, 0.2)
    assert r.k_kept == 2 and r.w == pytest.approx(np.sum(s[2:] ** 2), rel=1e-13)


def test_zero_nan_and_invalid():
    Z = np.zeros((8, 5))
    for res in (oracle.fullsvd(Z, 3, 0.1), oracle.rsvd(Z, 3, 2, 1, 1, 0.1)):
        assert res.status == 0 and res.k_kept == 0 and res.w == 0.0
        assert np.all(res.U == 0) and np.all(res.S == 0) and np.all(res.VT == 0)
    X = np.ones((4, 4)); X[1, 2] = np.nan
    assert oracle.fullsvd(X, 2).status == oracle.ERR_NONFINITE
    assert oracle.rsvd(X, 2, 1, 1, 1).status == oracle.ERR_NONFINITE
    assert oracle.rsvd(np.ones((4, 4)), 2, 1, 1, 1, -1.0).status == oracle.ERR_INVALID
    assert oracle.rsvd(np.ones((4, 4)), 2, 1, 1, 1, float("nan")).status == oracle.ERR_INVALID
    assert oracle.rsvd(np.ones((4, 4)), 0, 1, 1, 1).status == oracle.ERR_INVALID


def test_jacobi_sweep_cap_reports_noconv():
    rng = np.random.default_rng(6)
    G, J, st, sw = oracle.jacobi_cols(rng.standard_normal((20, 12)), max_sweeps=1)
    assert st == oracle.ERR_NOCONV and sw == 1


# ---------------------------------------------------------------- RSVD
def test_rsvd_full_width_is_exact():
    """l = min(m, n): Q spans the range of A, so B = Q^T A has exactly the
    singular values of A (paper Sec. II.B, step 3 with A_l = A)."""
    s = wl.spectrum_exp(48, 0.08)
    A = wl.make_matrix(64, 48, s, seed=7)
    res = oracle.rsvd(A, 40, 20, 1, seed=11)
    assert res.l == 48 and res.status == 0
    assert np.max(np.abs(res.sig_all - s)) < 20 * 64 * EPS * s[0]


def test_rsvd_wide_matrix_full_width_is_exact():
    s = wl.spectrum_power(30, 1.0)
    A = wl.make_matrix(30, 70, s, seed=8)
    res = oracle.rsvd(A, 10, 40, 0, seed=12)
    assert res.l == 30
    assert np.max(np.abs(res.sig_all - s)) < 20 * 70 * EPS * s[0]


@pytest.mark.parametrize("m,n,k,p,q,gamma", [(128, 128, 64, 10, 2, None), (96, 140, 20, 8, 1, 1.5),
                                            (150, 90, 16, 6, 2, 1.2)])
def test_rsvd_invariants(m, n, k, p, q, gamma):
    r = min(m, n)
    s = wl.spectrum_exp(r, 0.08) if gamma is None else wl.spectrum_power(r, gamma)
    A = wl.make_matrix(m, n, s, seed=9)
    res = oracle.rsvd(A, k, p, q, seed=13)
    assert res.status == 0 and res.k_kept == k
    # interlacing: sigma~_j <= sigma_j (B = Q^T A is a compression of A)
    assert np.all(res.sig_all <= s[:res.l] * (1 + 1e-12) + 1e-15 * s[0])
    # exact isometries (paper: Q U~ and V~ are exact isometries)
    iso = 50 * res.l * EPS
    assert np.linalg.norm(res.U.T @ res.U - np.eye(k)) < iso
    assert np.linalg.norm(res.VT @ res.VT.T - np.eye(k)) < iso
    assert np.linalg.norm(res.Q.T @ res.Q - np.eye(res.l)) < iso
    # Pythagorean identity: ||A - U S V^T||_F^2 = ||A||^2 - sum sigma~^2 = w
    err2 = np.linalg.norm(A - (res.U * res.S) @ res.VT) ** 2
    tot = np.sum(s ** 2)
    assert abs(err2 - res.w) < 1e-11 * tot
    # never better than the optimum (Eckart-Young-Mirsky)
    assert err2 >= np.sum(s[k:] ** 2) * (1 - 1e-10)
    # U S V^T = Q Q^T A restricted to the top-k: U columns lie in span(Q)
    assert np.linalg.norm(res.U - res.Q @ (res.Q.T @ res.U)) < 1e-13


def test_rsvd_scaling_and_rotation_equivariance():
    s = wl.spectrum_power(60, 1.5)
    A = wl.make_matrix(80, 60, s, seed=10)
    r1 = oracle.rsvd(A, 12, 6, 2, seed=21)
    r2 = oracle.rsvd(2.0 * A, 12, 6, 2, seed=21)
    assert np.array_equal(r2.S, 2.0 * r1.S)
    assert np.array_equal(r2.U, r1.U) and np.array_equal(r2.VT, r1.VT)
    P = wl.haar_frame(np.random.default_rng(5), 80, 80)
    r3 = oracle.rsvd(P @ A, 12, 6, 2, seed=21)
    assert np.allclose(r3.S, r1.S, rtol=1e-12, atol=0)
    # left vectors rotate with P (up to the sign convention), right ones are kept
    for j in range(12):
        a = P @ r1.U[:, j]
        sgn = np.sign(a @ r3.U[:, j])
        assert np.linalg.norm(a - sgn * r3.U[:, j]) < 1e-9
        assert np.linalg.norm(r1.VT[j] - sgn * r3.VT[j]) < 1e-9


def test_rsvd_depends_on_seed_only_through_omega():
    s = wl.spectrum_power(50, 0.5)
    A = wl.make_matrix(50, 50, s, seed=14)
    a = oracle.rsvd(A, 8, 4, 0, seed=1)
    b = oracle.rsvd(A, 8, 4, 0, seed=1)
    c = oracle.rsvd(A, 8, 4, 0, seed=2)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.U, b.U)
    assert not np.array_equal(a.S, c.S)


def test_rsvd_power_iteration_improves_toward_optimum():
    """Each power step multiplies the emphasis by sigma^2 (Sec. II.B); the mean
    error over seeds decreases in q toward the Eckart-Young optimum."""
    s = wl.spectrum_power(120, 0.6)
    A = wl.make_matrix(120, 120, s, seed=15)
    k, p = 10, 5
    opt = math.sqrt(np.sum(s[k:] ** 2))
    means = []
    for q in range(4):
        errs = []
        for seed in range(8):
            r = oracle.rsvd(A, k, p, q, seed=100 + seed)
            errs.append(math.sqrt(r.w))
        means.append(np.mean(errs))
    assert all(means[i + 1] < means[i] for i in range(3))
    assert means[0] > 1.01 * opt
    assert means[3] < 1.01 * opt


def test_rsvd_hmt_frobenius_bound_q0():
    """Halko-Martinsson-Tropp Thm 10.5: E||A - QQ^T A||_F <= (1 + k/(p-1))^(1/2) tail_F."""
    s = wl.spectrum_power(80, 0.7)
    A = wl.make_matrix(100, 80, s, seed=16)
    k, p = 10, 4
    tail = math.sqrt(np.sum(s[k:] ** 2))
    errs = []
    for seed in range(32):
        r = oracle.rsvd(A, k, p, 0, seed=500 + seed)
        errs.append(np.linalg.norm(A - r.Q @ (r.Q.T @ A)))
    assert np.mean(errs) <= math.sqrt(1 + k / (p - 1)) * tail


@pytest.mark.parametrize("q", [1, 2])
def test_rsvd_hmt_spectral_bound_power(q):
    """Halko-Martinsson-Tropp Cor. 10.10 (power scheme, spectral norm)."""
    s = wl.spectrum_power(90, 0.5)
    A = wl.make_matrix(90, 90, s, seed=17)
    k, p = 8, 4
    e = 2 * q + 1
    bound = ((1 + math.sqrt(k / (p - 1))) * s[k] ** e
             + math.e * math.sqrt(k + p) / p * math.sqrt(np.sum(s[k:] ** (2 * e)))) ** (1.0 / e)
    errs = []
    for seed in range(32):
        r = oracle.rsvd(A, k, p, q, seed=900 + seed)
        errs.append(np.linalg.norm(A - r.Q @ (r.Q.T @ A), 2))
    assert np.mean(errs) <= bound


# ---------------------------------------------------------------- sector post-selection
def test_postselect_worked_example_with_ties():
    """Hand-ranked example: the value 3 appears in sectors 0 and 1; sector 2 is empty."""
    S = [np.array([5.0, 3.0, 1.0]), np.array([4.0, 3.0, 2.0]), np.array([7.0])]
    kk = [3, 3, 0]
    assert oracle.postselect(S, kk, 0) == [0, 0, 0]
    assert oracle.postselect(S, kk, 1) == [1, 0, 0]
    assert oracle.postselect(S, kk, 3) == [2, 1, 0]  # the tie at 3 goes to the lower sector
    assert oracle.postselect(S, kk, 4) == [2, 2, 0]
    assert oracle.postselect(S, kk, 5) == [2, 3, 0]
    assert oracle.postselect(S, kk, 100) == [3, 3, 0]


def test_postselect_block_diagonal_matches_svd_of_the_whole_matrix():
    """For a block-diagonal A the singular values are the union of the blocks'
    ones, so keeping the chi largest over the per-block full SVDs must keep
    exactly the chi largest singular values of A (LAPACK on the whole matrix),
    and the summed discarded weight must be the Eckart-Young error of the
    rank-chi truncation of A."""
    rng = np.random.default_rng(7)
    sizes = [(30, 24), (18, 40), (50, 50), (12, 9)]
    blocks = [rng.standard_normal((m, n)) * rng.uniform(0.2, 3.0) for m, n in sizes]
    A = np.zeros((sum(m for m, _ in sizes), sum(n for _, n in sizes)))
    r = c = 0
    for B, (m, n) in zip(blocks, sizes):
        A[r:r + m, c:c + n] = B
        r += m
        c += n
    chi = 40
    res = [oracle.fullsvd(B, min(B.shape)) for B in blocks]
    chi_s = oracle.postselect([x.S for x in res], [x.k_kept for x in res], chi)
    assert sum(chi_s) == chi
    kept = np.sort(np.concatenate([x.S[:cs] for x, cs in zip(res, chi_s)]))[::-1]
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(kept, ref[:chi], rtol=1e-12, atol=1e-12 * ref[0])
    w = sum(x.w + np.sum(x.S[cs:x.k_kept] ** 2) for x, cs in zip(res, chi_s))
    assert abs(w - np.sum(ref[chi:] ** 2)) <= 1e-10 * np.sum(A * A)


@pytest.mark.parametrize("seed", range(4))
def test_postselect_invariants_random(seed):
    """Count, dominance (every kept value >= every dropped one) and the prefix
    property, on random sorted spectra with deliberate cross-sector ties."""
    rng = np.random.default_rng(seed)
    nsec = int(rng.integers(1, 9))
    S, kk = [], []
    pool = rng.uniform(0.0, 1.0, 6)
    for _ in range(nsec):
        k = int(rng.integers(0, 12))
        v = np.sort(np.concatenate([rng.choice(pool, k // 2), rng.uniform(0, 1, k - k // 2)]))[::-1]
        S.append(np.concatenate([v, np.zeros(3)]))
        kk.append(int(rng.integers(0, k + 1)) if k else 0)
    total = sum(kk)
    for chi in range(0, total + 3):
        cs = oracle.postselect(S, kk, chi)
        assert sum(cs) == min(chi, total)
        assert all(0 <= c <= k for c, k in zip(cs, kk))
        kept = [S[b][j] for b in range(nsec) for j in range(cs[b])]
        dropped = [S[b][j] for b in range(nsec) for j in range(cs[b], kk[b])]
        if kept and dropped:
            assert min(kept) >= max(dropped)


# ---------------------------------------------------------------- adaptive rank
def test_adaptive_rank_exact_low_rank():
    """A of exact rank r: the cut binds at k_kept = r as soon as the sketch
    holds r directions, so the rank doubles from k0 until it first exceeds r,
    and the result reproduces A."""
    rng = np.random.default_rng(3)
    m, n, r = 90, 70, 21
    s = np.linspace(3.0, 1.0, r)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    A = (U * s) @ V.T
    for k0, expect in [(4, 4), (6, 3), (22, 1), (21, 2)]:  # 4 8 16 32 | 6 12 24 | 22 | 21 42
        res, att = oracle.rsvd_adaptive(A, k0, 70, 5, 1, 11, 1e-12)
        assert att == expect, (k0, att)
        assert res.k_kept == r
        assert np.allclose((res.U[:, :r] * res.S[:r]) @ res.VT[:r], A, atol=1e-12)


def test_adaptive_rank_meets_the_target_or_stops_at_the_cap():
    """Decaying spectrum: the final truncation meets w <= delta ||A||^2 when the
    cut binds; with a cap below the needed rank it stops at the cap."""
    A = wl.make_matrix(128, 100, np.exp(-0.08 * np.arange(1, 101)), 5)
    a2 = np.sum(A * A)
    res, att = oracle.rsvd_adaptive(A, 4, 100, 8, 2, 13, 1e-6)
    assert res.k_kept < min(128, 100) and res.w <= 1e-6 * a2 * (1 + 1e-9)
    assert att >= 2
    # the exact truncation needs more than 8 triplets for 1e-6: capped at 8
    res8, att8 = oracle.rsvd_adaptive(A, 4, 8, 8, 2, 13, 1e-6)
    assert res8.k_kept == 8 and res8.w > 1e-6 * a2 and att8 == 2
