"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs and the same Gaussian test matrix."""
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return P


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().double().numpy()


def sigma_tol_f64(s_ref):
    """FP64 bar: |d sigma_i| <= 1e-10 sigma_i where sigma_i >= 1e-5 sigma_1,
    else <= 1e-15 sigma_1 (exponential tails reach far below)."""
    s1 = s_ref[0] if len(s_ref) else 0.0
    return np.where(s_ref >= 1e-5 * s1, 1e-10 * s_ref, 1e-15 * s1)


def align_and_compare(U, VT, Ur, VTr, S_ref, tol):
    """Compare singular vectors up to sign, only where the value is separated
    from its neighbours by a relative gap > 1e-6."""
    k = len(S_ref)
    for j in range(k):
        gap_lo = abs(S_ref[j] - S_ref[j + 1]) / S_ref[0] if j + 1 < k else 1.0
        gap_hi = abs(S_ref[j - 1] - S_ref[j]) / S_ref[0] if j > 0 else 1.0
        if min(gap_lo, gap_hi) < 1e-6 or S_ref[j] < 1e-8 * S_ref[0]:
            continue
        sgn = np.sign(U[:, j] @ Ur[:, j]) or 1.0
        assert np.max(np.abs(sgn * U[:, j] - Ur[:, j])) < tol, (j, "U")
        assert np.max(np.abs(sgn * VT[j] - VTr[j])) < tol, (j, "VT")


# ---------------------------------------------------------------- generator
def test_philox_device_known_answers(lib):
    from conftest import load_kat
    from paper_1710_01463_amd.rsvd import philox4x32_10
    rows = load_kat()
    words = np.array([list(c) + list(k) for c, k, _ in rows], dtype=np.uint32)
    out = philox4x32_10(words)
    for r, (_, _, expect) in zip(out, rows):
        assert tuple(int(x) for x in r) == expect


def test_philox_device_matches_oracle_words(lib):
    from paper_1710_01463_amd.rsvd import philox4x32_10
    rng = np.random.default_rng(0)
    words = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64).astype(np.uint32)
    out = philox4x32_10(words)
    for i in range(0, 300, 7):
        ref = oracle.philox4x32_10(words[i, :4], words[i, 4:])
        assert np.array_equal(out[i], ref)


@pytest.mark.parametrize("seed,n,l", [(0, 1, 1), (2001, 128, 74), ((1 << 40) + 7, 301, 33)])
def test_gaussian_matches_oracle(lib, seed, n, l):
    from paper_1710_01463_amd.rsvd import gaussian
    g = host(gaussian(seed, n, l))
    r = oracle.gaussian(seed, n, l)
    # same Philox words; log/sqrt/sin/cos from two math libraries: a few ulp
    assert np.max(np.abs(g - r) / np.maximum(np.abs(r), 1e-300)) < 64 * EPS or \
        np.max(np.abs(g - r)) < 16 * EPS * np.max(np.abs(r))


# ---------------------------------------------------------------- RSVD FP64 parity
CASES = [
    # m, n, k, p, q, spectrum, seed
    (128, 128, 64, 10, 2, "exp0.08", 2001),      # the C1 workload
    (96, 80, 20, 8, 2, "pow1.5", 11),
    (200, 150, 40, 10, 1, "pow1.2", 12),         # l = 50: ragged tiles and blocks
    (64, 300, 16, 10, 2, "exp0.2", 13),          # wide
    (300, 45, 30, 5, 0, "pow1.0", 14),           # tall, q = 0
    (37, 53, 70, 4, 1, "exp0.1", 15),            # k > min(m, n): clamped, l = min(m, n)
    (1, 7, 1, 0, 1, "exp0.1", 16),               # single row
    (260, 33, 9, 3, 3, "pow2.0", 17),
]


def spectrum(name, r):
    kind, v = name[:3], float(name[3:])
    return wl.spectrum_exp(r, v) if kind == "exp" else wl.spectrum_power(r, v)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}k{c[2]}p{c[3]}q{c[4]}")
def test_rsvd_f64_matches_oracle(lib, case):
    m, n, k, p, q, spec, seed = case
    s = spectrum(spec, min(m, n))
    A = wl.make_matrix(m, n, s, seed=seed + 100)
    ref = oracle.rsvd(A, k, p, q, seed)
    assert ref.status == 0
    U, S, VT, w, kk = lib.rsvd_truncate(dev(A), k, p, q, seed, 0.0, "f64")
    U, S, VT, w, kk = host(U), host(S), host(VT), host(w)[0], int(host(kk)[0])
    assert kk == ref.k_kept
    assert np.all(np.abs(S - ref.S) <= sigma_tol_f64(ref.S))
    assert abs(w - ref.w) <= 1e-10 * max(ref.w, 1e-300) + 1e-13 * np.sum(s ** 2)
    align_and_compare(U, VT, ref.U, ref.VT, ref.S, 1e-8)
    # isometries
    kk2 = len(S)
    assert np.linalg.norm(U.T @ U - np.eye(kk2)) < 100 * max(m, n) * EPS
    assert np.linalg.norm(VT @ VT.T - np.eye(kk2)) < 100 * max(m, n) * EPS


def test_rsvd_f32_storage_f64_arith(lib):
    m, n, k = 150, 120, 30
    A = wl.make_matrix(m, n, wl.spectrum_power(120, 1.5), seed=21).astype(np.float32)
    ref = oracle.rsvd(A.astype(np.float64), k, 10, 2, 5)
    U, S, VT, w, kk = lib.rsvd_truncate(dev(A, torch.float32), k, 10, 2, 5, 0.0, "f64")
    S = host(S)
    # FP64 arithmetic on the exact FP32 values; outputs rounded to FP32
    assert np.all(np.abs(S - ref.S) <= 4e-7 * ref.S[0])


def test_rsvd_delta_cut_and_weight(lib):
    m, n = 180, 160
    s = wl.spectrum_exp(160, 0.1)
    A = wl.make_matrix(m, n, s, seed=31)
    for delta in (1e-4, 1e-8, 1e-10):
        ref = oracle.rsvd(A, 120, 16, 2, 7, delta)
        U, S, VT, w, kk = lib.rsvd_truncate(dev(A), 120, 16, 2, 7, delta, "f64")
        kk = int(host(kk)[0])
        rel = ref.w / np.sum(s ** 2)
        # the cut is an integer decided by FP64 on both sides: equal unless at the boundary
        assert kk == ref.k_kept or abs(rel - delta) < 1e-12
        S = host(S)
        assert np.all(S[kk:] == 0)
        assert np.all(host(U)[:, kk:] == 0) and np.all(host(VT)[kk:] == 0)


def test_rsvd_full_width_exact(lib):
    s = wl.spectrum_exp(48, 0.08)
    A = wl.make_matrix(64, 48, s, seed=41)
    U, S, VT, w, kk = lib.rsvd_truncate(dev(A), 40, 20, 1, 3, 0.0, "f64")
    assert np.max(np.abs(host(S) - s[:40])) < 20 * 64 * EPS * s[0]


def test_zero_and_nonfinite(lib):
    from paper_1710_01463_amd._lib import RsvdError
    Z = torch.zeros((40, 30), dtype=torch.float64, device="cuda")
    U, S, VT, w, kk = lib.rsvd_truncate(Z, 5, 4, 1, 1, 0.1)
    assert int(host(kk)[0]) == 0 and host(w)[0] == 0.0
    assert np.all(host(U) == 0) and np.all(host(S) == 0) and np.all(host(VT) == 0)
    X = torch.ones((40, 30), dtype=torch.float64, device="cuda")
    X[3, 4] = float("nan")
    with pytest.raises(RsvdError) as e:
        lib.rsvd_truncate(X, 5, 4, 1, 1)
    assert e.value.status == -4
    with pytest.raises(RsvdError) as e:
        lib.rsvd_truncate(Z, 5, -1, 1, 1)
    assert e.value.status == -1


# ---------------------------------------------------------------- full SVD
# 300^2, 512 x 280 and 280 x 512 have 19 and 18 row blocks of 16: from 16 blocks
# on the Jacobi rounds 2.. of a sweep rotate only the cross-block row pairs,
# the schedule the benchmark's 500^2 and 512^2 full SVDs run.  300 x 600 (and
# its transpose) has Jacobi rows of 600 columns and 300 rows of P, more than
# the register-resident variants hold, so its pairs stream their column
# chunks; 200 x 900 takes the variant with eight column chunks resident.
@pytest.mark.parametrize("m,n,k", [(64, 64, 20), (100, 37, 30), (37, 100, 30), (150, 150, 150), (5, 3, 2),
                                   (300, 300, 120), (512, 280, 280), (280, 512, 200), (300, 600, 150),
                                   (600, 300, 150), (200, 900, 100)])
def test_fullsvd_matches_oracle(lib, m, n, k):
    s = wl.spectrum_power(min(m, n), 1.0)
    A = wl.make_matrix(m, n, s, seed=51)
    ref = oracle.fullsvd(A, k)
    U, S, VT, w, kk = lib.fullsvd_truncate(dev(A), k)
    S = host(S)
    assert int(host(kk)[0]) == ref.k_kept
    assert np.max(np.abs(S - ref.S)) <= 1e-13 * s[0] * max(m, n)
    assert np.max(np.abs(S - s[:len(S)])) <= 1e-13 * s[0] * max(m, n)
    assert abs(host(w)[0] - ref.w) <= 1e-12 * np.sum(s ** 2)
    align_and_compare(host(U), host(VT), ref.U, ref.VT, ref.S, 1e-8)


# ---------------------------------------------------------------- batching
def test_plan_batch_equals_one_at_a_time(lib):
    probs, mats = [], []
    shapes = [(100, 80, 20), (40, 200, 12), (257, 130, 33), (64, 64, 64), (33, 17, 5)]
    for i, (m, n, k) in enumerate(shapes):
        s = wl.spectrum_exp(min(m, n), 0.05 + 0.02 * i)
        mats.append(wl.make_matrix(m, n, s, seed=60 + i))
        probs.append(dict(m=m, n=n, k=k, p=8, q=2, seed=70 + i))
    plan = lib.Plan(probs, torch.float64, "f64")
    outs, w, kk, info = plan.execute([dev(A) for A in mats])
    torch.cuda.synchronize()
    for i, (A, pr) in enumerate(zip(mats, probs)):
        U1, S1, VT1, w1, k1 = lib.rsvd_truncate(dev(A), pr["k"], pr["p"], pr["q"], pr["seed"])
        assert np.array_equal(host(outs[i][1]), host(S1))
        assert np.array_equal(host(outs[i][0]), host(U1))
        assert np.array_equal(host(outs[i][2]), host(VT1))
        assert host(w)[i] == host(w1)[0]
        assert int(host(info)[i]) == 0


def test_graph_replays_are_identical(lib):
    m, n = 120, 90
    A = dev(wl.make_matrix(m, n, wl.spectrum_power(90, 1.0), seed=81))
    plan = lib.Plan([dict(m=m, n=n, k=20, p=10, q=2, seed=3)], torch.float64, "f64", graph=True)
    first = None
    for rep in range(4):
        outs, w, kk, info = plan.execute([A])
        S = host(outs[0][1]).copy()
        _ = torch.randn(1000, device="cuda").sum()  # eager work between replays
        if first is None:
            first = S
        assert np.array_equal(S, first)
    ref = oracle.rsvd(host(A), 20, 10, 2, 3)
    assert np.all(np.abs(first - ref.S) <= sigma_tol_f64(ref.S))


def test_persistent_jacobi_equals_round_launches(lib):
    """Small plans run the Jacobi phase as one persistent launch; the same plan
    with one launch per round must give bit-identical outputs (same rotations
    in the same order per problem), for the RSVD, the triangular-factor path,
    FP32 storage and the full SVD."""
    shapes = [(100, 80, 20, 8, 2), (40, 200, 12, 6, 1), (130, 257, 33, 8, 2), (64, 64, 64, 0, 1), (33, 17, 5, 3, 0),
              (90, 700, 24, 8, 2),  # the triangular-factor path (n >= 2 l)
              (300, 600, 150, 8, 1)]  # full SVD: 600-column rows and 300 rows of P, the streaming Jacobi variant
    # exp(-a i) spectra; the last one gentle (sigma_300 / sigma_1 = 2.5e-3): with
    # singular values far below the FP64 floor the full SVD's one-sided Jacobi
    # needs more sweeps than the plan's cap (the oracle takes 42 at a = 0.16)
    decay = [0.04 + 0.02 * i for i in range(6)] + [0.02]
    mats = [wl.make_matrix(m, n, wl.spectrum_exp(min(m, n), decay[i]), seed=90 + i)
            for i, (m, n, _, _, _) in enumerate(shapes)]
    probs = [dict(m=m, n=n, k=k, p=p, q=q, seed=95 + i) for i, (m, n, k, p, q) in enumerate(shapes)]
    for dtype, full in ((torch.float64, False), (torch.float32, False), (torch.float64, True)):
        As = [dev(A, dtype) for A in mats]
        pl = [dict(m=pr["m"], n=pr["n"], k=pr["k"]) for pr in probs] if full else probs
        res = []
        for rl in (False, True):
            plan = lib.Plan(pl, dtype, "f64", fullsvd=full, graph=True, round_launches=rl)
            outs, w, kk, info = plan.execute(As)
            torch.cuda.synchronize()
            assert int(info.abs().sum()) == 0
            res.append(([t.clone() for o in outs for t in o], w.clone(), kk.clone()))
            plan.close()
        (a, wa, ka), (b, wb, kb) = res
        assert all(torch.equal(x, y) for x, y in zip(a, b)) and torch.equal(wa, wb) and torch.equal(ka, kb), (dtype, full)


def test_qr_kernel_classes_in_one_batch(lib):
    """One plan whose sketch widths straddle the register-resident Cholesky and
    substitution (l <= 288) and the general kernels (l > 288), so every
    orthonormalisation launches both kernel classes, each skipping the other's
    problems: l = 288, 289, 320, and 50 (the last with n >= 2 l, so its small
    SVD also runs the triangular-factor Cholesky QR).  Every problem against
    the oracle at the FP64 bars."""
    shapes = [(360, 330, 272, 16), (330, 400, 273, 16), (400, 352, 304, 16), (200, 180, 40, 10)]
    mats, probs = [], []
    for b, (m, n, k, p) in enumerate(shapes):
        mats.append(wl.make_matrix(m, n, wl.spectrum_power(min(m, n), 1.5), seed=880 + b))
        probs.append(dict(m=m, n=n, k=k, p=p, q=2, seed=890 + b))
    assert [min(pr["k"] + pr["p"], pr["m"], pr["n"]) for pr in probs] == [288, 289, 320, 50]
    plan = lib.Plan(probs, torch.float64, "f64", graph=True)
    outs, w, kk, info = plan.execute([dev(A) for A in mats])
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    w, kk = w.cpu().numpy(), kk.cpu().numpy()
    for b, (A, pr) in enumerate(zip(mats, probs)):
        ref = oracle.rsvd(A, pr["k"], pr["p"], pr["q"], pr["seed"])
        U, S, VT = host(outs[b][0]), host(outs[b][1]), host(outs[b][2])
        assert kk[b] == ref.k_kept, b
        assert np.all(np.abs(S - ref.S) <= sigma_tol_f64(ref.S)), b
        assert abs(w[b] - ref.w) <= 1e-10 * max(ref.w, 1e-300) + 1e-13 * np.sum(A * A), b
        align_and_compare(U, VT, ref.U, ref.VT, ref.S, 1e-8)
        kk2 = len(S)
        assert np.linalg.norm(U.T @ U - np.eye(kk2)) < 100 * max(A.shape) * EPS, b
        assert np.linalg.norm(VT @ VT.T - np.eye(kk2)) < 100 * max(A.shape) * EPS, b
    plan.close()
