"""Pins of the complex-valued oracle (oracle/complex.py) against what the
mathematics fixes: moments and layout of the circular Gaussian, the unique
QR with a real non-negative diagonal (against LAPACK through numpy), the
closed-form singular values of a 2 x 2 matrix, exactness of the RSVD when the
sketch spans the whole column space, Eckart-Young on matrices with known
spectra, invariance under a global phase and equivariance under a left
unitary, the truncation rule, the real case against the real C oracle, and
planted mistakes that these pins must catch."""
import cmath
import math
import os
import types

import numpy as np
import pytest

import oracle
import oracle.complex as oc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def crandn(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def haar_unitary_frame(rng, m, r):
    q, R = np.linalg.qr(crandn(rng, m, r))
    d = np.diag(R)
    return q * (d / np.abs(d))


def known(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U = haar_unitary_frame(rng, m, len(s))
    V = haar_unitary_frame(rng, n, len(s))
    return (U * s) @ V.conj().T


# ---------------------------------------------------------------- pins as functions of the module


def pin_gaussian(M):
    om = M.cgaussian(12345, 120, 40)
    assert om.shape == (120, 40) and om.dtype == np.complex128
    assert abs(np.mean(np.abs(om) ** 2) - 1.0) < 0.05
    assert abs(np.mean(om * om)) < 0.05  # circular: E w^2 = 0
    assert abs(np.var(om.real) - 0.5) < 0.04 and abs(np.var(om.imag) - 0.5) < 0.04
    assert abs(np.mean(om)) < 0.05
    big = M.cgaussian(12345, 123, 42)
    assert np.array_equal(big[:120, :40], om)  # entry (i, j) depends on (seed, i, j) only
    assert not np.allclose(M.cgaussian(12346, 120, 40), om)


def pin_qr(M):
    rng = np.random.default_rng(1)
    Y = crandn(rng, 30, 10)
    Q, R = M.chqr(Y)
    assert np.allclose(Q @ R, Y, atol=1e-13)
    assert np.allclose(Q.conj().T @ Q, np.eye(10), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0) and np.all(np.abs(np.diag(R).imag) < 1e-14)
    assert np.all(np.diag(R).real >= 0)
    q2, r2 = np.linalg.qr(Y)
    d = np.diag(r2) / np.abs(np.diag(r2))
    assert np.allclose(Q, q2 * d, atol=1e-12)  # the QR with diag(R) > 0 is unique


def pin_jacobi_2x2(M):
    rng = np.random.default_rng(2)
    for _ in range(5):
        A = crandn(rng, 2, 2)
        G, J, st, _ = M.cjacobi_cols(A)
        assert st == 0
        # sigma^2 are the eigenvalues of A^H A: tr/2 +- sqrt(tr^2/4 - |det A|^2)
        tr = float(np.sum(np.abs(A) ** 2))
        det2 = abs(A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]) ** 2
        disc = math.sqrt(tr * tr / 4 - det2)
        expect = sorted([math.sqrt(tr / 2 + disc), math.sqrt(max(tr / 2 - disc, 0.0))])
        got = sorted(np.linalg.norm(G, axis=0))
        assert np.allclose(got, expect, rtol=1e-12)
        assert abs(np.vdot(G[:, 0], G[:, 1])) < 1e-13 * tr
        assert np.allclose(A @ J, G, atol=1e-13)


def pin_rsvd_full_width(M):
    rng = np.random.default_rng(3)
    A = crandn(rng, 12, 9)
    r = M.crsvd(A, 6, 10, 1, 77)
    s = np.linalg.svd(A, compute_uv=False)
    assert r.status == 0 and r.l == 9 and r.k_kept == 6
    assert np.allclose(r.S, s[:6], rtol=1e-12)
    assert r.w == pytest.approx(float(np.sum(s[6:] ** 2)), rel=1e-10)
    u, ss, vh = np.linalg.svd(A)
    best = (u[:, :6] * ss[:6]) @ vh[:6]
    assert np.allclose((r.U * r.S) @ r.VT, best, atol=1e-12)


def pin_rsvd_known_spectrum(M):
    s = np.exp(-0.3 * np.arange(1, 41))
    A = known(60, 40, s, 4)
    r = M.crsvd(A, 10, 6, 2, 91)
    assert r.status == 0 and r.k_kept == 10
    assert np.allclose(r.S, s[:10], rtol=1e-6)
    tail = float(np.sum(s[10:] ** 2))
    assert tail * (1 - 1e-9) <= r.w <= tail * 1.0201  # Eckart-Young, and within 1 % in norm
    assert r.w == pytest.approx(float(np.sum(np.abs(A - (r.U * r.S) @ r.VT) ** 2)), rel=1e-9)
    assert np.allclose(r.U.conj().T @ r.U, np.eye(10), atol=1e-12)
    assert np.allclose(r.VT @ r.VT.conj().T, np.eye(10), atol=1e-12)
    big = np.argmax(np.abs(r.U), axis=0)
    lead = r.U[big, np.arange(10)]
    assert np.all(np.abs(lead.imag) < 1e-14) and np.all(lead.real > 0)  # canonical phases


def pin_phase_and_left_unitary(M):
    s = 0.9 ** np.arange(30)
    A = known(40, 30, s, 5)
    r0 = M.crsvd(A, 8, 5, 1, 13)
    # a global phase: Q -> e^{it} Q, so B = Q^H A is unchanged; the canonical U is
    # unchanged and the phase moves into the rows of VT
    r1 = M.crsvd(cmath.exp(0.7j) * A, 8, 5, 1, 13)
    assert np.allclose(r1.S, r0.S, rtol=1e-12)
    assert np.allclose(r1.U, r0.U, atol=1e-11) and np.allclose(r1.VT, cmath.exp(0.7j) * r0.VT, atol=1e-11)
    W = haar_unitary_frame(np.random.default_rng(6), 40, 40)
    r2 = M.crsvd(W @ A, 8, 5, 1, 13)  # Q -> W Q, the same B: U -> W U up to phases
    assert np.allclose(r2.S, r0.S, rtol=1e-11)
    ph = np.einsum("ij,ij->j", (W @ r0.U).conj(), r2.U)
    assert np.allclose(np.abs(ph), 1.0, atol=1e-10)
    assert np.allclose(r2.VT, r0.VT * ph.conj()[:, None], atol=1e-10)  # W A = (W U0 D) S (D^H VT0)


def pin_truncation_rule(M):
    s = np.array([1.0, 0.5, 0.25, 0.1, 0.01, 0.001])
    A = known(8, 6, s, 7)
    tail3 = float(np.sum(s[3:] ** 2))
    a2 = float(np.sum(s ** 2))
    r = M.crsvd(A, 5, 10, 0, 3, delta=tail3 / a2 * 1.0001)
    assert r.k_kept == 3 and r.w == pytest.approx(tail3, rel=1e-9)
    assert np.all(r.S[3:] == 0) and np.all(r.U[:, 3:] == 0) and np.all(r.VT[3:] == 0)
    z = M.crsvd(np.zeros((5, 4), dtype=complex), 2, 1, 1, 1)
    assert z.k_kept == 0 and z.w == 0.0
    # delta >= 1: w(1) <= ||A||^2 always holds, so the smallest k' >= 1 is 1
    for big in (1.0, 3.0):
        r1 = M.crsvd(A, 5, 10, 0, 3, delta=big)
        assert r1.k_kept == 1 and r1.w == pytest.approx(a2 - 1.0, rel=1e-9)
        f1 = M.cfullsvd(A, 5, delta=big)
        assert f1.k_kept == 1 and f1.w == pytest.approx(a2 - 1.0, rel=1e-9)
    bad = np.ones((4, 4), dtype=complex)
    bad[1, 2] = np.nan
    assert M.crsvd(bad, 2, 1, 1, 1).status == M.ERR_NONFINITE


def pin_fullsvd(M):
    rng = np.random.default_rng(8)
    for m, n in ((9, 14), (14, 9)):
        A = crandn(rng, m, n)
        r = M.cfullsvd(A, 5)
        s = np.linalg.svd(A, compute_uv=False)
        assert r.status == 0 and np.allclose(r.S, s[:5], rtol=1e-12)
        assert r.w == pytest.approx(float(np.sum(s[5:] ** 2)), rel=1e-10)
        u, ss, vh = np.linalg.svd(A)
        assert np.allclose((r.U * r.S) @ r.VT, (u[:, :5] * ss[:5]) @ vh[:5], atol=1e-12)


PINS = [pin_gaussian, pin_qr, pin_jacobi_2x2, pin_rsvd_full_width, pin_rsvd_known_spectrum,
        pin_phase_and_left_unitary, pin_truncation_rule, pin_fullsvd]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_complex_oracle_pin(pin):
    pin(oc)


def test_real_input_matches_the_real_oracle():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((11, 7))
    rc = oc.cfullsvd(A.astype(complex), 4)
    rr = oracle.fullsvd(A, 4)
    assert np.allclose(rc.S, rr.S, rtol=1e-12)
    assert rc.w == pytest.approx(rr.w, rel=1e-10)
    assert np.allclose(rc.U.imag, 0, atol=1e-13)  # canonical phases make a real SVD real


# ---------------------------------------------------------------- planted mistakes

MUTATIONS = {
    "cut_search_from_zero": ("for kp in range(1, kk + 1):", "for kp in range(0, kk + 1):"),
    "B_uses_plain_transpose": ("B = Q.conj().T @ A", "B = Q.T @ A"),
    "no_phase_alignment": ("y = M[:, j] * e.conjugate()", "y = M[:, j] * e"),
    "gaussian_variance_two": ("complex(r * math.cos(t), r * math.sin(t)) / math.sqrt(2.0)",
                              "complex(r * math.cos(t), r * math.sin(t))"),
    "power_step_skips_adjoint": ("Z, _ = chqr(A.conj().T @ Q)", "Z, _ = chqr(A.T @ Q)"),
    "qr_phase_not_fixed": ("return Q * d, d.conj()[:, None] * R", "return Q, R"),
    "canonical_phase_on_u_only": ("VT[j, :] = Vt_full[j, :] * ph", "VT[j, :] = Vt_full[j, :]"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name):
    src = open(os.path.join(ROOT, "oracle", "complex.py")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1
    mod = types.ModuleType("oracle.complex_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "complex_mutant.py", "exec"), mod.__dict__)
    failed = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except Exception:
            failed += 1
    assert failed > 0, f"no pin caught the planted mistake {name}"
