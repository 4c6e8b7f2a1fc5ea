"""Pins of the single-view oracle (oracle/single_view.py): exact on matrices
of rank at most l; never better than the two-pass RSVD with the same range
sketch (both approximations live in span Q, and the two-pass one is the best
there) and never better than Eckart-Young; the expected error of Q X over the
co-range sketch equals (1 + l / (s - l - 1)) times the error of Q Q^T A
(Gaussian Psi); Psi independent of Omega; invariants; truncation rule;
planted mistakes."""
import os
import types

import numpy as np
import pytest

import oracle
import oracle.single_view as sv
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def pin_exact_on_low_rank(M):
    s = np.array([3.0, 2.0, 1.0, 0.5, 0.25])
    A = wl.make_matrix(40, 30, s, 51)  # rank 5 <= l = 8
    r = M.single_view_rsvd(A, 4, 4, 7)
    assert np.allclose(r.S, s[:4], rtol=1e-10)
    assert np.allclose(r.QX, A, atol=1e-11)
    assert r.w == pytest.approx(0.25 ** 2, rel=1e-8)


def pin_bounded_by_two_pass_and_optimum(M):
    for seed in range(4):
        A = wl.make_matrix(80, 60, wl.spectrum_power(60, 1.0), 60 + seed)
        sv_all = np.linalg.svd(A, compute_uv=False)
        r = M.single_view_rsvd(A, 10, 5, 200 + seed)
        ref = oracle.rsvd(A, 10, 5, 0, 200 + seed)  # the same Omega
        assert r.w >= ref.w * (1 - 1e-9) >= float(np.sum(sv_all[10:] ** 2)) * (1 - 1e-9)


def pin_expected_error_over_psi(M):
    A = wl.make_matrix(90, 70, wl.spectrum_power(70, 0.5), 61)
    num = den = 0.0
    for seed in range(48):
        r = M.single_view_rsvd(A, 6, 4, 300 + seed)
        num += float(np.sum((A - r.QX) ** 2))
        den += float(np.sum((A - r.Q @ (r.Q.T @ A)) ** 2))
    l, s = 10, 21
    assert num / den == pytest.approx(1 + l / (s - l - 1), rel=0.12)


def pin_independent_sketches(M):
    A = np.ones((60, 50))
    r = M.single_view_rsvd(A, 10, 10, 17)
    assert r.Psi.shape == (41, 60) and r.Omega.shape == (50, 20)
    overlap = r.Psi.T[:50, :20]  # the entries a shared Philox key would make equal to Omega
    c = np.corrcoef(overlap.ravel(), r.Omega.ravel())[0, 1]
    assert abs(c) < 0.1
    assert abs(np.mean(r.Psi ** 2) - 1.0) < 0.1 and abs(np.mean(r.Psi)) < 0.05


def pin_invariants(M):
    A = wl.make_matrix(60, 45, wl.spectrum_exp(45, 0.2), 62)
    r = M.single_view_rsvd(A, 8, 6, 11)
    assert r.status == 0 and r.k_kept == 8 and r.s == 29
    assert np.allclose(r.U.T @ r.U, np.eye(8), atol=1e-12)
    assert np.allclose(r.VT @ r.VT.T, np.eye(8), atol=1e-12)
    assert np.all(np.diff(r.S) <= 0)
    assert np.all(r.U[np.argmax(np.abs(r.U), axis=0), np.arange(8)] > 0)


def pin_truncation_rule(M):
    s = np.array([1.0, 0.5, 0.25, 0.1, 0.01])
    A = wl.make_matrix(12, 9, s, 63)  # rank 5 <= l: exact, so the errors are the tails
    tail3 = float(np.sum(s[3:] ** 2))
    r = M.single_view_rsvd(A, 5, 3, 4, delta=tail3 / float(np.sum(s ** 2)) * 1.0001)
    assert r.k_kept == 3 and r.w == pytest.approx(tail3, rel=1e-8)
    assert np.all(r.S[3:] == 0) and np.all(r.VT[3:] == 0)
    z = M.single_view_rsvd(np.zeros((7, 6)), 2, 1, 1)
    assert z.k_kept == 0 and z.w == 0.0
    # delta >= 1: w(1) <= ||A||^2 always holds, so the smallest k' >= 1 is 1
    for big in (1.0, 3.0):
        r1 = M.single_view_rsvd(A, 5, 3, 4, delta=big)
        assert r1.k_kept == 1 and r1.w == pytest.approx(float(np.sum(s[1:] ** 2)), rel=1e-8)


PINS = [pin_exact_on_low_rank, pin_bounded_by_two_pass_and_optimum, pin_expected_error_over_psi,
        pin_independent_sketches, pin_invariants, pin_truncation_rule]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_single_view_oracle_pin(pin):
    pin(sv)


MUTATIONS = {
    "cut_search_from_zero": ("for kp in range(1, kk + 1):", "for kp in range(0, kk + 1):"),
    "psi_shares_omega_key": ("Psi = gaussian(seed ^ (1 << 63), m, s).T", "Psi = gaussian(seed, m, s).T"),
    "x_without_psi_q_inverse": ("X = np.linalg.solve(R2, Q2.T @ W)", "X = Q2.T @ W"),
    "co_range_too_narrow": ("s = min(2 * l + 1, m)", "s = min(l + 2, m)"),
    "sign_on_u_only": ("            Vt[j] *= -1.0\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name):
    src = open(os.path.join(ROOT, "oracle", "single_view.py")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1
    mod = types.ModuleType("oracle.single_view_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "single_view_mutant.py", "exec"), mod.__dict__)
    failed = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except Exception:
            failed += 1
    assert failed > 0, f"no pin caught the planted mistake {name}"
