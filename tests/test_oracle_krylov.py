"""Pins of the block-Krylov oracle (oracle/krylov.py): with q = 0 it is the
oracle RSVD on the same Omega; when the Krylov space spans the whole column
space it is the exact truncated SVD; its subspace contains the RSVD's last
basis, so its discarded weight never exceeds the RSVD's for the same seed
and never beats Eckart-Young; the usual isometry and exact-weight
invariants; the truncation rule; planted mistakes."""
import os
import types

import numpy as np
import pytest

import oracle
import oracle.krylov as ok
import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def pin_q0_is_the_rsvd(M):
    A = wl.make_matrix(50, 40, wl.spectrum_power(40, 1.0), 21)
    r = M.block_krylov_rsvd(A, 8, 4, 0, 5)
    ref = oracle.rsvd(A, 8, 4, 0, 5)
    assert np.allclose(r.S, ref.S, rtol=1e-12)
    assert np.allclose(r.U, ref.U, atol=1e-10) and np.allclose(r.VT, ref.VT, atol=1e-10)
    assert r.w == pytest.approx(ref.w, rel=1e-10)


def pin_full_space_is_exact(M):
    A = np.random.default_rng(22).standard_normal((30, 18))
    r = M.block_krylov_rsvd(A, 5, 1, 2, 9)  # l = 6, L = min(18, 18): the whole row space
    s = np.linalg.svd(A, compute_uv=False)
    assert r.L == 18 and np.allclose(r.S, s[:5], rtol=1e-10)
    assert r.w == pytest.approx(float(np.sum(s[5:] ** 2)), rel=1e-9)


def pin_never_worse_than_rsvd(M):
    for seed in range(4):
        A = wl.make_matrix(120, 90, wl.spectrum_power(90, 0.6), 30 + seed)
        s = np.linalg.svd(A, compute_uv=False)
        tail = float(np.sum(s[10:] ** 2))
        for q in (1, 2):
            r = M.block_krylov_rsvd(A, 10, 2, q, 100 + seed)
            ref = oracle.rsvd(A, 10, 2, q, 100 + seed)
            assert tail * (1 - 1e-10) <= r.w <= ref.w * (1 + 1e-10)
            assert np.all(r.S <= s[:10] * (1 + 1e-12))  # interlacing: never above the exact values


def pin_invariants(M):
    A = wl.make_matrix(70, 50, wl.spectrum_exp(50, 0.1), 23)
    r = M.block_krylov_rsvd(A, 12, 3, 2, 8)
    assert r.status == 0 and r.k_kept == 12
    assert np.allclose(r.U.T @ r.U, np.eye(12), atol=1e-12)
    assert np.allclose(r.VT @ r.VT.T, np.eye(12), atol=1e-12)
    assert r.w == pytest.approx(float(np.sum((A - (r.U * r.S) @ r.VT) ** 2)), rel=1e-9)
    assert np.all(np.diff(r.S) <= 0)
    big = np.argmax(np.abs(r.U), axis=0)
    assert np.all(r.U[big, np.arange(12)] > 0)


def pin_truncation_rule(M):
    s = np.array([1.0, 0.5, 0.25, 0.1, 0.01, 0.001])
    A = wl.make_matrix(9, 6, s, 24)
    tail3 = float(np.sum(s[3:] ** 2))
    r = M.block_krylov_rsvd(A, 5, 1, 1, 2, delta=tail3 / float(np.sum(s ** 2)) * 1.0001)
    assert r.k_kept == 3 and r.w == pytest.approx(tail3, rel=1e-9)
    assert np.all(r.S[3:] == 0) and np.all(r.U[:, 3:] == 0)
    z = M.block_krylov_rsvd(np.zeros((6, 5)), 2, 1, 1, 1)
    assert z.k_kept == 0 and z.w == 0.0
    # delta >= 1: w(1) <= ||A||^2 always holds, so the smallest k' >= 1 is 1
    for big in (1.0, 3.0):
        r1 = M.block_krylov_rsvd(A, 5, 1, 1, 2, delta=big)
        assert r1.k_kept == 1 and r1.w == pytest.approx(float(np.sum(s[1:] ** 2)), rel=1e-9)


PINS = [pin_q0_is_the_rsvd, pin_full_space_is_exact, pin_never_worse_than_rsvd, pin_invariants,
        pin_truncation_rule]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_krylov_oracle_pin(pin):
    pin(ok)


def test_krylov_beats_rsvd_at_equal_passes_on_a_flat_spectrum():
    """The point of the variant: on a slowly decaying spectrum the Krylov space
    of q power steps gets closer to the optimum than the last basis alone."""
    A = wl.make_matrix(200, 150, wl.spectrum_power(150, 0.3), 40)
    s = np.linalg.svd(A, compute_uv=False)
    tail = float(np.sum(s[20:] ** 2))
    r = ok.block_krylov_rsvd(A, 20, 0, 2, 3)
    ref = oracle.rsvd(A, 20, 0, 2, 3)
    assert (r.w - tail) < 0.5 * (ref.w - tail)


MUTATIONS = {
    "cut_search_from_zero": ("for kp in range(1, kk + 1):", "for kp in range(0, kk + 1):"),
    "basis_from_last_block_only": ("Q, _ = hqr(np.concatenate(blocks, axis=1)[:, :L])", "Q = blocks[-1]"),
    "power_step_without_transpose": ("Z, _ = hqr(A.T @ Qj)", "Z, _ = hqr(A @ Qj)"),
    "weight_from_all_values": ("w = max(0.0, a2 - _ksum(sig[:k_kept] ** 2))", "w = max(0.0, a2 - _ksum(sig ** 2))"),
    "sign_on_u_only": ("VT[j] = sgn * Vt[j]", "VT[j] = Vt[j]"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name):
    src = open(os.path.join(ROOT, "oracle", "krylov.py")).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1
    mod = types.ModuleType("oracle.krylov_mutant")
    mod.__dict__["__package__"] = "oracle"
    exec(compile(src.replace(old, new), "krylov_mutant.py", "exec"), mod.__dict__)
    failed = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(mod)
        except Exception:
            failed += 1
    assert failed > 0, f"no pin caught the planted mistake {name}"
