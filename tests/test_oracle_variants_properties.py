"""Properties of the complex, block-Krylov and single-view oracles over random
small shapes (m < n and m > n, k clamped, p and q from 0): isometric factors,
descending singular values (bounded by the exact ones for the projection
methods), discarded weight equal to the squared Frobenius error and never
below the optimum."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle.complex as oc
import oracle.krylov as ok
import oracle.single_view as sv

shapes = st.tuples(st.integers(3, 24), st.integers(3, 24), st.integers(1, 30), st.integers(0, 6),
                   st.integers(0, 2), st.integers(0, 2 ** 32))


def check(A, r, k, projected=True):
    m, n = A.shape
    kk = min(k, m, n)
    s = np.linalg.svd(A, compute_uv=False)
    assert r.status == 0 and r.k_kept == kk and r.U.shape == (m, kk) and r.VT.shape == (kk, n)
    assert np.allclose(r.U.conj().T @ r.U, np.eye(kk), atol=1e-10)
    assert np.allclose(r.VT @ r.VT.conj().T, np.eye(kk), atol=1e-10)
    assert np.all(np.diff(r.S) <= 1e-12 * s[0])
    if projected:  # U S V^T is a truncation of Q Q^H A: its values interlace those of A
        assert np.all(r.S <= s[:kk] * (1 + 1e-10) + 1e-12)
    err = float(np.sum(np.abs(A - (r.U * r.S) @ r.VT) ** 2))
    assert abs(r.w - err) <= 1e-9 * float(np.sum(np.abs(A) ** 2))
    assert r.w >= float(np.sum(s[kk:] ** 2)) * (1 - 1e-9) - 1e-12


@settings(max_examples=25, deadline=None)
@given(shapes)
def test_complex_rsvd_properties(sh):
    m, n, k, p, q, seed = sh
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
    check(A, oc.crsvd(A, k, p, q, seed), k)


@settings(max_examples=25, deadline=None)
@given(shapes)
def test_block_krylov_properties(sh):
    m, n, k, p, q, seed = sh
    A = np.random.default_rng(seed).standard_normal((m, n))
    check(A, ok.block_krylov_rsvd(A, k, p, q, seed), k)


@settings(max_examples=25, deadline=None)
@given(shapes)
def test_single_view_properties(sh):
    m, n, k, p, _, seed = sh
    A = np.random.default_rng(seed).standard_normal((m, n))
    check(A, sv.single_view_rsvd(A, k, p, seed), k, projected=False)  # Q X is not a projection of A
