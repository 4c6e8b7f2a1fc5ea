"""Pins of the oracle's adjoints: central finite differences of the oracle's
forward (a separate code path), the RSVD gradient at l = min(m, n) against the
independently built full-SVD reference gradient, and a rotation-invariant loss
on a near-degenerate pair with broadening."""
import numpy as np
import pytest

import oracle
import workloads as wl


def loss(res, dU, dS, dVT):
    return np.sum(dU * res.U) + np.sum(dS * res.S) + np.sum(dVT * res.VT)


def fd_rsvd(A, k, p, q, seed, dU, dS, dVT, E, h):
    lp = loss(oracle.rsvd(A + h * E, k, p, q, seed), dU, dS, dVT)
    lm = loss(oracle.rsvd(A - h * E, k, p, q, seed), dU, dS, dVT)
    return (lp - lm) / (2 * h)


@pytest.mark.parametrize("m,n,k,p,q", [(24, 20, 4, 3, 1), (18, 30, 5, 4, 2), (30, 16, 6, 10, 0),
                                       (22, 22, 6, 2, 2)])
def test_rsvd_adjoint_matches_finite_differences(m, n, k, p, q):
    rng = np.random.default_rng(m * 100 + n)
    s = 0.5 ** (np.arange(min(m, n)) / 2.0)          # well separated, decaying
    A = wl.make_matrix(m, n, s, seed=m + n)
    dU, dS, dVT = rng.standard_normal((m, k)), rng.standard_normal(k), rng.standard_normal((k, n))
    dA = oracle.rsvd_backward(A, k, p, q, 9, dU, dS, dVT)
    for t in range(3):
        E = rng.standard_normal((m, n))
        E /= np.linalg.norm(E)
        fd = fd_rsvd(A, k, p, q, 9, dU, dS, dVT, E, 1e-6)
        an = np.sum(dA * E)
        assert abs(fd - an) <= 2e-6 * max(abs(fd), np.linalg.norm(dA)), (t, fd, an)


@pytest.mark.parametrize("m,n,k", [(20, 14, 5), (13, 21, 4)])
def test_fullsvd_adjoint_matches_finite_differences(m, n, k):
    rng = np.random.default_rng(7)
    s = 0.6 ** np.arange(min(m, n))
    A = wl.make_matrix(m, n, s, seed=3)
    dU, dS, dVT = rng.standard_normal((m, k)), rng.standard_normal(k), rng.standard_normal((k, n))
    dA = oracle.fullsvd_backward(A, k, dU, dS, dVT)
    E = rng.standard_normal((m, n))
    E /= np.linalg.norm(E)
    h = 1e-6
    fd = (loss(oracle.fullsvd(A + h * E, k), dU, dS, dVT) - loss(oracle.fullsvd(A - h * E, k), dU, dS, dVT)) / (2 * h)
    assert abs(fd - np.sum(dA * E)) <= 2e-6 * np.linalg.norm(dA)


@pytest.mark.parametrize("m,n,k,q", [(20, 14, 5, 1), (14, 20, 4, 2)])
def test_rsvd_at_full_width_has_the_full_svd_gradient(m, n, k, q):
    """With l = min(m, n) the RSVD is the exact truncated SVD, so its gradient
    through the QR and GEMM chain equals the SVD adjoint applied to A."""
    rng = np.random.default_rng(11)
    s = 0.7 ** np.arange(min(m, n))
    A = wl.make_matrix(m, n, s, seed=5)
    dU, dS, dVT = rng.standard_normal((m, k)), rng.standard_normal(k), rng.standard_normal((k, n))
    g1 = oracle.rsvd_backward(A, k, 50, q, 3, dU, dS, dVT)
    g2 = oracle.fullsvd_backward(A, k, dU, dS, dVT)
    assert np.linalg.norm(g1 - g2) <= 1e-9 * np.linalg.norm(g2)


def test_broadened_adjoint_on_near_degenerate_pair():
    """A loss that depends on the pair only through its projector is finite at
    degeneracy; the broadened adjoint matches its finite difference."""
    m = n = 16
    s = 0.7 ** np.arange(16)
    s[3] = s[2] * (1 - 1e-6)                         # near-degenerate pair (3rd, 4th)
    A = wl.make_matrix(m, n, s, seed=21)
    rng = np.random.default_rng(4)
    Gs = rng.standard_normal((m, m)); Gs = Gs + Gs.T
    Hs = rng.standard_normal((n, n)); Hs = Hs + Hs.T
    k = 6

    def proj_loss(A_):
        r = oracle.rsvd(A_, k, 10, 2, 1)
        Up, Vp = r.U[:, 2:4], r.VT[2:4].T
        return np.trace(Gs @ Up @ Up.T) + np.trace(Hs @ Vp @ Vp.T) + np.sum(r.S)

    r = oracle.rsvd(A, k, 10, 2, 1)
    dU = np.zeros((m, k)); dU[:, 2:4] = 2 * Gs @ r.U[:, 2:4]
    dVT = np.zeros((k, n)); dVT[2:4] = (2 * Hs @ r.VT[2:4].T).T
    dS = np.ones(k)
    dA = oracle.rsvd_backward(A, k, 10, 2, 1, dU, dS, dVT, broad=1e-12)
    E = rng.standard_normal((m, n)); E /= np.linalg.norm(E)
    h = 1e-9
    fd = (proj_loss(A + h * E) - proj_loss(A - h * E)) / (2 * h)
    assert abs(fd - np.sum(dA * E)) <= 1e-4 * np.linalg.norm(dA)


def test_broadening_vanishes_on_separated_spectra():
    m, n, k = 20, 18, 5
    A = wl.make_matrix(m, n, 0.6 ** np.arange(18), seed=8)
    rng = np.random.default_rng(2)
    cot = rng.standard_normal((m, k)), rng.standard_normal(k), rng.standard_normal((k, n))
    g0 = oracle.rsvd_backward(A, k, 6, 1, 2, *cot)
    g1 = oracle.rsvd_backward(A, k, 6, 1, 2, *cot, broad=1e-14)
    assert np.linalg.norm(g1 - g0) <= 1e-6 * np.linalg.norm(g0)
