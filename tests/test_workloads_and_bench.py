"""Host-side checks of the seeded input recipes and of the benchmark's
command line (no GPU): the synthetic matrices have exactly the spectra they
are built with, the workload definitions have the stated shapes and
parameters, and a multi-GPU request is refused before any device work."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("m,n", [(40, 40), (60, 25), (25, 60)])
def test_make_matrix_has_the_requested_spectrum_and_is_seeded(m, n):
    s = wl.spectrum_exp(min(m, n), 0.1)
    A = wl.make_matrix(m, n, s, 11)
    assert A.shape == (m, n)
    assert np.allclose(np.linalg.svd(A, compute_uv=False), s, rtol=1e-12, atol=1e-14)
    assert np.array_equal(A, wl.make_matrix(m, n, s, 11))
    assert not np.array_equal(A, wl.make_matrix(m, n, s, 12))


def test_haar_frame_is_orthonormal():
    F = wl.haar_frame(np.random.default_rng(3), 50, 20)
    assert np.allclose(F.T @ F, np.eye(20), atol=1e-13)


def test_spectra():
    assert np.allclose(wl.spectrum_power(4, 1.5), [1.0, 2 ** -1.5, 3 ** -1.5, 4 ** -1.5])
    s = wl.spectrum_power_with_pairs(200, 1.5)
    for i in (8, 40, 100):  # 1-based positions of the near-degenerate pairs
        assert s[i] / s[i - 1] == pytest.approx(1 - 1e-6, rel=1e-12)
    noisy = wl.spectrum_noisy_power(300, 1.2, 0.05, 7)
    assert np.all(np.diff(noisy) <= 0) and np.all(noisy > 0)


def test_workload_shapes_and_parameters():
    c1 = wl.c1().problems
    assert len(c1) == 1 and (c1[0].m, c1[0].n, c1[0].k, c1[0].p, c1[0].q, c1[0].l) == (128, 128, 64, 10, 2, 74)
    c2 = wl.c2().problems
    assert len(c2) == 32 and all((p.m, p.n, p.k, p.p, p.q, p.l) == (512, 512, 256, 16, 2, 272) for p in c2)
    assert len({p.seed for p in c2}) == 32 and len({p.a_seed for p in c2}) == 32
    c3 = wl.c3().problems
    assert len(c3) == 16 and all((p.m, p.k, p.q, p.l) == (1024, 64, 3, 80) for p in c3)
    c5 = wl.c5().problems
    assert len(c5) == 64 and all((p.m, p.n, p.k, p.l) == (1024, 1024, 128, 144) for p in c5)
    c4 = wl.c4().problems
    assert len(c4) == 512
    for p in c4:
        r = min(p.m, p.n)
        assert 32 <= p.m <= 2048 and 32 <= p.n <= 2048
        assert p.k % 8 == 0 and abs(p.k - r / 4) <= 4 and p.delta == 1e-10
        assert len(p.spectrum) == r
    # the algorithmic GEMM work of one C2 factorisation: 2 m n l (2 q + 2) + 2 m l k
    p = c2[0]
    assert p.gemm_flops() == 2.0 * 512 * 512 * 272 * 6 + 2.0 * 512 * 272 * 256


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_bench_help_lists_its_legs():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--no-tune", "--no-extra", "--no-cpu-baseline"):
        assert flag in r.stdout
