"""The oracle's pins must be able to fail: plant plausible mistakes in copies
of the oracle (CPU only), load each copy in place of the real one, and check
that the pin suites reject it.  (Conventions with no external reference, such
as which Box-Muller normal goes to even rows, are fixed by the GPU/oracle
agreement of the generator tests instead.)"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    # forward
    "philox_multiplier": ("mult0 = 0xD2511F53u", "mult0 = 0xD2511F55u", "test_oracle.py"),
    "power_iteration_dropped": ("for (int64_t it = 0; it < q; ++it) {", "for (int64_t it = 0; it < 0; ++it) {",
                                "test_oracle.py"),
    "hqr_sign_fix_dropped": ("if (R[j * l + j] < 0.0) {", "if (R[j * l + j] < -1e300) {", "test_oracle.py"),
    "jacobi_rotation_sign": ("G[s * c + p] = cs * gp - sn * gq;", "G[s * c + p] = cs * gp + sn * gq;",
                             "test_oracle.py"),
    "rsvd_discarded_weight_off_by_one": ("if (w_out) *w_out = (normA2 == 0.0) ? 0.0 : wk[kkeep];\n\n",
                                         "if (w_out) *w_out = (normA2 == 0.0) ? 0.0 : wk[kkeep > 0 ? kkeep - 1 : 0];\n\n",
                                         "test_oracle.py"),
    "tsvd_tail_sum_off_by_one": ("tail[j] = orc_sum_val(&acc);", "tail[j] = orc_sum_val(&acc) - sj * sj;",
                                 "test_oracle.py"),
    # adjoints
    "qr_adjoint_copyltu_sign": ("S[i * l + j] = -((i >= j) ? C[i * l + j] : C[j * l + i]);",
                                "S[i * l + j] = ((i >= j) ? C[i * l + j] : C[j * l + i]);", "test_oracle_adjoint.py"),
    "svd_adjoint_projector_term_dropped": ("N[i * c + t] += inv * v;", "N[i * c + t] += 0.0 * v;",
                                           "test_oracle_adjoint.py"),
    "omega_term_dropped": ("mm(0, 1, m, n, l, Mb, l, X, l, 1.0, dA, n);         /* dA += Mb X^T */",
                           "if (s > 0) mm(0, 1, m, n, l, Mb, l, X, l, 1.0, dA, n);", "test_oracle_adjoint.py"),
    "svd_adjoint_ju_transposed": ("double ju = f * (EU[i * r + j] - EU[j * r + i]);",
                                  "double ju = f * (EU[j * r + i] - EU[i * r + j]);", "test_oracle_adjoint.py"),
}

RUNNER = """
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle
oracle._HERE = {here!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", {target!r}]))
"""


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_reject_planted_mistake(name, tmp_path):
    old, new, target = MUTATIONS[name]
    src = open(SRC).read()
    assert old in src, f"mutation site of {name} not found"
    here = str(tmp_path)
    with open(os.path.join(here, "oracle.c"), "w") as f:
        f.write(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fno-fast-math",
                           "-ffp-contract=off", os.path.join(here, "oracle.c"), "-o",
                           os.path.join(here, "liboracle.so"), "-lm"])
    # keep the copy newer than its source so the loader does not rebuild
    os.utime(os.path.join(here, "liboracle.so"))
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), here=here,
                         target=os.path.join(ROOT, "tests", target))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"pins did not catch {name}:\n{r.stdout[-500:]}"
