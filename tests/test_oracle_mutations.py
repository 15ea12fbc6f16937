"""The oracle's pins catch plausible mistakes in its arithmetic: each case
plants one (a flipped sign, a dropped factor, a transposed or shifted index)
in a scratch copy of the oracle's sources, builds it, and runs the CPU pin
tests against that copy, which must fail.  Only the copy is changed."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle.py", "tests/test_oracle_mac.py"]

# (file, original text, planted mistake, what it breaks)
MUTATIONS = [
    ("oracle.cpp", "ph += -cc.M * ri - 0.5 * s * ri5;", "ph += -cc.M * ri + 0.5 * s * ri5;",
     "sign of the quadrupole term of the particle-cell potential"),
    ("oracle.cpp", "ph += -cc.M * ri - 0.5 * s * ri5;", "ph += -cc.M * ri - 1.0 * s * ri5;",
     "factor of the quadrupole term of the particle-cell potential"),
    ("oracle.cpp", "2.5 * s * R0 * ri7", "1.5 * s * R0 * ri7",
     "factor of the quadrupole's radial acceleration term"),
    ("oracle.cpp", "double q1 = Q[3] * R0", "double q1 = Q[4] * R0",
     "index of an off-diagonal quadrupole component"),
    ("oracle.cpp", "ph -= t.m[j] * ri;", "ph += t.m[j] * ri;",
     "sign of the particle-particle potential"),
    ("oracle_mac.cpp", "2.0f * (q[3] * q[3] + q[4] * q[4] + q[5] * q[5])",
     "1.0f * (q[3] * q[3] + q[4] * q[4] + q[5] * q[5])",
     "off-diagonal weight of the quadrupole's Frobenius norm (feature 2)"),
    ("oracle_mac.cpp", "const float rg = 0.5f *", "const float rg = 1.0f *",
     "group half-diagonal (feature 3)"),
    ("oracle_mac.cpp", "f[1] = std::log10(Mc / Mtot) / 3.0f;", "f[1] = std::log10(Mc / Mtot);",
     "scaling of the mass feature (feature 1)"),
    ("oracle_mac.cpp", "const float dc = (float)cc.com[k] - geo[k];",
     "const float dc = (float)cc.com[k] - 0.5f * geo[k];",
     "centre offset (feature 11)"),
    ("oracle_mac.cpp", "P[oW1 + j * kIn + k]", "P[oW1 + (k * kH + j) % (kH * kIn)]",
     "transposed first-layer weights"),
    ("oracle_mac.cpp", "P[oW2 + j * kH + k]", "P[oW2 + k * kH + j]",
     "transposed second-layer weights"),
    ("oracle_mac.cpp", "s.a2[j] = a + P[oB2 + j];", "s.a2[j] = a + P[oB1 + j];",
     "second-layer bias read from the first layer's"),
]


@pytest.mark.slow
@pytest.mark.parametrize("fname,orig,bad,what", MUTATIONS, ids=[m[3] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, fname, orig, bad, what):
    from oracle import build_oracle
    src = os.path.join(ROOT, "oracle")
    for f in os.listdir(src):
        if f.endswith((".cpp", ".h")):
            shutil.copy(os.path.join(src, f), tmp_path / f)
    text = (tmp_path / fname).read_text()
    assert text.count(orig) >= 1, f"mutation site not found: {orig}"
    (tmp_path / fname).write_text(text.replace(orig, bad, 1))
    lib = str(tmp_path / "liboracle.so")
    build_oracle.build(src_dir=str(tmp_path), out=lib)
    env = dict(os.environ, OCTGRAV_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PINS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 1, f"the pins did not catch: {what}\n{r.stdout[-2000:]}"
