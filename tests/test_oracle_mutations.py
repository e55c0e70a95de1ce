"""The oracle's pins are sensitive: each plausible mistake, planted in a copy
of the oracle on the CPU, makes at least one pin fail.

Every mutation below is a one-line change of the kind a transcription of the
method could contain: a flipped sign of the pair-term difference (Sec. 2,
Eq. Delta E_ij), the wall radius without the ion's radius (Sec. 5.2), the
contact distance of one ion instead of the additive one, a wrong Metropolis
exponent (Eq. trial-outcome), an off-centre displacement (Alg. 1), a dropped
Bjerrum length, a wrong Weyl constant or counter order of Philox4x32-10, and
the overlap tested on the old instead of the trial position (Sec. 3.3); and
in the delayed-acceptance stage a shifted feature bin, a dropped ReLU and
bfloat16 rounding with ties away from zero.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("pair term sign",
     "s += q[j] * (1.0 / sqrt(d2t) - 1.0 / sqrt(d2));",
     "s += q[j] * (1.0 / sqrt(d2) - 1.0 / sqrt(d2t));"),
    ("wall radius", "double a = R - 0.5 * sigma;", "double a = R;"),
    ("contact distance", "double sij = 0.5 * (sigma[i] + sigma[j]);", "double sij = sigma[i];"),
    ("Metropolis exponent", "return dE <= 0.0 || u3 < exp(-dE);", "return dE <= 0.0 || u3 < exp(-0.5 * dE);"),
    ("displacement centre", "double t = u - 0.5;", "double t = u - 0.49;"),
    ("Bjerrum length dropped", "return lB * q[i] * s;", "return q[i] * s;"),
    ("Philox Weyl constant", "#define PHILOX_W1 0xBB67AE85u", "#define PHILOX_W1 0xBB67AE86u"),
    ("Philox counter order", "uint32_t ctr[4] = {i, sweep, chain, tag};", "uint32_t ctr[4] = {sweep, i, chain, tag};"),
    ("overlap on old position", "if (d2t < sij * sij) ov = 1;", "if (d2 < sij * sij) ov = 1;"),
    ("feature bin offset", "int32_t k = (int32_t)floor(sqrt(d2) / dr);", "int32_t k = (int32_t)ceil(sqrt(d2) / dr);"),
    ("second ReLU dropped", "h2[h] = bf16_round(z > 0.0 ? z : 0.0);", "h2[h] = bf16_round(z);"),
    ("bfloat16 ties away", "b += 0x7FFFu + ((b >> 16) & 1u);", "b += 0x8000u;"),
]


def _run_mutant(tmp_root, name, old, new):
    d = os.path.join(tmp_root, name.replace(" ", "_"))
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(d, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "paper_1602_05716_amd"), os.path.join(d, "paper_1602_05716_amd"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "valu_peak", "csrc"))
    src = os.path.join(d, "oracle", "mc_oracle.c")
    with open(src) as f:
        text = f.read()
    if text.count(old) != 1:
        return name, "not applied"
    with open(src, "w") as f:
        f.write(text.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "tests/test_oracle_da_pins.py",
                        "-x", "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu and not slow"],
                       cwd=d, capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1"))
    return name, ("caught" if r.returncode == 1 else "survived rc=%d" % r.returncode)


def test_each_planted_mistake_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda m: _run_mutant(str(tmp_path), *m), MUTATIONS))
    bad = [r for r in results if r[1] != "caught"]
    assert not bad, bad
