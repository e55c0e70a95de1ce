"""The oracle's pins are sensitive: each plausible mistake, planted in a copy
of the oracle on the CPU, makes at least one pin fail.

Every mutation below is a one-line change of the kind a transcription of the
method could contain: a flipped sign of the pair-term difference (Sec. 2,
Eq. Delta E_ij), the wall radius without the ion's radius (Sec. 5.2), the
contact distance of one ion instead of the additive one, a wrong Metropolis
exponent (Eq. trial-outcome), an off-centre displacement (Alg. 1), a dropped
Bjerrum length, a wrong Weyl constant or counter order of Philox4x32-10, and
the overlap tested on the old instead of the trial position (Sec. 3.3); in
the delayed-acceptance stage a shifted feature bin, a dropped ReLU,
bfloat16 rounding with ties away from zero and a conflict rule that looks at
the old position of the move only; in the g(r) normalisation (Sec. 5.2) the
density of the neighbours without their radius or with the centre counted
among them and the shell volume taken at the bin centre; and in T_c
(Sec. 5.2) a dropped -1/2 and a sum stopped at the first negative lag.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C, PY = "oracle/mc_oracle.c", "oracle/oracle.py"
MUTATIONS = [
    ("pair term sign", C,
     "s += q[j] * (1.0 / sqrt(d2t) - 1.0 / sqrt(d2));",
     "s += q[j] * (1.0 / sqrt(d2) - 1.0 / sqrt(d2t));"),
    ("wall radius", C, "double a = R - 0.5 * sigma;", "double a = R;"),
    ("contact distance", C, "double sij = 0.5 * (sigma[i] + sigma[j]);", "double sij = sigma[i];"),
    ("Metropolis exponent", C, "return dE <= 0.0 || u3 < exp(-dE);", "return dE <= 0.0 || u3 < exp(-0.5 * dE);"),
    ("displacement centre", C, "double t = u - 0.5;", "double t = u - 0.49;"),
    ("Bjerrum length dropped", C, "return lB * q[i] * s;", "return q[i] * s;"),
    ("Philox Weyl constant", C, "#define PHILOX_W1 0xBB67AE85u", "#define PHILOX_W1 0xBB67AE86u"),
    ("Philox counter order", C, "uint32_t ctr[4] = {i, sweep, chain, tag};",
     "uint32_t ctr[4] = {sweep, i, chain, tag};"),
    ("overlap on old position", C, "if (d2t < sij * sij) ov = 1;", "if (d2 < sij * sij) ov = 1;"),
    ("feature bin offset", C, "int32_t k = (int32_t)floor(sqrt(d2) / dr);", "int32_t k = (int32_t)ceil(sqrt(d2) / dr);"),
    ("second ReLU dropped", C, "h2[h] = bf16_round(z > 0.0 ? z : 0.0);", "h2[h] = bf16_round(z);"),
    ("bfloat16 ties away", C, "b += 0x7FFFu + ((b >> 16) & 1u);", "b += 0x8000u;"),
    ("conflict tested at the old position only", C,
     "conflict = within(xi, old + 3 * j, rc) || within(xi, tri + 3 * j, rc) ||\n"
     "                               within(xt, old + 3 * j, rc) || within(xt, tri + 3 * j, rc);",
     "conflict = within(xi, old + 3 * j, rc) || within(xi, tri + 3 * j, rc);"),
    ("g(r) density without the ion radius", PY,
     "vb = 4.0 / 3.0 * np.pi * (R - 0.5 * sigma_of_type[b]) ** 3", "vb = 4.0 / 3.0 * np.pi * R ** 3"),
    ("g(r) neighbour count with the centre", PY,
     "nb = (n_of_type[b] - (1 if a == b else 0)) / vb", "nb = n_of_type[b] / vb"),
    ("g(r) shell volume at the bin centre", PY,
     "vk = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)",
     "vk = 4.0 * np.pi * (0.5 * (edges[1:] + edges[:-1])) ** 2 * dr"),
    ("T_c without the -1/2", PY, "    tau = -0.5\n    for m in range(n // 2):", "    tau = 0.0\n    for m in range(n // 2):"),
    ("T_c stopped at the first negative lag", PY,
     "pair = c(2 * m) + c(2 * m + 1)", "pair = c(m + 1) if m else c(0) + c(1)"),
]


def _run_mutant(tmp_root, name, path, old, new):
    d = os.path.join(tmp_root, name.replace(" ", "_").replace("/", "_"))
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(d, "tests"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "paper_1602_05716_amd"), os.path.join(d, "paper_1602_05716_amd"),
                    ignore=shutil.ignore_patterns("*.so", "__pycache__", "valu_peak", "csrc"))
    src = os.path.join(d, path)
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
