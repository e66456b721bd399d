"""The erfcx polynomial of the Ewald kernel: the committed include equals
what its generator writes, and erf(z) = 1 - exp(-z^2) * poly(2/z) matches
the error function to double precision over the range it serves."""
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_08621_amd", "csrc")


def _parse(text):
    scale = float(re.search(r"kErfcxScale = ([^;]+);", text).group(1))
    shift = float(re.search(r"kErfcxShift = ([^;]+);", text).group(1))
    body = text[text.index("c_erfcx"):]
    coef = [float(v) for v in re.findall(r"^\s+([-+0-9.e]+),", body, flags=re.M)]
    return scale, shift, coef


def test_include_is_what_the_generator_writes(tmp_path):
    pytest.importorskip("scipy")
    src = os.path.join(CSRC, "gen_erfcx.py")
    work = tmp_path / "csrc"
    work.mkdir()
    (work / "gen_erfcx.py").write_text(open(src).read())
    subprocess.check_call([sys.executable, str(work / "gen_erfcx.py")], cwd=work,
                          stdout=subprocess.DEVNULL)
    assert (work / "erfcx_poly.inc").read_text() == open(os.path.join(CSRC, "erfcx_poly.inc")).read()


def test_erf_from_the_polynomial_is_double_accurate():
    scale, shift, coef = _parse(open(os.path.join(CSRC, "erfcx_poly.inc")).read())
    assert len(coef) == 19
    for z in np.linspace(math.sqrt(2.0), 6.5, 4001):
        t = 2.0 / z * scale + shift
        h = 0.0
        for c in reversed(coef):
            h = h * t + c
        # math.erf / math.erfc are the C library's, independent of the fit
        assert abs((1.0 - math.exp(-z * z) * h) - math.erf(z)) < 4e-16
        assert abs(math.exp(-z * z) * h - math.erfc(z)) < 2e-16 + 1e-13 * math.erfc(z)
