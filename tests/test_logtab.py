"""The committed logarithm table (csrc/logtab.h) is what its generator
writes, and its entries are what they claim: 1/c_j rounded from j/128, and
head + tail of -log of that double to well below a double's resolution."""
import os
import re
import subprocess
import sys
from decimal import Decimal, getcontext

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1803_07772_amd", "csrc")


def _rows(text):
    return [tuple(float.fromhex(v) for v in m.groups())
            for m in re.finditer(r"\{(-?0x[0-9a-fp.+-]+), (-?0x[0-9a-fp.+-]+), (-?0x[0-9a-fp.+-]+)\}", text)]


def test_generator_reproduces_committed_table(tmp_path):
    committed = open(os.path.join(CSRC, "logtab.h")).read()
    gen = open(os.path.join(CSRC, "gen_logtab.py")).read()
    # run the generator against a copy so the committed file is untouched
    work = tmp_path / "csrc"
    work.mkdir()
    (work / "gen_logtab.py").write_text(gen)
    subprocess.run([sys.executable, str(work / "gen_logtab.py")], check=True, capture_output=True)
    assert (work / "logtab.h").read_text() == committed


def test_entries():
    rows = _rows(open(os.path.join(CSRC, "logtab.h")).read())
    assert len(rows) == 91
    getcontext().prec = 50
    for j, (invc, hi, lo) in zip(range(91, 182), rows):
        assert invc == float(Decimal(128) / Decimal(j))
        exact = -Decimal(invc).ln()
        assert abs(Decimal(hi) + Decimal(lo) - exact) <= abs(exact) * Decimal(2) ** -100 + Decimal(2) ** -1074
        if j == 128:
            assert (invc, hi, lo) == (1.0, 0.0, 0.0)
