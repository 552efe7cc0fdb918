"""The oracle's pins catch planted mistakes.

Each case replaces one oracle function with a plausibly wrong version (a flipped sign, a
dropped factor, a shifted index, a missing conjugate, a wrong grid pitch; see
_oracle_mutations.py) and runs the pins of test_oracle_pins.py in a fresh process: at least
one pin must fail.  The mistakes are planted in the oracle only, on the CPU.
"""
import os
import subprocess
import sys

import pytest

import _oracle_mutations as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

RUN = """
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import _oracle_mutations as M
M.apply({name!r})
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", {pins!r}]))
"""


@pytest.mark.parametrize("name", sorted(M.MUTATIONS))
def test_pins_catch_planted_mistake(name):
    code = RUN.format(root=ROOT, tests=os.path.join(ROOT, "tests"), name=name,
                      pins=os.path.join(ROOT, "tests", "test_oracle_pins.py"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 1, (name, r.returncode, r.stdout[-2000:])
    assert "failed" in r.stdout, (name, r.stdout[-2000:])
