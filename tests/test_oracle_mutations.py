"""Every planted mistake of tests/oracle_mutants.py is caught by the oracle's
pin tests (no GPU): each mutant runs its module's pin file in a child pytest
process with the mutated oracle installed, which must end with failed tests
(exit status 1); the unmutated oracle passes the same files in the main
suite."""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.oracle_mutants import MUTANTS, ROOT

pytestmark = pytest.mark.slow


def _run(mid):
    env = dict(os.environ, HC_ORACLE_MUTANT=mid)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-p", "no:xdist",
                        os.path.join(ROOT, "tests", MUTANTS[mid][3])],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return mid, r.returncode, (r.stdout + r.stderr)[-1500:]


def test_every_planted_mistake_is_caught():
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_run, sorted(MUTANTS)))
    survivors = [mid for mid, rc, _ in results if rc == 0]
    broken = [(mid, rc, out) for mid, rc, out in results if rc not in (0, 1)]
    assert not broken, broken[:2]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
