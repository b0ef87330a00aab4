"""The pins catch planted mistakes: every mutant of tests/oracle_mutants.py
(one plausible error in one oracle file) is written into a copy of the
oracle next to copies of the pin tests, and those pins must fail on it.  The
mistakes are planted in the oracle only, on the CPU."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from tests.oracle_mutants import FIRST, MUTANTS, PIN_FILES

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")


def _mutated_tree(dst, name, fname, old, new):
    """A tree with the oracle (one file mutated), the scene generator and the pins."""
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copytree(os.path.join(ROOT, "scenes"), os.path.join(dst, "scenes"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    for f in ["__init__.py", "conftest.py", "parity.py", "workloads.py", *PIN_FILES]:
        if os.path.exists(os.path.join(TESTS, f)):
            shutil.copy(os.path.join(TESTS, f), os.path.join(dst, "tests", f))
    shutil.copytree(os.path.join(TESTS, "golden"), os.path.join(dst, "tests", "golden"))
    path = os.path.join(dst, "oracle", fname)
    src = open(path).read()
    assert src.count(old) == 1, f"mutant {name}: its original text occurs {src.count(old)} times in {fname}"
    open(path, "w").write(src.replace(old, new))


def _run_pins(dst, fname):
    order = [FIRST[fname]] + [f for f in PIN_FILES if f != FIRST[fname]]
    env = {k: v for k, v in os.environ.items() if k != "PYTHONPATH"}
    env["OMP_NUM_THREADS"] = "1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           *[os.path.join("tests", f) for f in order]]
    return subprocess.run(cmd, cwd=dst, env=env, capture_output=True, text=True, timeout=600)


def test_every_planted_mistake_fails_a_pin(tmp_path):
    def one(m):
        name, fname, old, new = m
        dst = str(tmp_path / name)
        _mutated_tree(dst, name, fname, old, new)
        r = _run_pins(dst, fname)
        tail = (r.stdout + r.stderr).strip().splitlines()
        return name, r.returncode, tail[-1] if tail else ""

    workers = max(1, min(6, (os.cpu_count() or 2) - 1))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(one, MUTANTS))
    survived = [(n, last) for n, rc, last in results if rc == 0]
    broken = [(n, rc, last) for n, rc, last in results if rc not in (0, 1)]
    for n, rc, last in results:
        print(f"{n:40s} rc={rc} {last}")
    assert not broken, f"mutants that did not run as tests: {broken}"
    assert not survived, f"planted mistakes no pin catches: {survived}"


def test_unmutated_copy_passes_the_pins(tmp_path):
    """The copy the mutants run in is sound: unmutated, its pins pass (the
    fast ones here; the whole pin suite runs on the real tree anyway)."""
    dst = str(tmp_path / "clean")
    _mutated_tree(dst, "clean", "vct_oracle.py", "mips.append(total / 8.0)", "mips.append(total / 8.0)")
    env = {k: v for k, v in os.environ.items() if k != "PYTHONPATH"}
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join("tests", "test_voxelize_pins.py"), os.path.join("tests", "test_shade_pins.py")],
                       cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:]
    # the copy, not the repository, is what the tests imported
    probe = subprocess.run([sys.executable, "-c", "import oracle, sys; print(oracle.__file__)"], cwd=dst, env=env,
                           capture_output=True, text=True, timeout=120)
    assert probe.stdout.strip().startswith(dst), probe.stdout + probe.stderr
