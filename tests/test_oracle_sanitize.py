"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only): oracle/sanitize_driver.c calls every entry point on small grids with
the edge cases (axes, radial edges, leaving, neutral, massless and empty
slots, filter passes, the absorbing layer, the general map, injection up to
the capacity); any access outside an array or undefined arithmetic ends it
with a report and a non-zero status.  A planted write one past the field set
shows that the build catches such a mistake."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "oracle", "sanitize_driver.c")
FLAGS = ["-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
         "-fno-sanitize-recover=undefined", "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas"]


def build_and_run(tmp_path, extra=()):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = os.path.join(str(tmp_path), "orc_san")
    subprocess.run(["gcc", *FLAGS, *extra, "-o", exe, DRIVER, "-lm"], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)


def test_oracle_clean_under_sanitizers(tmp_path):
    r = build_and_run(tmp_path)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_sanitizer_build_catches_a_planted_overrun(tmp_path):
    r = build_and_run(tmp_path, ["-DPLANT_OUT_OF_BOUNDS"])
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr
