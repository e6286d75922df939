"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): a sanitized copy of the C oracle runs a representative part of the
pin suite; any out-of-bounds access, overflow or other undefined behaviour
aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "stratego_oracle.c")


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.parametrize("kind", ["undefined", "address,undefined"])
def test_pins_pass_under_sanitizers(tmp_path, kind):
    preload = None
    if "address" in kind:
        preload = _runtime("libasan.so")
        if preload is None:
            pytest.skip("no libasan runtime")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                           f"-fsanitize={kind}", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           SRC, "-o", str(lib), "-lm"])
    env = dict(os.environ, STRATEGO_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    if preload:
        env["LD_PRELOAD"] = preload
    keep = ("battle or geometry or brute_force_random or lone_scout or terminal or deaths or threat or "
            "evasion or protection or probability_channels_at_ply0 or round_trip or resample_invariants or "
            "two_square or magnet_probabilities or search_policy_special or chasing_rule_forbids or acting")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-q", "-x", "-p", "no:cacheprovider", "-k", keep],
                       env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
