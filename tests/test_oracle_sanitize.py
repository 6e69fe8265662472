"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(host build with gcc): a driver calls every entry point on small seeded cases
(ragged sizes, W above and below the cell count, every max(V) and clamp mode,
16 fields) and must finish without a sanitizer report or leak."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _sanitizers_available(tmp):
    probe = os.path.join(tmp, "probe.c")
    with open(probe, "w") as fh:
        fh.write("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", "-static-libasan", probe, "-o", os.path.join(tmp, "probe")],
                       capture_output=True, text=True)
    return r.returncode == 0


def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    tmp = str(tmp_path)
    if not _sanitizers_available(tmp):
        pytest.skip("gcc sanitizer runtimes not available")
    exe = os.path.join(tmp, "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan",
           "-I", os.path.join(ROOT, "oracle"),
           os.path.join(ROOT, "oracle", "dvl_oracle.c"), os.path.join(HERE, "oracle_sanitize_driver.c"),
           "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok"), r.stdout[-2000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
