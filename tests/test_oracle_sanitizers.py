"""The oracle under the address and undefined-behaviour sanitizers.

The oracle's C source is built with ``-fsanitize=address,undefined`` (no
recovery: the first report aborts) and every pin runs against that build in a
child interpreter with the sanitizer runtime preloaded. A second build of a
copy with one planted out-of-bounds write (the scheduler-row clear one byte
too long) must be stopped by the sanitizer, which shows the instrumented build
is the one that ran.
"""
import os
import subprocess
import sys

import pytest

from oracle import ranc_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_FLAGS = ("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all")

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
from oracle import ranc_oracle as O
from tests import oracle_pins as P
lib = O._bind({lib!r})
for pin in P.ALL_PINS:
    pin(lib)
    print("pin ok", pin.__name__, flush=True)
print("ALL PINS OK", flush=True)
"""


def _asan_runtime():
    try:
        path = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run_pins(lib_path):
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib_path)], env=env,
                          capture_output=True, text=True, timeout=600)


@pytest.fixture(scope="module")
def runtime():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's sanitizer runtime is not installed")
    return rt


def test_pins_pass_under_sanitizers(runtime, tmp_path):
    lib = O.build_variant(O.source_text(), str(tmp_path / "orc_san.so"), SAN_FLAGS, bind=False)
    r = _run_pins(lib)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and "ALL PINS OK" in r.stdout, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]


def test_sanitizer_stops_a_planted_overflow(runtime, tmp_path):
    src = O.source_text()
    old = "memset(sram_row(s, c, s->curr[c]), 0, (size_t)A);"
    assert old in src
    lib = O.build_variant(src.replace(old, "memset(sram_row(s, c, s->curr[c]), 0, (size_t)A + 1);", 1),
                          str(tmp_path / "orc_san_bad.so"), SAN_FLAGS, bind=False)
    r = _run_pins(lib)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, (r.stdout + r.stderr)[-3000:]
