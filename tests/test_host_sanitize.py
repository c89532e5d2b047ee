"""Host-side set-up and validation code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU needed).

Every library source is compiled with the sanitizers on the host pass only (each
-fsanitize after -Xarch_host; device code is built as usual) and linked with
tests/native/host_checks.cpp, which drives bie::build through its host work (input
checks, near / close pair lists, grid and transform tables, the separation threshold)
and the solver's option checks, on good and bad inputs.  The build is cached under
_build/sanitize/ and redone when a source changes."""
import hashlib
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_06551_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
DRIVER = os.path.join(ROOT, "tests", "native", "host_checks.cpp")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")


def _sources():
    sys.path.insert(0, ROOT)
    from paper_1707_06551_amd.build import HIP_FLAGS, SOURCES
    return [os.path.join(CSRC, s) for s in SOURCES] + [DRIVER], [f for f in HIP_FLAGS if f != "-O3"]


def _compile(src, flags):
    obj = os.path.join(OUT, os.path.basename(src) + ".o")
    cmd = ["hipcc", *flags, "-O1", "-g", *SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip", "-c",
           src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return obj


@pytest.fixture(scope="module")
def checker():
    srcs, flags = _sources()
    h = hashlib.sha256()
    for p in srcs + [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".h")] + \
            [os.path.join(ROOT, "include", "bie.h")]:
        h.update(open(p, "rb").read())
    h.update(" ".join(flags + SAN).encode())
    exe = os.path.join(OUT, "host_checks")
    stamp = os.path.join(OUT, "stamp")
    if not (os.path.exists(exe) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest()):
        os.makedirs(OUT, exist_ok=True)
        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            objs = list(ex.map(lambda s: _compile(s, flags), srcs))
        r = subprocess.run(["hipcc", "--offload-arch=gfx950", *SAN, *objs, "-o", exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        with open(stamp, "w") as f:
            f.write(h.hexdigest())
    return exe


def test_host_setup_and_validation_under_sanitizers(checker):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([checker], capture_output=True, text=True, env=env, timeout=900)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "host checks: 0 failure(s)" in out, out[-4000:]
