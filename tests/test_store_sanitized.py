"""Host C++ of the library under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the clause/occurrence store builder and the DIMACS reader
(csrc/tsat_store.cpp, plain C++) are compiled with g++ together with
tests/store_check.cpp, which checks random stores against a naive
restatement, the size limits of the occurrence store, the argument errors
and the DIMACS parser on good and malformed files."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2511_07737_amd", "csrc")


@pytest.mark.timeout(300)
def test_store_builder_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "store_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(CSRC, "tsat_store.cpp"), os.path.join(HERE, "store_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the sanitizer runtime need not be the first
    # library the loader maps (the environment may preload others)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=240)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
