"""Host bookkeeping under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): the server
arena's first-fit allocator (exact fits, reuse, merging, random traffic against an ownership
map) and the C ABI's argument checks and workspace sizing, which return before any device
call.  The library's host source is compiled here with the sanitizers on its host pass only
(-Xarch_host), linked with the library's other objects, and run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_13731_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2507_13731_amd", "_build")


def test_host_code_under_sanitizers(tmp_path):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    objs = [os.path.join(BUILD, f + ".o") for f in ("omega.hip", "qgemm.hip", "lowp.hip", "chol.hip", "qsvd.hip",
                                                   "heig.hip", "heig_big.hip", "util.hip", "complete.hip",
                                                   "noalloc.hip")]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    lib_obj = str(tmp_path / "qlra_san.o")
    test_obj = str(tmp_path / "main.o")
    exe = str(tmp_path / "sanitize_main")
    common = ["hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC"] + inc + san
    subprocess.run(common + ["-c", os.path.join(CSRC, "qlra.cpp"), "-o", lib_obj], check=True, capture_output=True)
    subprocess.run(common + ["-c", os.path.join(ROOT, "tests", "host", "sanitize_main.cpp"), "-o", test_obj],
                   check=True, capture_output=True)
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", test_obj, lib_obj] + objs + ["-o", exe], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "passed" in r.stdout
