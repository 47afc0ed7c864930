"""Sanitizer runs of the host-side code (CPU only, no GPU touched).

* The oracle (``oracle/gv_oracle.c``) built with gcc's AddressSanitizer and
  UndefinedBehaviorSanitizer, driven over every entry point on small
  circuits (``tests/sanitize/oracle_main.c``).
* The library's host code (``csrc/gv_api.cpp``, ``csrc/gv_batch.cpp``: ingest,
  planning, size queries, argument checks) built with the same sanitizers on
  the host side only and linked with the library's device objects, driven by
  ``tests/sanitize/host_main.cpp``.
Any sanitizer report aborts the program (``-fno-sanitize-recover``)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
HOST_SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
            "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=900, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", *HOST_SAN, "-o", exe,
          os.path.join(ROOT, "oracle", "gv_oracle.c"), os.path.join(SAN, "oracle_main.c"), "-lm"])
    r = _run([exe], env=dict(os.environ, OMP_NUM_THREADS="2"))
    assert "0 failures" in r.stdout


def test_library_host_code_under_asan_ubsan(tmp_path):
    from paper_2607_02749_amd import build as B
    hipcc = B.hipcc()
    device_objs = [os.path.join(B.BUILD_DIR, s + ".o") for s in B.SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(o) for o in device_objs):
        B.build(incremental=True)
    # host-side sanitizers only: each -fsanitize= behind -Xarch_host
    xsan = [a for f in HOST_SAN for a in ("-Xarch_host", f)]
    common = ["-O1", "-g", "-std=c++17", f"--offload-arch={B.ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include")]
    objs = []
    for src in ("gv_api.cpp", "gv_batch.cpp"):
        o = str(tmp_path / (src + ".o"))
        _run([hipcc, *common, *xsan, "-x", "hip", "-c", os.path.join(B.CSRC, src), "-o", o])
        objs.append(o)
    main_o = str(tmp_path / "host_main.o")
    _run([hipcc, *xsan, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(SAN, "host_main.cpp"), "-o", main_o])
    exe = str(tmp_path / "host_san")
    _run([hipcc, f"--offload-arch={B.ARCH}", *xsan, "-o", exe, main_o, *objs, *device_objs])
    r = _run([exe])
    assert "0 failures" in r.stdout
