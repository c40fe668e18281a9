"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
  * the device library built with the sanitizers on its host side (hipcc
    -Xarch_host -fsanitize=...; device code is built as usual and never runs
    here), driving the mesh preparation, tiling and layout export of
    test_host_layout.py;
  * the FP64 oracle built with g++ and the sanitizers, driving the physics
    pins and the timing-mode tests.
Each run happens in a subprocess with the sanitizer runtime preloaded; any
report aborts it (halt_on_error), so a zero exit status is the pass."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = "-fsanitize=address,undefined"


def _clang_asan_runtime():
    out = subprocess.run(["/opt/rocm/lib/llvm/bin/clang", "-print-file-name="
                          "libclang_rt.asan-x86_64.so"], capture_output=True,
                         text=True).stdout.strip()
    if not os.path.isfile(out):
        import glob
        hits = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/"
                         "libclang_rt.asan-x86_64.so")
        out = hits[0] if hits else ""
    return out


def _gcc_runtime(name):
    return subprocess.run(["gcc", f"-print-file-name={name}"],
                          capture_output=True, text=True).stdout.strip()


def _instrumented(lib):
    """The library calls into both sanitizer runtimes (instrumented code)."""
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib],
                          capture_output=True, text=True).stdout
    return "__asan_report" in syms and "__ubsan_handle" in syms


def _run_pytest(tests, env_extra, preload):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = os.path.join(ROOT, "tests", "sanitize") + os.pathsep + ROOT
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "_asan_plugin",
           "-p", "no:cacheprovider", "-m", "not gpu", *tests]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error:" not in tail, tail
    return tail


def test_host_library_under_asan_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    if not rt:
        pytest.skip("clang AddressSanitizer runtime not found")
    csrc = os.path.join(ROOT, "paper_2003_03130_amd", "csrc")
    from paper_2003_03130_amd.build import SOURCES
    srcs = [os.path.join(csrc, s) for s in SOURCES]
    lib = str(tmp_path / "libcellmech_san.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
           "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", SAN, "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), "-o", lib, *srcs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert _instrumented(lib)
    tail = _run_pytest(["tests/test_host_layout.py"], {"CM_SANITIZED_LIB": lib}, rt)
    assert "passed" in tail


def test_oracle_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not (os.path.isfile(asan) and os.path.isfile(ubsan)):
        pytest.skip("gcc sanitizer runtimes not found")
    so = str(tmp_path / "libcm_oracle_san.so")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math",
           SAN, "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-o", so,
           os.path.join(ROOT, "oracle", "cm_oracle.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    assert _instrumented(so)
    tail = _run_pytest(["tests/test_oracle_pins.py", "tests/test_oracle_batch.py"],
                       {"ORACLE_SANITIZED_LIB": so}, asan + ":" + ubsan)
    assert "passed" in tail
