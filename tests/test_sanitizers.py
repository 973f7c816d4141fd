"""CPU AddressSanitizer + UndefinedBehaviorSanitizer runs of the host-side code:

* the oracle's C (oracle.c) built with gcc's sanitizers, under the oracle pins that call it;
* the host side of the library (rt_api.hip: argument validation, schedules, replica
  selection, plan tables, error reporting) built with clang's host sanitizers and linked
  with the unchanged device objects, under the C-ABI checks of test_abi.py (no device call).

Each runs in a child process with the sanitizer runtime preloaded (the Python interpreter
itself is not instrumented), leak detection off, and every report fatal."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["tests/test_oracle_cosmology.py", "tests/test_oracle_bundles.py", "tests/test_oracle_field.py",
                "tests/test_oracle_geodesic.py", "tests/test_oracle_nfw.py"]


def _run_pytest(tests, env_extra, tmp_path):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    log = tmp_path / "child.log"
    with open(log, "w") as fh:
        rc = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider"] + tests,
                            cwd=ROOT, env=env, stdout=fh, stderr=subprocess.STDOUT, timeout=900).returncode
    out = log.read_text()
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert rc == 0, out[-4000:]
    return out


def test_oracle_c_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc missing")
    libasan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's libasan.so missing")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run([gcc, "-O1", "-g", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", str(lib), os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
                   check=True)
    out = _run_pytest(ORACLE_TESTS, {"ORACLE_LIB": str(lib), "LD_PRELOAD": libasan}, tmp_path)
    assert " passed" in out


def _clang_asan_runtime():
    base = "/opt/rocm/llvm/lib/clang"
    if not os.path.isdir(base):
        return None
    for ver in sorted(os.listdir(base), reverse=True):
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    return None


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_1110_4894_amd import build as libbuild
    objs = [os.path.join(ROOT, "_build", f) for f in ("rt_kernels.o", "rt_pm.o")]
    rtasan = _clang_asan_runtime()
    clang = os.path.join(os.path.dirname(libbuild.llvm_tool("clang++")), "clang++")
    if rtasan is None or not os.path.exists(clang) or not all(os.path.exists(o) for o in objs):
        pytest.skip("clang's ASan runtime, clang++ or the device objects missing (build first)")
    api = tmp_path / "rt_api_san.o"
    # sanitizers on the host pass only (the device code of rt_api.hip is none)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-shared-libasan"]
    subprocess.run([libbuild.hipcc()] + libbuild.FLAGS + ["-g", "-O1", "-fno-omit-frame-pointer"] + san +
                   ["-c", os.path.join(libbuild.CSRC, "rt_api.hip"), "-o", str(api)], check=True)
    lib = tmp_path / "librt_san.so"
    subprocess.run([clang, "-shared", "-fsanitize=address,undefined", "-shared-libasan", "-o", str(lib), str(api)] +
                   objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
    out = _run_pytest(["tests/test_abi.py"], {"RT_LIB_PATH": str(lib), "LD_PRELOAD": rtasan}, tmp_path)
    assert " passed" in out
