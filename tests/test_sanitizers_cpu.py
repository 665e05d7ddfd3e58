"""Host sanitizer runs (CPU only, no device code):

* the C oracle under AddressSanitizer + UndefinedBehaviorSanitizer
  (tests/oracle_sanitize_check.c: every exported routine, every boundary
  type, unequal extents);
* the library's host code -- the csrc/*.hip files without device code,
  compiled for the host only, linked with the regular objects of the kernel
  files -- under ASan + UBSan and under ThreadSanitizer
  (tests/host_sanitize_check.cpp: argument validation, workspace planning,
  the tuning cache and its file format, the serving scheduler in simulation
  mode with concurrent submitting and polling threads).

A sanitizer finding aborts its program with a report, which fails the test."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2503_16994_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = {"asan_ubsan": ["address", "undefined"], "tsan": ["thread"]}
HOST_FILES = {"lqcd_abi.hip", "lqcd_server.hip", "lqcd_solver.hip", "lqcd_tune.hip"}


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:] + r.stderr[-4000:]
    return r


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_check")
    _run([gcc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(ROOT, "tests", "oracle_sanitize_check.c"), "-o", exe, "-lm"])
    r = _run([exe], timeout=300)
    assert "all ok" in r.stdout, r.stdout


@pytest.mark.parametrize("kind", sorted(SAN))
def test_library_host_code_under_sanitizers(tmp_path, kind):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("no ROCm toolchain")
    # every sanitizer flag of a hipcc line applies to the host pass only
    san_host = []
    for s in SAN[kind]:
        san_host += ["-Xarch_host", f"-fsanitize={s}"]

    def obj(src):
        o = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fPIC", *san_host,
              "-c", src, "-o", o])
        return o

    # the host-side files (no device code) are rebuilt instrumented; the
    # kernel files come from the library's regular build, since their host
    # part is only launch code
    from paper_2503_16994_amd import build
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    host = [s for s in srcs if os.path.basename(s) in HOST_FILES]
    assert len(host) == len(HOST_FILES)
    regular = [os.path.join(build.BUILD_DIR, os.path.basename(s) + ".o") for s in srcs if s not in host]
    if not all(os.path.exists(o) for o in regular):
        build.build()
    with cf.ThreadPoolExecutor(len(host)) as ex:
        objs = list(ex.map(obj, host)) + regular
    exe = str(tmp_path / "host_check")
    link_san = "-fsanitize=" + ",".join(SAN[kind])
    _run([CLANGXX, "-O1", "-g", "-std=c++17", link_san, f"-I{os.path.join(ROOT, 'include')}",
          os.path.join(ROOT, "tests", "host_sanitize_check.cpp"), *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-lpthread", "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1")
    r = _run([exe, str(tmp_path)], timeout=300, env=env)
    print(r.stdout)
    assert "all ok" in r.stdout, r.stdout + r.stderr
