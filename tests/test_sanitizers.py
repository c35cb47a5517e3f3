"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The C oracle is rebuilt with gcc -fsanitize=address,undefined and its pin
suite run against it; a copy with a planted heap overflow must be caught.
The HIP library's host code (the serving scheduler, the context and frame
management) is rebuilt with the sanitizers on the host side only
(-Xarch_host; device code unchanged) and the scheduler's tests run on the
simulated device.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_SRC = os.path.join(ROOT, "oracle", "duplex_oracle.c")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _build_oracle(src, out):
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                           "-shared", "-fPIC", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", out, src, "-lm"])


def _run_pins(lib):
    env = dict(os.environ, DUPLEX_ORACLE_LIB=lib, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=0",
               LD_PRELOAD=f"{_gcc_runtime('libasan.so')} {_gcc_runtime('libubsan.so')}")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py")], env=env, cwd=ROOT,
                          capture_output=True, text=True, timeout=600)


@pytest.mark.skipif(not (_gcc_runtime("libasan.so") and _gcc_runtime("libubsan.so")), reason="no gcc sanitizers")
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    _build_oracle(ORACLE_SRC, lib)
    r = _run_pins(lib)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    # the instrumentation is live: a heap overflow planted in a copy is caught
    src = open(ORACLE_SRC).read()
    anchor = "int32_t *first = malloc(sizeof(int32_t) * (N + 1));"
    assert anchor in src
    bad = tmp_path / "overflow.c"
    bad.write_text(src.replace(anchor, "int32_t *first = malloc(sizeof(int32_t) * N);", 1))
    badlib = str(tmp_path / "liboverflow.so")
    _build_oracle(str(bad), badlib)
    r = _run_pins(badlib)
    assert r.returncode != 0 and "heap-buffer-overflow" in (r.stdout + r.stderr)


def _clang_asan():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


@pytest.mark.skipif(not (_clang_asan() and os.path.exists(HIPCC)), reason="no hipcc or clang ASan runtime")
def test_scheduler_under_asan_and_ubsan(tmp_path):
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2508_03180_amd", "csrc", "*.hip")))
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fhip-fp32-correctly-rounded-divide-sqrt",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2508_03180_amd", "csrc"),
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer"]
    procs, objs = [], []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC, *flags, "-c", s, "-o", o], stderr=subprocess.DEVNULL))
    assert all(p.wait() == 0 for p in procs)
    lib = str(tmp_path / "libduplexgs_san.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-o", lib, *objs])
    runner = tmp_path / "run.py"
    runner.write_text(
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "from paper_2508_03180_amd import _capi\n"
        f"_capi.LIB_PATH = {lib!r}\n"
        "import pytest\n"
        f"sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', {os.path.join(ROOT, 'tests', 'test_serving_sim.py')!r}]))\n")
    env = dict(os.environ, LD_PRELOAD=_clang_asan(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(runner)], env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
