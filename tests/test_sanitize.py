"""The kernel bodies under AddressSanitizer and UndefinedBehaviorSanitizer on
the CPU.

tests/native/emu.cpp compiles the GPU kernel bodies as host code; here it is
built once more with both sanitizers (host code only, line lengths up to 64 to
keep the build short) together with tests/native/sanitize_main.cpp, which runs
every emulated kernel family on exactly sized arrays.  Any access outside an
array, misaligned access, signed overflow or out-of-range shift in the shared
index code aborts the run."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")
OUT = os.path.join(NATIVE, "_build", "emu_sanitize")
SRCS = [os.path.join(NATIVE, "emu.cpp"), os.path.join(NATIVE, "sanitize_main.cpp")]
CSRC = os.path.join(ROOT, "paper_2307_07749_amd", "csrc")


def _stale():
    if not os.path.exists(OUT):
        return True
    deps = SRCS + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp")]
    t = os.path.getmtime(OUT)
    return any(os.path.getmtime(p) > t for p in deps)


def _build():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    # host-only build; each sanitizer flag applies to the host pass
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-host-only", "-std=c++17", "-O0", "-g1",
           "-DEMU_MAX_L=64",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SRCS, "-o", OUT + ".tmp", "-lpthread"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError(r.stdout[-4000:])
    os.replace(OUT + ".tmp", OUT)


@pytest.mark.timeout(900)
def test_kernel_bodies_clean_under_asan_and_ubsan():
    if not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc not available")
    if _stale():
        _build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([OUT], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout
    assert r.stdout.strip().endswith("ok")
