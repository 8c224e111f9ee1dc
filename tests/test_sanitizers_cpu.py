"""The host-side C and C++ under AddressSanitizer and UndefinedBehaviorSanitizer:
the library's host code (context, keygen, decryption, CRT and fixed point, wire
format, plans and server bookkeeping, tuning) and the C oracle are rebuilt with
both sanitizers (host code only; the kernel objects are the normal build) and
the CPU tests of the client calls, the wire format, the library's host paths
and the oracle pins run against them in a child process.  Any sanitizer report
fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_05496_amd", "csrc")
OBJS = os.path.join(ROOT, "paper_2204_05496_amd", "_build")
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SOURCES = ("host.cpp", "plan.cpp", "wire.cpp", "prof.cpp")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libsan", "-fno-omit-frame-pointer",
       "-Wno-pass-failed",
       "-g", "-O1", "-fPIC", "-fopenmp"]


def asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def san_libs(tmp_path_factory):
    rt = asan_runtime()
    if not rt or not os.path.exists(CLANG + "++"):
        pytest.skip("clang sanitizer runtime not available")
    kobjs = [os.path.join(OBJS, "kernels.hip.o"), os.path.join(OBJS, "valu_rate.hip.o")] + \
        sorted(glob.glob(os.path.join(OBJS, "ks_step.ln*.o")))
    if not all(os.path.exists(o) for o in kobjs[:2]) or len(kobjs) < 8:
        pytest.skip("kernel objects not built (run paper_2204_05496_amd/build.py first)")
    d = tmp_path_factory.mktemp("san")
    ora = str(d / "liboracle_san.so")
    subprocess.check_call([CLANG, "-std=c11", *SAN, "-shared", os.path.join(ROOT, "oracle", "bfv_oracle.c"), "-o", ora])
    hobjs = []
    for src in HOST_SOURCES:
        o = str(d / (src + ".o"))
        subprocess.check_call([CLANG + "++", "-x", "c++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                               "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SAN, "-c",
                               os.path.join(CSRC, src), "-o", o])
        hobjs.append(o)
    lib = str(d / "liblrhe_san.so")
    subprocess.check_call([CLANG + "++", "-shared", *SAN, *hobjs, *kobjs, "-L/opt/rocm/lib", "-lamdhip64",
                           "-Wl,-rpath,/opt/rocm/lib", "-o", lib])
    return rt, lib, ora


def test_cpu_suites_under_sanitizers(san_libs):
    rt, lib, ora = san_libs
    env = dict(os.environ, LD_PRELOAD=rt, LRHE_LIB=lib, LRHE_ORACLE_LIB=ora,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_boundary_cpu.py", "test_wire_cpu.py", "test_lib_cpu.py", "test_oracle_pins.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider", *tests],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
