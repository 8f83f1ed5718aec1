"""Host code and oracle under AddressSanitizer + UndefinedBehaviorSanitizer
(CPU only): builds the library's host sources (construction, schedule
lowering, kernel-source generation, C ABI, request server) and the oracle
with -fsanitize=address,undefined into a temporary directory, then runs the
host-side library tests and the oracle pins against those builds in a child
process.  Device code is built without sanitizers (it is not run here)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_00353_amd", "csrc")
HOST_SOURCES = ["api.cpp", "construct.cpp", "unrolled.cpp", "server.cpp"]
DEVICE_SOURCES = ["decode.hip", "noalloc.hip"]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    if res.returncode != 0:
        raise AssertionError("%s failed (%d):\n%s\n%s" % (cmd[0], res.returncode, res.stdout[-4000:],
                                                           res.stderr[-4000:]))
    return res


def _build(tmp):
    sys.path.insert(0, ROOT)
    from paper_1504_00353_amd import build as libbuild
    libbuild.write_embedded()
    objs = []
    for src in DEVICE_SOURCES:  # device code: no sanitizer
        obj = os.path.join(tmp, src + ".o")
        _run(["/opt/rocm/bin/hipcc", "-c"] + [f for f in libbuild.HIPCC_FLAGS if f != "-shared"] +
             [os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HOST_SOURCES:  # host code: g++ with the sanitizers
        obj = os.path.join(tmp, src + ".o")
        _run(["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
              "-I" + CSRC] + SAN + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = os.path.join(tmp, "libpolar_san.so")
    _run(["g++", "-shared"] + SAN + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-lhiprtc", "-ldl",
                                            "-Wl,-rpath,/opt/rocm/lib", "-o", lib])
    orc = os.path.join(tmp, "liboracle_san.so")
    _run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
          "-pthread"] + SAN + [os.path.join(ROOT, "oracle", "oracle.cpp"), "-o", orc])
    return lib, orc


@pytest.mark.timeout(900)
def test_host_and_oracle_under_asan_ubsan(tmp_path):
    lib, orc = _build(str(tmp_path))
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    assert os.path.isabs(asan) and os.path.exists(asan)
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": asan,
        # the interpreter and the HIP runtime keep allocations to exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1:exitcode=87",
        "POLAR_LIBRARY": lib,
        "POLAR_ORACLE_LIBRARY": orc,
        "POLAR_KERNEL_CACHE": str(tmp_path / "kernels"),
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                          "-k", "not unrolled_kernel_builds",
                          os.path.join(ROOT, "tests", "test_library_host.py"),
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=850)
    out = res.stdout[-3000:] + res.stderr[-6000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert res.returncode == 0, out
    assert " passed" in res.stdout
    # the child processes load the sanitized builds, not the regular ones
    probe = ("import oracle; from paper_1504_00353_amd import binding; binding.lib(); oracle.lib(); "
             "m = open('/proc/self/maps').read(); print('libpolar_san.so' in m, 'liboracle_san.so' in m, "
             "'libasan' in m)")
    res = subprocess.run([sys.executable, "-c", probe], cwd=ROOT, env=env, capture_output=True, text=True)
    assert res.stdout.split() == ["True", "True", "True"], res.stdout + res.stderr
