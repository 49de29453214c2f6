"""The FP64 oracle and the host side of the HIP library built with the
address and undefined-behaviour sanitizers (g++, host code only) and driven
through every set-up call, the table builders and the error paths
(tests/native/*_sanitize_main.cpp).  The oracle driver also steps grids with
every element kind.  No GPU is used: the library's device code objects are
linked unsanitized and never launched."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def _run(exe, tmp):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600, cwd=tmp)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-3000:] + r.stderr[-3000:]


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_san")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off"] + SAN +
                   ["-I", os.path.join(ROOT, "oracle"), "-o", exe, os.path.join(NATIVE, "orc_sanitize_main.cpp"),
                    os.path.join(ROOT, "oracle", "orc.cpp")], check=True)
    _run(exe, tmp_path)


def test_host_runtime_under_address_and_ub_sanitizers(tmp_path):
    from paper_2207_06908_amd.csrc import build as hipbuild
    build = os.path.join(ROOT, "paper_2207_06908_amd", "_build")
    # the FDTD kernel objects (device code as built; only the host side is
    # instrumented)
    objs = [os.path.join(build, f + ".o") for f in hipbuild.SOURCES if f.startswith("fdtd_") and f.endswith(".hip")]
    if not all(os.path.exists(o) for o in objs):
        hipbuild.build()
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    if not os.path.exists(os.path.join(rocm, "lib", "libamdhip64.so")):
        pytest.skip("no HIP runtime library to link")
    host_o = str(tmp_path / "fdtd_host.o")
    main_o = str(tmp_path / "main.o")
    exe = str(tmp_path / "host_san")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2207_06908_amd", "csrc")]
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include")] +
                   inc + SAN + ["-c", os.path.join(ROOT, "paper_2207_06908_amd", "csrc", "fdtd_host.cpp"), "-o", host_o],
                   check=True)
    subprocess.run(["g++", "-O1", "-g", "-std=c++17"] + inc + SAN +
                   ["-c", os.path.join(NATIVE, "host_sanitize_main.cpp"), "-o", main_o], check=True)
    subprocess.run(["g++"] + SAN + ["-o", exe, main_o, host_o] + objs +
                   ["-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")],
                   check=True)
    _run(exe, tmp_path)
