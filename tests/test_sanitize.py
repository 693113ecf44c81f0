"""The C runtime's host paths under AddressSanitizer and UBSan.

The runtime source is compiled with g++ and the sanitizers (host code only),
linked with the normally built kernel objects into a small C driver
(tests/abi_sanitize_driver.c) that exercises every path reachable without a
GPU.  Any out-of-bounds access, use-after-free or undefined behaviour aborts
that program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2404_04441_amd", "csrc")
# every kernel object the library is linked from (the .hip units of the build)
KOBJS = [os.path.join(ROOT, "paper_2404_04441_amd", "_build", n) for n in
         ("step_f32.o", "step_f16.o", "step_bf16.o", "step_f16m.o", "step_bf16m.o", "step_adj.o", "wave_kernels.o")]
ROCM = "/opt/rocm"


@pytest.mark.skipif(not shutil.which("g++") or not os.path.isdir(os.path.join(ROCM, "include", "hip")),
                    reason="needs g++ and the ROCm headers")
def test_host_paths_clean_under_asan_and_ubsan(tmp_path):
    if not all(os.path.exists(k) for k in KOBJS):
        pytest.skip("build the library first (paper_2404_04441_amd.build)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__"]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
    robj = tmp_path / "runtime.o"
    subprocess.run(["g++", "-std=c++17", *san, *inc, "-c", os.path.join(CSRC, "wave_runtime.cpp"), "-o", str(robj)],
                   check=True)
    dobj = tmp_path / "driver.o"
    subprocess.run(["gcc", "-std=c11", *san, *inc, "-c", os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), "-o",
                    str(dobj)], check=True)
    exe = tmp_path / "driver"
    subprocess.run(["g++", *san, str(dobj), str(robj), *KOBJS, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", str(exe)], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(res.stdout, res.stderr[-3000:])
    assert res.returncode == 0 and "ok" in res.stdout
