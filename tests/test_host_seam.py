"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer, without a GPU.

Every source of the library is compiled host-only (the device code is parsed, not emitted) and
linked with a host stand-in for the HIP runtime (tests/host_seam/hip_stub.cpp: host memory,
launch checks, stream / event / graph objects that enforce the capture rules) and a driver that
calls every entry point of the C ABI (tests/host_seam/driver.cpp).  The run must end without a
sanitizer report, a leak or a forbidden call, with every status as documented.  Two planted
mistakes, on the CPU, show that the seam reports what it is meant to."""

import concurrent.futures as cf
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_11790_amd", "csrc")
SEAM = os.path.join(ROOT, "tests", "host_seam")


def _tool(name):
    for cand in (shutil.which(name), f"/opt/rocm/bin/{name}", f"/opt/rocm/llvm/bin/{name}"):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc, clangxx = _tool("hipcc"), _tool("clang++")
    if not hipcc or not shutil.which("nm") or not shutil.which("gcc"):
        pytest.skip("hipcc / nm / gcc not available")
    out = tmp_path_factory.mktemp("host_seam")
    srcs = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC))
            if f.endswith((".hip", ".cpp"))]
    srcs += [os.path.join(SEAM, "hip_stub.cpp"), os.path.join(SEAM, "driver.cpp")]
    flags = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
             "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC]

    def compile_one(src):
        obj = os.path.join(out, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, f"{src}:\n{r.stderr[-3000:]}"
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    # host-only objects still name the device binaries their kernels would register: define
    # those symbols as empty blobs (the stand-in registration ignores them)
    und = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True).stdout
    blobs = sorted(set(re.findall(r"\b(__hip_fatbin_[0-9a-f]+)\b", und)))
    cfile = os.path.join(out, "fatbins.c")
    with open(cfile, "w") as f:
        f.writelines(f"char {b}[16];\n" for b in blobs)
    cobj = cfile + ".o"
    subprocess.run(["gcc", "-c", cfile, "-o", cobj], check=True)
    exe = os.path.join(out, "driver")
    linker = clangxx or hipcc
    r = subprocess.run([linker, "-fsanitize=address,undefined", "-o", exe, *objs, cobj],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe, out


def _run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)


def test_every_entry_point_runs_clean_under_sanitizers(driver):
    exe, out = driver
    r = _run(exe, os.path.join(out, "autotune.json"))
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    assert "host seam:" in r.stdout and "ok" in r.stdout, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text
    assert "LeakSanitizer" not in text
    launches = int(re.search(r"(\d+) kernel launches", r.stdout).group(1))
    assert launches > 500
    # the autotuner wrote its cache, and a second process reads it back
    assert os.path.getsize(os.path.join(out, "autotune.json")) > 0
    r2 = _run(exe, os.path.join(out, "autotune.json"))
    assert r2.returncode == 0, (r2.stdout + r2.stderr)[-4000:]


@pytest.mark.parametrize("what,report", [("capture", "while a stream capture is open"),
                                         ("oob", "heap-buffer-overflow")])
def test_seam_reports_planted_mistakes(driver, what, report):
    exe, _ = driver
    r = _run(exe, "--plant", what)
    assert r.returncode != 0
    assert report in r.stderr, r.stderr[-2000:]
    assert "not caught" not in r.stdout
