"""Host code under AddressSanitizer and UBSan, on the CPU: the oracle built
with gcc's sanitizers runs its own pinned tests, and libvdi built with the
sanitizers on its host code only (device code as usual) runs the C-ABI
tests (argument checks on the host, no device call).  Each run is a child
process with the sanitizer runtime preloaded; any report fails the test."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORT_MARKS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer", "SUMMARY: UndefinedBehavior")


def _run_pytest(files, env_extra, timeout, lib):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    # the runtimes are live in the child (the library under test loads and
    # both sanitizers' report entry points resolve)
    probe = (f"import ctypes; ctypes.CDLL({lib!r}, mode=ctypes.RTLD_GLOBAL); g = ctypes.CDLL(None); "
             "g.__asan_report_load8; g.__ubsan_handle_add_overflow")
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    bad = [m for m in REPORT_MARKS if m in out]
    assert r.returncode == 0 and not bad, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    so = str(tmp_path / "libvdi_oracle_asan.so")
    src = os.path.join(ROOT, "oracle", "vdi_oracle.c")
    # the oracle's own flags (fp contraction off, no fast math) plus the sanitizers
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                    "-shared", "-fPIC", src, "-o", so, "-lm"], check=True)
    files = sorted(os.path.relpath(f, ROOT) for f in glob.glob(os.path.join(ROOT, "tests", "test_oracle*.py")))
    out = _run_pytest(files, {"LD_PRELOAD": asan, "VDI_ORACLE_LIBRARY": so}, timeout=900, lib=so)
    assert "passed" in out


def test_libvdi_host_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2206_14503_amd import build as B
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc or clang AddressSanitizer runtime")
    # host code only: each sanitizer flag goes to the host compilation
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([B.HIPCC, *B.FLAGS, *host_san, "-c", src, "-o", obj], check=True, capture_output=True)
        return obj

    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2206_14503_amd", "csrc", "*.hip")))
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    so = str(tmp_path / "libvdi_asan.so")
    subprocess.run([B.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", so, *objs], check=True)
    out = _run_pytest(["tests/test_abi.py"], {"LD_PRELOAD": rt[0], "VDI_LIBRARY": so}, timeout=600, lib=so)
    assert "passed" in out
