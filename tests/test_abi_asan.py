"""The host driver under AddressSanitizer, on the CPU.

``csrc/api.hip`` (argument checks, workspace layout, error messages) is
compiled with host-side AddressSanitizer (``-Xarch_host -fsanitize=address``;
device code is built as usual) and linked, with the library's other objects
from the regular build (compiled afresh where stale), into
``tests/asan/abi_validation.cpp``: a program that
drives every entry point through the argument checks the C ABI refuses before
any HIP call.  The program must report every expected status and message, and
AddressSanitizer (with leak detection) must report nothing."""
import concurrent.futures as cf
import os
import subprocess

import pytest

from paper_1502_06216_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "asan", "abi_validation.cpp")
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _regular_objects(tmp):
    """Objects of the regular build for every source but api.hip: those the
    last build left, where they are newer than their source and every header,
    else compiled afresh (same flags) into `tmp`."""
    headers = [os.path.join(B.CSRC, f) for f in os.listdir(B.CSRC) if f.endswith(".h")]
    headers.append(os.path.join(B.INCLUDE, "jko.h"))
    newest = max(os.path.getmtime(f) for f in headers)
    hipcc = B._hipcc()
    objs, todo = [], []
    for src in B.sources():
        if os.path.basename(src) == "api.hip":
            continue
        obj = os.path.join(B.BUILD_DIR, os.path.basename(src)[:-4] + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(newest, os.path.getmtime(src)):
            obj = os.path.join(str(tmp), os.path.basename(src)[:-4] + ".o")
            todo.append((src, obj))
        objs.append(obj)
    with cf.ThreadPoolExecutor(max_workers=max(1, min(len(todo), 4))) as ex:
        for cmd, res in ex.map(lambda so: B._compile(hipcc, so[0], so[1], []), todo):
            assert res.returncode == 0, " ".join(cmd) + "\n" + res.stderr
    return objs


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    noise = "\n".join(ln for ln in (res.stderr or "").splitlines() if "packed-fp32-ops" not in ln)
    assert res.returncode == 0, " ".join(cmd) + "\n" + noise + "\n" + (res.stdout or "")
    return res


@pytest.mark.timeout(600)
def test_host_driver_under_address_sanitizer(tmp_path):
    hipcc = B._hipcc()
    objs = _regular_objects(tmp_path)
    api_o = str(tmp_path / "api_asan.o")
    drv_o = str(tmp_path / "abi_validation.o")
    exe = str(tmp_path / "abi_validation")
    _run([hipcc, f"--offload-arch={B.ARCH}", "-O1", "-g", "-std=c++17", "-c", *HOST_ASAN, *B.DEVICE_FLAGS,
          f"-I{B.INCLUDE}", f"-I{B.CSRC}", os.path.join(B.CSRC, "api.hip"), "-o", api_o])
    _run([hipcc, "-x", "c++", "-O1", "-g", "-std=c++17", "-c", *HOST_ASAN, f"-I{B.INCLUDE}", DRIVER, "-o", drv_o])
    _run([hipcc, f"--offload-arch={B.ARCH}", "-Xarch_host", "-fsanitize=address", api_o, *objs, drv_o, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:detect_stack_use_after_return=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "AddressSanitizer" not in res.stderr and "LeakSanitizer" not in res.stderr, res.stderr
    assert res.stdout.startswith("ok "), res.stdout
    assert int(res.stdout.split()[1]) >= 80
