"""The library's host code under AddressSanitizer (CPU only).

Every source is compiled with the sanitizer on the host side only (the
device code is built as usual) and linked into a small driver
(asan_host_driver.cpp) that runs the host paths: parameter validation, the
FP64 construction of every 2-D and 3-D plan's tables up to its first device
allocation, the argument checks of the other handles and the status strings.
A heap overflow, use after free or similar error in that code makes the run
fail."""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu_present() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not found")
@pytest.mark.skipif(_gpu_present(), reason="host-only check, meant for machines without a GPU")
def test_host_code_under_address_sanitizer():
    from paper_1810_11685_amd import build as B
    cc = B.hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    with tempfile.TemporaryDirectory(prefix="qpat_asan_") as tmp:
        srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(HERE, "asan_host_driver.cpp")]
        objs = [os.path.join(tmp, os.path.basename(s) + ".o") for s in srcs]

        def compile_one(src, obj):
            flags = B.SOURCE_FLAGS.get(os.path.basename(src), [])
            r = subprocess.run([cc, *B.HIP_FLAGS, *flags, "-O1", *san, "-c", src, "-o", obj],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]

        with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            for f in [ex.submit(compile_one, s, o) for s, o in zip(srcs, objs)]:
                f.result()
        exe = os.path.join(tmp, "host_checks")
        r = subprocess.run([cc, *B.HIP_FLAGS, *san, *objs, "-o", exe, *B.LINK_LIBS], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
        assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
        assert "host checks ok" in r.stdout
