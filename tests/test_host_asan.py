"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds tests/host_asan/epic_asan_check.cpp against library objects whose host
side is instrumented (device code compiled as usual) and runs its host mode:
the host-only helpers, argument errors and the plan-creation error path.  The
same executable's `gpu` mode drives plans through every host path around the
kernels, band model and teardown included, on a machine with a GPU."""
import os
import subprocess

import pytest


def test_host_code_clean_under_asan_ubsan(tmp_path):
    from paper_1603_02126_amd import build
    try:
        exe = build.build_asan_check(str(tmp_path / "asan"))
    except RuntimeError as err:   # toolchain without the sanitizer runtimes
        if "libclang_rt.asan" in str(err) or "cannot find" in str(err):
            pytest.skip(f"sanitizer runtime missing: {err}")
        raise
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe, "host"], capture_output=True, text=True, timeout=300, cwd=str(tmp_path), env=env)
    out = r.stdout + r.stderr
    print(out)
    assert "AddressSanitizer" not in out and "runtime error" not in out and "LeakSanitizer" not in out
    assert r.returncode == 0, out
    assert "host: 0 failure(s), leak check clean" in r.stdout
