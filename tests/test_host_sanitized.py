"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(host-only instrumentation, no GPU needed): build_sanitized() compiles every
source with the sanitizers on the host side and links tests/host_check.cpp,
which drives the C ABI through reference elements of every degree, mesh
building, geometry queries, workspace sizing and the error paths."""
import os
import subprocess

import numpy as np
import pytest

from workloads.mesh import kuhn_periodic_mesh


@pytest.mark.slow
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    from paper_1711_01175_amd import build as b
    exe = b.build_sanitized()
    EToV, VXYZ = kuhn_periodic_mesh(3, shuffle_seed=7)
    (tmp_path / "K.txt").write_text(str(EToV.shape[0]))
    np.ascontiguousarray(EToV, np.int64).tofile(tmp_path / "EToV.bin")
    np.ascontiguousarray(VXYZ, np.float64).tofile(tmp_path / "VXYZ.bin")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0
    assert "all checks passed" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
