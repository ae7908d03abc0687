"""The oracle's C direct sum (oracle/direct.c) built as a standalone program with
the host sanitizers (gcc: AddressSanitizer with UndefinedBehaviorSanitizer, and
ThreadSanitizer for its worker threads), run on small inputs with several
threads and every kernel: no report, and the values of the regular build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import direct
from workloads.rng import SplitMix64

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MAIN = os.path.join(ROOT, "tests", "sanitize", "oracle_direct_main.c")
SANITIZERS = {
    "address,undefined": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                          "-static-libasan", "-static-libubsan"],
    "thread": ["-fsanitize=thread", "-static-libtsan"],
}


def _build(tmp, name):
    exe = os.path.join(tmp, "oracle_direct_" + name.replace(",", "_"))
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-pthread", *SANITIZERS[name],
           direct.SRC, MAIN, "-o", exe, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip(f"gcc cannot build with -fsanitize={name}: {r.stderr[-300:]}")
    return exe


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
@pytest.mark.parametrize("name", list(SANITIZERS))
def test_oracle_direct_sum_is_clean_under_sanitizers(tmp_path, name):
    exe = _build(str(tmp_path), name)
    g = SplitMix64(91)
    ns, nt = 700, 333
    src = [g.uniform(ns, -1, 1) for _ in range(3)] + [g.uniform(ns, -1, 1), g.uniform(ns, 0, 1)]
    tgt = [g.uniform(nt, -1.2, 1.2) for _ in range(3)] + [g.uniform(nt, -1, 1)]
    tgt[0][:5] = src[0][:5]  # targets that coincide with sources
    tgt[1][:5] = src[1][:5]
    tgt[2][:5] = src[2][:5]
    inp = tmp_path / "in.bin"
    np.concatenate(src + tgt).astype(np.float64).tofile(inp)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    for kernel, code in direct.KERNELS.items():
        out = tmp_path / f"out_{kernel}.bin"
        r = subprocess.run([exe, str(inp), str(out), str(code), str(ns), str(nt), "4", "1.3",
                            "0.7"], capture_output=True, text=True, env=env, timeout=120)
        if name == "thread" and "unexpected memory mapping" in r.stderr:
            pytest.skip("ThreadSanitizer cannot run under this kernel's address layout")
        assert r.returncode == 0, (kernel, r.returncode, r.stderr[-2000:])
        assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-2000:]
        got = np.fromfile(out, dtype=np.float64)
        ref, ab = direct.direct_sum(kernel, *src, *tgt, kappa=1.3, alpha=0.7, threads=4,
                                    return_abs=True)
        assert np.allclose(got[:nt], ref, rtol=0, atol=1e-14 * ab.max()), kernel
        assert np.allclose(got[nt:], ab, rtol=1e-14), kernel
