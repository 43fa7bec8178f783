"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

boys_oracle.c is built with -fsanitize=address,undefined into a temporary library, loaded
by a child Python process with the ASan runtime preloaded, and driven through every entry
point the tests use, at small sizes: each class at orders 0, 1, 16 and 36 on arguments that
include zeros, subnormals, both sides of every cut-off, +inf, NaN, negatives and 1e300;
the exact function; the binary128 approximant; the split option; the consumer on ragged and
empty pair lists.  Any sanitizer report aborts the child and fails the test.
"""
import os
import shutil
import subprocess
import sys

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
from oracle import oracle as orc
from paper_2504_07637_amd import inputs
orc._lib = orc._load(sys.argv[1])
x = np.concatenate([inputs.integral_args(3000, seed=5), inputs.uniform_mix(1024, seed=6),
                    [0.0, -0.0, 5e-324, 1e-300, 2.0 ** -54, np.inf, np.nan, -1.0, 1e300,
                     1.7e308]])
for n in (0, 1, 16, 36):
    for cls in ("fp64", "fp32", "fp32x"):
        z = orc.record(cls, n)["z"]
        xx = np.concatenate([x, [z, np.nextafter(z, 0), np.nextafter(z, 1e9)]])
        if cls == "fp64":
            orc.approx_f64(xx, n)
            if n < 36:
                orc.approx_f64(xx, n + 1)
        elif cls == "fp32":
            orc.approx_mixed(xx, n)
            orc.approx_single(xx, n)
        else:
            orc.approx_f32x(xx, n)
    orc.exact(x[:200], n)
    orc.approx_exact_n(x[:200], n, "fp64")
orc.approx_split(x, 16, 6)
orc.exp_neg(x)
c, e, w = inputs.s_basis(4, 2, 3, seed=5, fixed_prim=False)
pairs, start = inputs.shell_pairs(c, e, w)
orc.eri_ssss(pairs, start, pairs, start, 8)
orc.eri_ssss(pairs, start, pairs[:, :0], np.array([0], dtype=np.int32), 3)
print("sanitized oracle ok")
"""


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not asan or not os.path.isabs(asan):
        pytest.skip("no libasan for the host compiler")
    lib = tmp_path / "liboracle_sanitized.so"
    cmd = [gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-o", str(lib),
           os.path.join(REPO, "oracle", "boys_oracle.c"), "-lquadmath", "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    out = subprocess.run([sys.executable, "-c", DRIVER, str(lib), REPO], env=env,
                         capture_output=True, text=True, timeout=600)
    assert out.returncode == 0 and "sanitized oracle ok" in out.stdout, \
        out.stdout[-2000:] + out.stderr[-4000:]
