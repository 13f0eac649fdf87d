"""The oracle's own pins rerun against a build of the oracle with
AddressSanitizer and UndefinedBehaviorSanitizer (gcc, every finding fatal):
no out-of-bounds access, use after free or undefined arithmetic anywhere the
pins reach (models, gradients, TV forms, prior, Philox, MH, ensemble,
askadam with its optimisers and stopping rules)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["test_oracle_models.py", "test_oracle_rng.py", "test_oracle_mh.py",
        "test_oracle_regularisers.py", "test_oracle_tv_fit.py", "test_oracle_optim_pins.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="gcc AddressSanitizer not available")
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-std=c11", "-fopenmp", "-fPIC",
           "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "gacelle_oracle.c"), "-o", str(lib), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, GACELLE_ORACLE_LIB=str(lib),
               LD_PRELOAD=" ".join(p for p in (_runtime("libasan.so"), _runtime("libubsan.so"))
                                   if p),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *[os.path.join(ROOT, "tests", f) for f in PINS]],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-6000:]
