"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc -fsanitize=address,undefined, no recovery) runs the oracle pins in a
child process: any out-of-bounds access, use after free, signed overflow,
misaligned access or other undefined behaviour in the C oracle fails it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _libasan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _libasan()
    if asan is None:
        pytest.skip("gcc has no libasan here")
    sys.path.insert(0, ROOT)
    import oracle
    lib = oracle.build(force=True, out=str(tmp_path / "libsail_oracle_asan.so"), sanitize=True)
    env = dict(os.environ)
    env.update(SAIL_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    # the pins that drive the C oracle (the rocRAND cross-check needs its own build and is left out)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", "not rocrand",
                        os.path.join(ROOT, "tests", "test_workloads.py")],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    print(r.stdout.strip().splitlines()[-1], flush=True)
