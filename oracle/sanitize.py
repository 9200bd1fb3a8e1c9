"""Run the oracle's pin tests against an AddressSanitizer + UndefinedBehavior
Sanitizer build of oracle.c (CPU only).

    python -m oracle.sanitize [extra pytest arguments]

Builds oracle/liboracle_asan.so from the same source with
-fsanitize=address,undefined, then runs tests/test_oracle_*.py in a child
Python process with the ASan runtime preloaded (Python itself is not
instrumented, so the runtime must come first).  Leak checking is off: the
interpreter's own allocations are not the oracle's.  Any report aborts the
child and fails the run.  Not for the GPU machine: it only exercises the CPU
oracle, and it does not override a preload that the environment already
sets.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def main(argv=None) -> int:
    argv = list(sys.argv[1:] if argv is None else argv)
    if os.environ.get("LD_PRELOAD"):
        print("sanitize: LD_PRELOAD is already set in this environment; not overriding it", file=sys.stderr)
        return 2
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        print("sanitize: gcc has no libasan.so", file=sys.stderr)
        return 2
    env = dict(os.environ, FACERT_ORACLE_SANITIZE="1", LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    subprocess.check_call([sys.executable, "-c", "import oracle; oracle.build(force=True)"], cwd=ROOT,
                          env={k: v for k, v in env.items() if k != "LD_PRELOAD"})
    tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *tests, *argv]
    return subprocess.call(cmd, cwd=ROOT, env=env)


if __name__ == "__main__":
    sys.exit(main())
