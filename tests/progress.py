"""Progress lines for long tests: printed as they happen, also while pytest captures output
(a run that stays silent for minutes is indistinguishable from a hung one)."""
import contextlib
import sys
import time

CAPTURE = None   # pytest's capture manager, set by conftest
_T0 = time.perf_counter()


def say(*a):
    ctx = CAPTURE.global_and_fixture_disabled() if CAPTURE is not None else contextlib.nullcontext()
    with ctx:
        print(f"[{time.perf_counter() - _T0:7.1f} s]", *a, flush=True)
        sys.stdout.flush()
