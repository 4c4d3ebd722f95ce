import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """Per-field error of every GPU-vs-oracle parity check of the run: relative
    2-norm (and max-norm) error per field against the bar the check used.  Set
    JFNK_ERROR_TABLE to a path to also write the table there."""
    try:
        from gpu_util import RECORDS
    except ImportError:
        return
    if not RECORDS:
        return
    lines = ["per-field error of each parity check, GPU against the FP64 oracle unless the check names another "
             "reference (relative 2-norm / max-norm; fields u[, v], w, p', theta')",
             f"{'check':<64} {'bar':>8}  per field"]
    for what, tol, e2, em in RECORDS:
        cells = "  ".join(f"{a:.1e}/{b:.1e}" for a, b in zip(e2, em))
        lines.append(f"{what[:64]:<64} {tol:>8.0e}  {cells}")
    worst = max((max(e2) / tol, what) for what, tol, e2, em in RECORDS if tol > 0)
    lines.append(f"{len(RECORDS)} checks; largest error / bar {worst[0]:.2e} ({worst[1]})")
    text = "\n".join(lines)
    terminalreporter.write_sep("=", "per-field parity errors")
    terminalreporter.write_line(text)
    path = os.environ.get("JFNK_ERROR_TABLE")
    if path:
        with open(path, "w") as fh:
            fh.write(text + "\n")
