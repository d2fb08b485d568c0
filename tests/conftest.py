import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libgsr.so")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(config, items):
    have_gpu = False
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU in this environment")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    """The gradient bar's audit: per test case and parameter group, how many
    elements the plain relative bar admits and how many need each further
    tolerance term (see tests/helpers.py AUDIT_KEYS). Also written as JSON
    lines to $GSR_AUDIT_OUT when that is set."""
    try:
        from tests import helpers
    except Exception:
        return
    log = helpers.AUDIT_LOG
    if not log:
        return
    tr = terminalreporter
    tr.write_sep("-", "gradient bar audit (elements admitted per tolerance term)")
    tr.write_line("%-28s %-9s %8s %8s %8s %8s %8s %8s %8s %6s" % ("case", "group", "n", "nonzero",
                                                                 *helpers.AUDIT_KEYS))
    for r in log:
        tr.write_line("%-28s %-9s %8d %8d %8d %8d %8d %8d %8d %6d" % (
            str(r["case"])[:28], r["group"], r["n"], r.get("nz", r["n"]), *[r[k] for k in helpers.AUDIT_KEYS]))
    path = os.environ.get("GSR_AUDIT_OUT")
    if path:
        import json
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            for r in log:
                f.write(json.dumps(r) + "\n")
