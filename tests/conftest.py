import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def load_golden(name):
    """Read a 'name k row col re im' fixture into a dict of complex arrays."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name)
    rows = []
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        p = line.split()
        rows.append((p[0], int(p[1]), int(p[2]), int(p[3]), float(p[4]), float(p[5])))
    out = {}
    for key in sorted({r[0] for r in rows}):
        sel = [r for r in rows if r[0] == key]
        nt1 = max(r[1] for r in sel) + 1
        n = max(max(r[2], r[3]) for r in sel) + 1
        a = np.zeros((nt1, n, n), dtype=np.complex128)
        for _, k, i, j, re, im in sel:
            a[k, i, j] = re + 1j * im
        out[key] = a
    return out


@pytest.fixture
def golden():
    return load_golden


def pytest_collection_modifyitems(config, items):
    """GPU tests are skipped (not passed) where no GPU is visible."""
    try:
        import torch
        have_gpu = torch.cuda.is_available()
    except Exception:  # pragma: no cover
        have_gpu = False
    if have_gpu:
        return
    skip = pytest.mark.skip(reason="no GPU visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
