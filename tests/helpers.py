"""Shared helpers of the tests: layout conversions, error norms, and copies
of the oracle with one planted mistake (for checking that a pin catches it)."""
import importlib.util
import os
import shutil

import numpy as np


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0)


def absolute_positions(cell, off, n, d):
    """FP64 absolute positions [3, np] of (cell, offset) pairs."""
    c = np.asarray(cell, dtype=np.int64)
    idx = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
    return np.stack([(idx[a] + np.asarray(off[a], dtype=np.float64)) * d[a] for a in range(3)])


def periodic_delta(x1, x0, L):
    """x1 - x0 mapped to (-L/2, L/2] per axis."""
    L = np.asarray(L, dtype=np.float64)[:, None]
    dx = x1 - x0
    return dx - L * np.round(dx / L)


def by_id(ids, *arrays):
    order = np.argsort(ids, kind="stable")
    return [a[..., order] for a in arrays]


def oracle_mutant(tmp_path, name, c_edit=None, py_edit=None):
    """A copy of the oracle package with one edit (old, new) in oracle.c
    and/or oracle.py, built and imported as a separate module."""
    from oracle import oracle as O

    src_dir = os.path.dirname(O.__file__)
    d = tmp_path / name
    d.mkdir()
    for f in ("oracle.c", "denoise.c", "circ.c", "oracle.py"):
        shutil.copy(os.path.join(src_dir, f), d / f)
    for fname, edit in (("oracle.c", c_edit), ("oracle.py", py_edit)):
        if edit:
            src = (d / fname).read_text()
            old, new = edit
            assert src.count(old) == 1, (fname, old)
            (d / fname).write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", d / "oracle.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.build(force=True)
    return mod
