"""Host-side checks of the C ABI: the library loads without a GPU, exports every
symbol include/pic.h declares, and validates descriptors (no GPU calls)."""
import ctypes
import os
import re

import pytest

from paper_1204_0838_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(pic_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = pic.lib()
    declared = _declared_symbols()
    assert len(declared) >= 15
    for name in sorted(declared):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert declared <= set(pic._SIGS), "binding lacks a declared entry point"


def _desc(**kw):
    base = dict(n=(64, 32, 32), d=(0.2, 0.2, 0.2), dt=0.0577350269, solver="yee")
    base.update(kw)
    return pic.make_desc(**base)


def test_validation_accepts_paper_shaped_grids():
    assert pic.validate(_desc())[0] == pic.PIC_OK
    pd = _desc(n=(512, 256, 256), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd", bc_x=1)
    assert pic.validate(pd)[0] == pic.PIC_OK


@pytest.mark.parametrize("kw,fragment", [
    (dict(solver="pd", d=(0.5, 0.25, 0.5), dt=0.25), "dx <= dy"),
    (dict(solver="pd", d=(0.25, 0.5, 0.5), dt=0.3), "c dt <= dx"),
    (dict(dt=0.2), "Courant"),
    (dict(n=(64, 3, 32)), "at least 4"),
    (dict(d=(0.2, -0.2, 0.2)), "positive"),
    (dict(dt=float("nan")), "positive"),
    (dict(jpost=7), "post-processing"),
    (dict(tile=(128, 8, 8)), "tile"),
    (dict(tile=(8, 2, 8)), "tile below 3"),
])
def test_validation_rejects_bad_descriptors(kw, fragment):
    st, msg = pic.validate(_desc(**kw))
    assert st == pic.PIC_EINVAL
    assert fragment in msg


def test_autotuner_lds_model_matches_the_library():
    """The autotuner's LDS footprint (padded tile planes) decides feasibility
    exactly as the library's own check does, for every tile shape and guard."""
    from paper_1204_0838_amd import autotune
    for tx in range(3, 17):
        for ty in (3, 4, 6, 8, 12, 16):
            for tz in (3, 4, 8, 16):
                for guard in range(4):
                    st, msg = pic.validate(_desc(n=(64, 64, 64), tile=(tx, ty, tz), guard=guard))
                    lib_ok = st == pic.PIC_OK
                    assert lib_ok or "LDS" in msg, msg
                    assert lib_ok == autotune.feasible(dict(tile=(tx, ty, tz), guard=guard)), (tx, ty, tz, guard)


def test_workspace_size_grows_with_particles_and_rejects_invalid():
    d = _desc()
    a = pic.workspace_bytes(d, 1000)
    b = pic.workspace_bytes(d, 100000)
    assert 0 < a < b
    assert pic.workspace_bytes(_desc(dt=1.0), 10) == 0


def test_absorbing_layer_size_and_limits():
    d = _desc(n=(64, 48, 40))

    def nbytes(layers):
        return int(pic.lib().pic_pml_bytes(ctypes.byref(d), ctypes.byref(pic.PmlDesc(layers, 0))))

    # coefficient table (16 L floats) and four arrays per transverse axis over
    # the 2 L layer cells, each part rounded up to 256 bytes
    up = lambda b: (b + 255) // 256 * 256
    L = 16
    want = up(16 * L * 4) + 4 * up(64 * 2 * L * 40 * 4) + 4 * up(64 * 48 * 2 * L * 4)
    assert nbytes(L) == want
    assert nbytes(7) == 0                      # too thin for the particle margin
    assert nbytes(20) == 0                     # 2 L + 1 > n[2] = 40
    assert nbytes(19) > 0
    assert int(pic.lib().pic_pml_bytes(ctypes.byref(_desc(dt=1.0)), ctypes.byref(pic.PmlDesc(8, 0)))) == 0
