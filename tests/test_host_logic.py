"""Host-side logic that needs no GPU: the C3 scan generator, size classes,
autotuner feasibility, the denoiser parameter layout and its binomial start,
and the benchmark's one-GPU guard."""
import subprocess
import sys

import numpy as np

from oracle import oracle as O
from paper_1204_0838_amd import autotune, c4, workloads


def test_c3_members_follow_the_scan_recipe():
    m = workloads.c3_members()
    assert len(m) == 64
    for cfg in m:
        nx, ny, nz = cfg["n"]
        assert 64 <= nx <= 256 and 32 <= ny <= 64 and 32 <= nz <= 64
        assert nx % 8 == 0 and ny % 8 == 0 and nz % 8 == 0
        assert 2.0 <= cfg["laser"]["a0"] <= 5.0 and 0.5 <= cfg["plasma"]["n_plateau"] <= 2.0
        assert cfg["d"] == workloads.C1["d"] and cfg["solver"] == "pd" and cfg["steps"] == 200
    cells = sum(c["n"][0] * c["n"][1] * c["n"][2] for c in m)
    assert 2.0e7 < cells < 2.8e7                      # about 2.36e7 expected
    assert m[0]["n"] == workloads.c3_members(1)[0]["n"]   # instance i depends on its own seed only
    assert {workloads.size_class(c) for c in m} == {"S", "M", "L"}


def test_window_start_and_initial_load_of_c1():
    assert workloads.window_start_step(workloads.C1) == 486
    assert workloads.initial_particles(workloads.C1) == (512 - 3 - 8) * 256 * 256 * 8


def test_autotuner_space_respects_lds():
    assert autotune.feasible(autotune.DEFAULT)
    # fields: 14 z-planes of 14x14 words padded to 200 (8 banks per z step), 6 components x 4 B;
    # current: 15 z-planes of 15x15 padded to 232 (8 mod 16 int64 words), 3 components x 8 B
    assert autotune.lds_bytes(dict(tile=(8, 8, 8), guard=1)) == 14 * 200 * 24 + 15 * 232 * 24 == 150720
    assert not autotune.feasible(dict(tile=(16, 8, 8), guard=2))
    assert autotune.class_key("M", workloads.C1) == "batch|M|ppc8|pd"


def test_denoiser_parameter_layout_round_trip():
    from paper_1204_0838_amd import pic

    rng = np.random.default_rng(1)
    P = [rng.standard_normal(s) for s in ((32, 3, 3, 3, 3), (32,), (32, 32, 3, 3, 3), (32,), (3, 32, 3, 3, 3), (3,))]
    w, b = pic.pack_params(P)
    assert w.size == pic.N_WEIGHTS and b.size == pic.N_BIASES
    for a, c in zip(P, pic.unpack_params(w, b)):
        assert np.array_equal(a.astype(np.float32), c)


def test_binomial_start_is_the_filter():
    P = c4.binomial_init(np.random.default_rng(2))
    rng = np.random.default_rng(3)
    J = rng.standard_normal((3, 4, 5, 6))
    g = O.make_grid((6, 5, 4), (0.25, 0.5, 0.5), 0.25)
    Jout, _ = O.denoise(J, [0.1, 0.2, 0.3], P, d=(0.25, 0.5, 0.5), round_bf16=False)
    assert np.abs(Jout - O.binomial(g, J)).max() < 1e-14


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_autotuner_knob_variants_change_one_knob_and_fit():
    """The whole-run search times every one-knob change of the default that
    fits in LDS: each variant differs from the default in exactly one knob,
    every value of every knob appears unless it does not fit, and none
    repeats the default."""
    base = dict(autotune.DEFAULT)
    vs = autotune.knob_variants(base)
    seen = {k: set() for k in autotune.SPACE}
    for c in vs:
        diff = [k for k in autotune.SPACE if c[k] != base[k]]
        assert len(diff) == 1
        assert autotune.feasible(c)
        seen[diff[0]].add(c[diff[0]] if diff[0] != "tile" else tuple(c["tile"]))
    for k, values in autotune.SPACE.items():
        for v in values:
            c = dict(base)
            c[k] = v
            if c != base and autotune.feasible(c):
                assert (tuple(v) if k == "tile" else v) in seen[k]
