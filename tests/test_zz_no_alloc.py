"""The allocation-free continuity check (pic_continuity_noalloc) through the
C ABI against pic_continuity on the same state: the same residual (both sum
the FP64 density with atomics, so to a tolerance far below the check's own
1e-6 max|J| bar) and the same max |J| (bit for bit), on two calls in a row
where the second has a smaller grid and fewer particles, so the second call
runs on the scratch the first one left.  Grids beyond the scratch's 2^21
cells are refused."""
import numpy as np
import pytest

from paper_1204_0838_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402


def _state(n, ppc, seed, steps):
    g = inputs.Grid(n, (0.25, 0.5, 0.5), 0.2, solver="pd")
    pl = inputs.uniform_random_plasma(g, ppc=ppc, seed=seed, temperature_ev=20000.0, ux_amp=0.1)
    sim = pic.Simulation(n, g.d, g.dt, solver="pd", max_particles=pl.count)
    sim.add_particles(pl)
    sim.step(steps)
    sim.gather_push(0)
    sim.deposit(0)
    return sim


@pytest.mark.parametrize("order", ["large_then_small"])
def test_noalloc_continuity_matches_the_workspace_version(order):
    for n, ppc, seed in (((64, 32, 24), 4, 3), ((24, 12, 16), 2, 5)):
        print(f"continuity_noalloc on {n}, {ppc} ppc", flush=True)
        sim = _state(n, ppc, seed, steps=3)
        r_ws, j_ws = sim.continuity(0)
        r_na, j_na = sim.continuity_noalloc(0)
        assert j_ws > 0 and j_na == j_ws
        assert r_ws <= 1e-6 * j_ws and r_na <= 1e-6 * j_ws
        assert abs(r_na - r_ws) <= 1e-9 * j_ws
        sim.field_step()
        sim.close()


def test_noalloc_continuity_refuses_grids_beyond_its_scratch():
    n = (160, 128, 128)          # 2.6e6 cells > 2^21
    sim = pic.Simulation(n, (0.25, 0.5, 0.5), 0.2, solver="pd", max_particles=16)
    sim.add_empty_species(16)
    with pytest.raises(pic.PicError) as e:
        sim.continuity_noalloc(0)
    assert e.value.status == pic.PIC_EINVAL and "2097152" in str(e.value)
    sim.close()
