"""Checkpoint / resume through the C ABI (pic_checkpoint_bytes, pic_copy_out,
pic_copy_in): a moving-window laser-wakefield run interrupted at step k,
copied to the host, restored into a fresh context and continued, ends bit
for bit where the uninterrupted run ends (fields, and particles by id),
both before the window moves (laser source active) and after (window
shifted, plasma injected at the leading edge).  Also the refusals: another
grid, a truncated blob, too small a capacity, a split-path step in
progress."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402

N = (48, 12, 12)
D = (0.25, 0.5, 0.5)
DT = 0.25
PLASMA = dict(x_start=8.0, ramp=10.0, n_plateau=1.0, ppc=(2, 2, 2))
LASER = dict(a0=2.0, omega0=1.508, waist=1.5, fwhm=1.0, t_peak=4.0, t_end=8.0, yc=3.0, zc=3.0, src_x=2)
START, STEPS = 32, 48
CAP = N[0] * N[1] * N[2] * 8 + STEPS * N[1] * N[2] * 8


def _context(n=N, cap=CAP, load=True, **kw):
    sim = pic.Simulation(n, D, DT, solver="pd", bc_x=1, max_particles=cap, **kw)
    sim.add_empty_species(cap)
    sim.set_plasma(0, **PLASMA)
    if load:
        sim.inject_plasma(0, 0, n[0] - 3)
    sim.set_laser(**LASER)
    sim.set_window(START)
    return sim


def _by_id(sim):
    p = sim.particles_host(0)
    live = p["cell"] >= 0
    o = np.argsort(p["id"][live])
    return {k: (v[..., live][..., o]) for k, v in p.items()}


@pytest.mark.parametrize("k", [20, 40])
def test_resume_is_bit_exact(k):
    print(f"checkpoint resume at step {k} of {STEPS}", flush=True)
    ref = _context(tile=(8, 4, 4), sort_interval=3)
    ref.step(STEPS)
    first = _context(tile=(8, 4, 4), sort_interval=3)
    first.step(k)
    blob = first.copy_out()
    sh_k, org_k = first.window_state()
    del first
    torch.cuda.synchronize()
    # a fresh context with another tiling: the stored state fixes the result
    second = _context(load=False, tile=(8, 8, 4), sort_interval=2)
    second.copy_in(blob)
    assert second.window_state() == (sh_k, org_k)
    assert second.reduce()["step"] == k
    second.step(STEPS - k)
    assert second.window_state() == ref.window_state()
    for a, b in ((ref.E, second.E), (ref.B, second.B), (ref.J, second.J)):
        assert torch.equal(a, b)
    pr, ps = _by_id(ref), _by_id(second)
    assert len(pr["id"]) > 1000
    for key in ("id", "cell", "off", "u", "w"):
        assert np.array_equal(pr[key], ps[key]), key
    # the blob's size is what the header's counts imply
    nb = 160 + 9 * N[0] * N[1] * N[2] * 4
    assert len(blob) >= nb


def test_checkpoint_refusals():
    print("checkpoint refusals", flush=True)
    a = _context()
    a.step(3)
    blob = a.copy_out()
    other = _context(n=(40, 12, 12), load=False)
    with pytest.raises(pic.PicError) as e:
        other.copy_in(blob)
    assert e.value.status == pic.PIC_EINVAL
    fresh = _context(load=False)
    with pytest.raises(pic.PicError) as e:
        fresh.copy_in(blob[:-4])
    assert e.value.status == pic.PIC_EINVAL
    small = _context(load=False, cap=1000)
    with pytest.raises(pic.PicError) as e:
        small.copy_in(blob)
    assert e.value.status == pic.PIC_ENOMEM
    a.gather_push(0)
    with pytest.raises(pic.PicError) as e:
        a.copy_out()
    assert e.value.status == pic.PIC_ESTATE
    a.deposit(0)
    a.field_step()
    assert len(a.copy_out()) > 0
