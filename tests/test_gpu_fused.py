"""The production path (cell sort + fused LDS-tiled gather/push/deposit) against
the split kernels: identical results bit for bit, whatever the tile shape,
guard, in-tile interleave or sort interval (integer current sums make the
result independent of particle order and of which path handled a particle)."""
import numpy as np
import pytest

from paper_1204_0838_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import pic  # noqa: E402


def _pair(grid, pl, **kw):
    a = pic.Simulation(grid.n, grid.d, grid.dt, solver=grid.solver, max_particles=pl.count, **kw)
    b = pic.Simulation(grid.n, grid.d, grid.dt, solver=grid.solver, max_particles=pl.count)
    a.add_particles(pl)
    b.add_particles(pl)
    return a, b


def _assert_same(a, b):
    for fa, fb in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert torch.equal(fa, fb)
    pa, pb = a.particles_host(0), b.particles_host(0)
    assert pa["id"].shape == pb["id"].shape
    ia, ib = np.argsort(pa["id"]), np.argsort(pb["id"])
    assert np.array_equal(pa["id"][ia], pb["id"][ib])
    assert np.array_equal(pa["u"][:, ia], pb["u"][:, ib])
    assert np.array_equal(pa["off"][:, ia], pb["off"][:, ib])
    assert np.array_equal(pa["cell"][ia], pb["cell"][ib])


CASES = [
    dict(tile=(8, 8, 8), guard=1, interleave=17, sort_interval=2, threads=512),
    dict(tile=(4, 4, 4), guard=0, interleave=1, sort_interval=3, threads=256),
    dict(tile=(8, 4, 4), guard=2, interleave=5, sort_interval=1, threads=1024),
    dict(tile=(5, 3, 7), guard=1, interleave=0, sort_interval=4, threads=512),
    dict(tile=(8, 8, 8), guard=1, interleave=0, sort_interval=3, threads=1024),
]


@pytest.mark.parametrize("kw", CASES, ids=lambda k: "t{}g{}i{}s{}".format(k["tile"][0], k["guard"],
                                                                         k["interleave"], k["sort_interval"]))
def test_fused_step_equals_split_bit_exact_yee(kw):
    grid = inputs.Grid(n=(13, 10, 9), d=(0.3, 0.25, 0.35), dt=0.1)
    pl = inputs.uniform_random_plasma(grid, ppc=6, seed=41, temperature_ev=30000.0, ux_amp=0.1)
    a, b = _pair(grid, pl, **kw)
    a.step(6)
    for _ in range(6):
        b.gather_push(0)
        b.deposit(0)
        b.field_step()
    _assert_same(a, b)


def test_fused_step_equals_split_bit_exact_pd_larger():
    grid = inputs.Grid(n=(40, 24, 20), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=8, seed=43, temperature_ev=100000.0, ux_amp=0.3)
    a, b = _pair(grid, pl, tile=(8, 8, 8), guard=1, interleave=17, sort_interval=2)
    a.step(5)
    for _ in range(5):
        b.gather_push(0)
        b.deposit(0)
        b.field_step()
    _assert_same(a, b)


def test_retiling_a_live_run_does_not_change_results():
    """pic_set_tiling between steps (what the autotuner does) keeps bit-exactness."""
    grid = inputs.Grid(n=(32, 16, 16), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=8, seed=45, temperature_ev=80000.0, ux_amp=0.2)
    a, b = _pair(grid, pl)
    tilings = [dict(tile=(8, 8, 8), guard=1, threads=512, interleave=8, sort_interval=2),
               dict(tile=(8, 4, 4), guard=2, threads=1024, interleave=4, sort_interval=3),
               dict(tile=(16, 4, 4), guard=0, threads=256, interleave=1, sort_interval=1),
               dict(tile=(4, 4, 4), guard=1, threads=512, interleave=16, sort_interval=4)]
    for t in tilings:
        a.set_tiling(**t)
        a.step(2)
    for _ in range(2 * len(tilings)):
        b.gather_push(0)
        b.deposit(0)
        b.field_step()
    _assert_same(a, b)


def test_sort_groups_particles_by_tile_and_keeps_them():
    grid = inputs.Grid(n=(24, 16, 12), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=4, seed=44)
    T = (8, 4, 6)
    sim = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", tile=T, max_particles=pl.count)
    sim.add_particles(pl)
    sim.sort(0)
    got = sim.particles_host(0)
    assert np.array_equal(np.sort(got["id"]), np.sort(pl.id))
    order = np.argsort(got["id"])
    assert np.array_equal(got["cell"][order], pl.cell)
    assert np.array_equal(got["off"][:, order], pl.off)
    c = got["cell"].astype(np.int64)
    nx, ny, _ = grid.n
    tx, ty, tz = (c % nx) // T[0], ((c // nx) % ny) // T[1], (c // (nx * ny)) // T[2]
    tile = tx + 3 * (ty + 4 * tz)
    assert np.all(np.diff(tile) >= 0)   # tiles are contiguous and in order


def _brick_key(c, n, T):
    """(tile, in-tile key) of cells c: 8x2x4-cell bricks, x fastest, then z,
    then y inside a brick, bricks y-major (the order the sort stores tiles of
    8 x 2m x 4k cells in)."""
    x, y, z = c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])
    nt = [(n[d] + T[d] - 1) // T[d] for d in range(3)]
    tile = x // T[0] + nt[0] * (y // T[1] + nt[1] * (z // T[2]))
    lx, ly, lz = x % T[0], y % T[1], z % T[2]
    return tile, lx + 8 * (lz % 4) + 32 * (ly % 2) + 64 * (ly // 2 + (T[1] // 2) * (lz // 4))


def test_sort_stores_tiles_in_level_order():
    """Default storage (level order): inside each tile, level r holds the
    (r + 1)-th particle of every cell with more than r particles, cells in
    brick-key order, levels one after another -- checked slot by slot against
    the order computed here from the cell counts, on a plasma of uneven
    counts (Poisson per cell, one dense slab) with ragged tiles."""
    grid = inputs.Grid(n=(24, 20, 16), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    ncell = 24 * 20 * 16
    rng = np.random.default_rng(46)
    cell = rng.integers(0, ncell, 6 * ncell)                 # Poisson counts
    slab = rng.integers(0, ncell, 6 * ncell)
    cell = np.concatenate([cell, slab[(slab % 24 >= 8) & (slab % 24 < 12)]]).astype(np.int32)   # a dense slab
    off = rng.random((3, cell.size)).astype(np.float32)
    u = np.zeros((3, cell.size), np.float32)
    w = np.full(cell.size, 0.1, np.float32)
    ids = np.arange(cell.size, dtype=np.int32)
    T = (8, 8, 8)
    sim = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", tile=T, max_particles=cell.size)
    sim.add_species(cell, off, u, w, ids)
    sim.sort(0)
    got = sim.particles_host(0)
    assert np.array_equal(np.sort(got["id"]), ids)
    tile, key = _brick_key(got["cell"].astype(np.int64), grid.n, T)
    ct, ck = _brick_key(cell.astype(np.int64), grid.n, T)
    want_t, want_k = [], []
    for t in range(int(ct.max()) + 1):
        cnt = np.bincount(ck[ct == t], minlength=512)
        for r in range(int(cnt.max()) if cnt.size else 0):
            ks = np.nonzero(cnt > r)[0]
            want_t.append(np.full(ks.size, t))
            want_k.append(ks)
    per_cell = np.bincount(cell, minlength=ncell)
    assert per_cell.max() > 2 * np.median(per_cell)              # counts are uneven
    assert np.array_equal(tile, np.concatenate(want_t))
    assert np.array_equal(key, np.concatenate(want_k))


def _level_order(cells, n, T):
    """(tile, in-tile key) sequence of the level order of the given cells."""
    ct, ck = _brick_key(cells.astype(np.int64), n, T)
    want_t, want_k = [], []
    for t in range(int(ct.max()) + 1):
        cnt = np.bincount(ck[ct == t], minlength=512)
        for r in range(int(cnt.max()) if cnt.size else 0):
            ks = np.nonzero(cnt > r)[0]
            want_t.append(np.full(ks.size, t))
            want_k.append(ks)
    return np.concatenate(want_t), np.concatenate(want_k)


def test_resort_keeps_level_order():
    """A re-sort (particles still in the last sort's tile ranges: counted tile
    by tile, those that stayed in their tile placed by the level pass, the
    others scattered) stores the same level order as a first sort: after
    steps that move particles across cells and tiles, and with more
    particles appended by hand, slot by slot against the order computed from
    the new cells; also for a tile too dense to be staged in LDS (more than
    8192 particles)."""
    grid = inputs.Grid(n=(24, 16, 16), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    ncell = 24 * 16 * 16
    rng = np.random.default_rng(48)
    cell = rng.integers(0, ncell, 5 * ncell)
    dense = np.full(9000, 3 + 24 * (2 + 16 * 3))               # one cell of tile 0 over the staging size
    cell = np.concatenate([cell, dense]).astype(np.int32)
    off = rng.random((3, cell.size)).astype(np.float32)
    u = (0.6 * rng.standard_normal((3, cell.size))).astype(np.float32)   # ~0.3-0.6 cells per step
    w = np.full(cell.size, 0.01, np.float32)
    ids = np.arange(cell.size, dtype=np.int32)
    T = (8, 8, 8)
    sim = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", tile=T, sort_interval=100,
                         max_particles=cell.size)
    sim.add_species(cell, off, u, w, ids)
    sim.sort(0)                                                   # first sort
    for _ in range(3):
        sim.gather_push(0)                                        # moves particles, keeps their places
    before = sim.particles_host(0)
    sim.sort(0)                                                   # re-sort
    got = sim.particles_host(0)
    assert np.array_equal(np.sort(got["id"]), ids)
    moved = np.mean(before["cell"] != cell[before["id"]])
    assert moved > 0.3                                            # many particles changed cell
    tile, key = _brick_key(got["cell"].astype(np.int64), grid.n, T)
    wt, wk = _level_order(got["cell"], grid.n, T)
    assert np.array_equal(tile, wt)
    assert np.array_equal(key, wk)


def test_sort_orders_tiles_in_bricks():
    """With plain (depth-1) storage the sorted particles of 8x8x8 tiles follow
    the brick order of their cells; the key is a bijection onto the tile's
    512 slots, so the 64 cells of each brick are exactly an 8x2x4 block."""
    grid = inputs.Grid(n=(16, 16, 24), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    pl = inputs.uniform_random_plasma(grid, ppc=2, seed=45)
    T = (8, 8, 8)
    sim = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", tile=T, interleave=1, max_particles=pl.count)
    sim.add_particles(pl)
    sim.sort(0)
    got = sim.particles_host(0)
    assert np.array_equal(np.sort(got["id"]), np.sort(pl.id))
    tile, key = _brick_key(got["cell"].astype(np.int64), grid.n, T)
    full = tile * 512 + key
    assert np.all(np.diff(full) >= 0)
    cells = np.arange(16 * 16 * 24)
    t_all, k_all = _brick_key(cells, grid.n, T)
    assert np.array_equal(np.sort(t_all * 512 + k_all), np.arange(cells.size))
    brick = (t_all * 512 + k_all) // 64
    for b in np.unique(brick)[:12]:
        c = cells[brick == b]
        ext = [np.ptp(c % 16), np.ptp((c // 16) % 16), np.ptp(c // 256)]
        assert ext == [7, 1, 3]


def test_two_species_keep_their_own_tile_ranges():
    """Two species of very different sizes, sorted every third step: each
    species' fused steps between sorts must use its own tile ranges (fused ==
    split bit for bit, both species)."""
    grid = inputs.Grid(n=(24, 16, 16), d=(0.25, 0.5, 0.5), dt=0.25, solver="pd")
    big = inputs.uniform_random_plasma(grid, ppc=8, seed=51, temperature_ev=50000.0, ux_amp=0.2)
    small = inputs.uniform_random_plasma(grid, ppc=1, seed=52, temperature_ev=50000.0)
    small.m = 3.0
    sims = []
    for kw in (dict(tile=(8, 8, 8), sort_interval=3), {}):
        s = pic.Simulation(grid.n, grid.d, grid.dt, solver="pd", max_particles=big.count + small.count, **kw)
        s.add_particles(small)     # the smaller species sorts first, the larger one last
        s.add_particles(big)
        sims.append(s)
    a, b = sims
    a.step(7)
    for _ in range(7):
        for sp in range(2):
            b.gather_push(sp)
            b.deposit(sp)
        b.field_step()
    for fa, fb in ((a.E, b.E), (a.B, b.B), (a.J, b.J)):
        assert torch.equal(fa, fb)
    for sp in range(2):
        pa, pb = a.particles_host(sp), b.particles_host(sp)
        ia, ib = np.argsort(pa["id"]), np.argsort(pb["id"])
        assert np.array_equal(pa["id"][ia], pb["id"][ib])
        assert np.array_equal(pa["u"][:, ia], pb["u"][:, ib])
        assert np.array_equal(pa["cell"][ia], pb["cell"][ib])


def _fast_beam(grid, seed, ux):
    pl = inputs.uniform_random_plasma(grid, ppc=4, seed=seed, temperature_ev=1000.0)
    pl.u[0] += np.float32(ux)
    return pl


def _share_beyond_guard(pl, grid, tile_x, steps):
    """Share of particles whose x drift over `steps` steps leaves the tile of
    their cell at the last sort (guard 0), from the initial state."""
    v = float(pl.u[0].mean()) / np.sqrt(1.0 + float(pl.u[0].mean()) ** 2)
    cx = pl.cell % grid.n[0]
    local = (cx % tile_x) + pl.off[0]
    return float(np.mean(local + v * grid.dt / grid.d[0] * steps >= tile_x))


def test_particles_beyond_the_guard_take_the_rest_pass():
    """A drift of about half a cell per step carries many particles out of their
    tile between sorts (guard 0, sort every 4 steps); the tile kernel leaves
    them to the global-memory rest pass and the result is still the split
    kernels' bit for bit."""
    grid = inputs.Grid(n=(16, 8, 12), d=(0.25, 0.3, 0.3), dt=0.15)
    pl = _fast_beam(grid, 47, 2.0)
    assert _share_beyond_guard(pl, grid, 4, 3) > 0.25
    for threads in (256, 1024):
        a, b = _pair(grid, pl, tile=(4, 4, 4), guard=0, interleave=1, sort_interval=4, threads=threads)
        a.step(9)
        for _ in range(9):
            b.gather_push(0)
            b.deposit(0)
            b.field_step()
        _assert_same(a, b)
        assert float(a.J.abs().max()) > 0.0
