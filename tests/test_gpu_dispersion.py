"""Laser group velocity on the GPU under the Yee and perfect-dispersion
solvers (pic_field_moments on runs through the C ABI).

- A plane C1 pulse on a 320x4x4 grid: the GPU's centroid track and fitted
  group velocity equal the oracle's (FP32 fields against FP64), for both
  solvers.
- The C1 grid (512x256x256, waist 5): the perfect-dispersion pulse is
  faster than the Yee pulse by the plane-wave slowdown, to 30% (the
  Gaussian beam's transverse wavenumbers change the Yee error slightly)."""
import numpy as np
import pytest

from tests.test_oracle_dispersion import D, NX, plane_pulse_run, yee_dt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1204_0838_amd import dispersion  # noqa: E402


@pytest.mark.parametrize("solver", ["pd", "yee"])
def test_plane_pulse_group_velocity_matches_oracle(solver):
    print(f"plane pulse, {solver}", flush=True)
    r = dispersion.measure(solver, n=(NX, 4, 4), d=D, waist=1e12, t_from=30.0, t_to=70.0, every=5)
    dt = D[0] if solver == "pd" else yee_dt()
    assert abs(r["dt"] - dt) < 1e-15
    ts, xc, _ = plane_pulse_run(solver, dt)
    assert np.allclose(r["times"], ts, rtol=0, atol=1e-12)
    assert np.abs(np.array(r["centroids"]) - xc).max() < 1e-5
    v_ora = np.polyfit(ts, xc, 1)[0]
    assert abs(r["v_g"] - v_ora) < 1e-6, (r["v_g"], v_ora)


def test_c1_grid_yee_pulse_lags_the_perfect_dispersion_pulse():
    print("C1 grid, vacuum pulse, both solvers", flush=True)
    pd = dispersion.measure("pd", t_from=30.0, t_to=100.0)
    yee = dispersion.measure("yee", t_from=30.0, t_to=100.0)
    ts, xc, _ = plane_pulse_run("yee", yee_dt())
    plane_slowdown = 1.0 - np.polyfit(ts, xc, 1)[0]
    slowdown = pd["v_g"] - yee["v_g"]
    print(f"C1 grid: v_g pd {pd['v_g']:.6f}, yee {yee['v_g']:.6f}; slowdown {slowdown:.5f} "
          f"(plane wave {plane_slowdown:.5f})", flush=True)
    assert pd["residual"] < 0.05 and yee["residual"] < 0.05
    assert pd["v_g"] > 0.97
    assert abs(slowdown - plane_slowdown) < 0.3 * plane_slowdown
