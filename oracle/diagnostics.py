"""FP64 reference definitions of the run diagnostics of Section 3.2.

TEST INFRASTRUCTURE ONLY: imported by the tests (and nothing in the product
path).  Plain numpy, one formula per function, written from the quantities
the paper reports for its runs:

- the on-axis longitudinal field and the length of the accelerating phase,
  the region inside the bubble where E_x < 0 (Section 3.2, Fig. 1(a));
- the normalised transverse emittance
  eps_N,i = [(<p_i^2> - <p_i>^2)(<r_i^2> - <r_i>^2) - (<p_i r_i> - <r_i><p_i>)^2]^(1/2) / (m_e c)
  with i = y, z (Section 3.2, Table 1), averages weighted by charge;
- energy and longitudinal-momentum spectra (Section 3.2, Figs. 3-4;
  Section 3.3) as charge histograms;
- the selection of accelerated electrons with their tags (the collection
  phase space of Fig. 1(b), (c): momenta against initial positions);
- first and second moments of the electromagnetic energy along x (the
  laser pulse's centroid and length, whose motion gives its group velocity,
  Section 3.3).

Units are those of the oracle (c = 1, lengths c/w_p, momenta m_e c).
Positions are window coordinates (x from the window's trailing face).
"""
from __future__ import annotations

import numpy as np

# staggering of E_x, E_y, E_z, B_x, B_y, B_z along x (cells)
X_STAGGER = (0.5, 0.0, 0.0, 0.0, 0.5, 0.5)
YZ_STAGGER = ((0.0, 0.0), (0.5, 0.0), (0.0, 0.5), (0.5, 0.5), (0.0, 0.5), (0.5, 0.0))


def axis_line(F, comp, d, yc, zc):
    """Field component `comp` (0..5 = E_x..B_z, array [nz, ny, nx]) along x at
    the transverse point (yc, zc), bilinear in y and z between the four
    nearest nodes of the component's own staggered grid (periodic y, z)."""
    nz, ny, nx = F.shape
    sy, sz = YZ_STAGGER[comp]
    gy = yc / d[1] - sy
    gz = zc / d[2] - sz
    j0, k0 = int(np.floor(gy)), int(np.floor(gz))
    ty, tz = gy - j0, gz - k0
    out = np.zeros(nx)
    for dk, wk in ((0, 1.0 - tz), (1, tz)):
        for dj, wj in ((0, 1.0 - ty), (1, ty)):
            out += wk * wj * F[(k0 + dk) % nz, (j0 + dj) % ny, :]
    return out


def accelerating_length(line, dx, x_from, stagger=0.5):
    """Length of the first region with line < 0 at or behind x_from (window
    coordinates; line[i] sits at (i + stagger) dx).  Going backward from the
    last sample at or behind x_from, samples with line >= 0 are skipped (the
    front of the bubble); the accelerating phase is the run of negative
    samples that follows.  Its ends are the zero crossings found by linear
    interpolation between neighbouring samples; a run that reaches past
    x_from ends at x_from, one that reaches the window's back at the first
    sample.  0 if there is no negative sample behind x_from."""
    xs = (np.arange(len(line)) + stagger) * dx
    i = int(np.searchsorted(xs, x_from, side="right")) - 1
    if i < 0:
        return 0.0
    start = i
    while i >= 0 and line[i] >= 0:
        i -= 1
    if i < 0:
        return 0.0
    hi = i                                  # frontmost negative sample
    while i >= 0 and line[i] < 0:
        i -= 1
    lo = i + 1                              # rearmost negative sample

    def crossing(a, b):                     # zero between samples a (>= 0) and b (< 0)
        return xs[a] + (xs[b] - xs[a]) * line[a] / (line[a] - line[b])

    if hi < start:
        front = crossing(hi + 1, hi)
    else:                                   # negative at x_from itself
        front = x_from if hi + 1 >= len(line) or line[hi + 1] < 0 else crossing(hi + 1, hi)
    rear = crossing(lo - 1, lo) if lo >= 1 else xs[lo]
    return front - rear


def spectrum(u, w, q, dv, quantity, lo, hi, nbins):
    """Charge histogram |q| w dV of particles binned by kinetic energy
    gamma - 1 (quantity 0) or by u_x (quantity 1) over [lo, hi) in nbins
    equal bins; particles outside the range are not counted.  Returns
    (charge per bin, count per bin)."""
    u = np.asarray(u, dtype=np.float64)
    a, b, c = u[0], u[1], u[2]
    if quantity == 0:
        u2 = a * a + b * b + c * c
        val = u2 / (np.sqrt(1.0 + u2) + 1.0)         # gamma - 1
    else:
        val = a
    t = (val - lo) / (hi - lo) * nbins
    idx = np.floor(t)
    ok = (t >= 0) & (idx < nbins)
    k = idx[ok].astype(np.int64)
    charge = np.bincount(k, weights=abs(q) * dv * np.asarray(w, dtype=np.float64)[ok], minlength=nbins)
    count = np.bincount(k, minlength=nbins)
    return charge, count


def beam_moments(x, u, w, q, dv, ux_min):
    """Charge, count, mean u_x and the normalised emittances in y and z of
    the particles with u_x > ux_min (weights w; positions x [3, np] and
    momenta u [3, np] in m_e c)."""
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    sel = u[0] > ux_min
    ws = w[sel]
    out = {"count": int(sel.sum()), "charge": abs(q) * dv * ws.sum()}
    if ws.sum() <= 0:
        out.update(mean_ux=0.0, eps_ny=0.0, eps_nz=0.0)
        return out
    W = ws.sum()

    def avg(v):
        return (ws * v).sum() / W

    out["mean_ux"] = avg(u[0, sel])
    for name, i in (("eps_ny", 1), ("eps_nz", 2)):
        r, p = x[i, sel], u[i, sel]
        var_p = avg(p * p) - avg(p) ** 2
        var_r = avg(r * r) - avg(r) ** 2
        cov = avg(p * r) - avg(r) * avg(p)
        out[name] = float(np.sqrt(max(var_p * var_r - cov * cov, 0.0)))
    return out


def select(ids, x, u, ux_min):
    """Tags, window x and u_x of the particles with u_x > ux_min, in tag order."""
    ids = np.asarray(ids)
    sel = np.asarray(u[0], dtype=np.float64) > ux_min
    order = np.argsort(ids[sel], kind="stable")
    return ids[sel][order], np.asarray(x[0])[sel][order], np.asarray(u[0])[sel][order]


def field_moments(E, B, d, transverse_only=False):
    """(sum e dV, sum e x dV, sum e x^2 dV) of the energy density
    e = (E^2 + B^2)/2, each component at its own staggered x position
    ((i + stagger) dx).  transverse_only: E_y, E_z, B_y, B_z only (the
    laser's components for a pulse along x)."""
    dv = d[0] * d[1] * d[2]
    comps = [E[0], E[1], E[2], B[0], B[1], B[2]]
    use = (1, 2, 4, 5) if transverse_only else range(6)
    m0 = m1 = m2 = 0.0
    for c in use:
        nx = comps[c].shape[-1]
        xs = (np.arange(nx) + X_STAGGER[c]) * d[0]
        e = 0.5 * (np.asarray(comps[c], dtype=np.float64) ** 2).sum(axis=(0, 1)) * dv
        m0 += e.sum()
        m1 += (e * xs).sum()
        m2 += (e * xs * xs).sum()
    return m0, m1, m2
