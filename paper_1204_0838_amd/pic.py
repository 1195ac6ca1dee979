"""Thin ctypes binding of the C ABI in include/pic.h (libpic355.so).

Argument marshalling only: every step of the PIC cycle runs in the HIP
library.  PyTorch-ROCm provides the device memory (fields, particles,
workspace) and the stream; this module passes raw pointers across the ABI
and turns status codes into exceptions.  There is no fallback: without the
built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic355.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_EOVERFLOW, PIC_ENONFINITE, PIC_ECFL, PIC_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE", -4: "PIC_EOVERFLOW",
                -5: "PIC_ENONFINITE", -6: "PIC_ECFL", -7: "PIC_ESTATE"}
SOLVERS = {"yee": 0, "pd": 1}
JPOST = {"none": 0, "binomial": 1, "denoiser": 2}


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("solver", ctypes.c_int32), ("d", ctypes.c_double * 3),
                ("dt", ctypes.c_double), ("pd_variant", ctypes.c_int32), ("bc_x", ctypes.c_int32),
                ("jpost", ctypes.c_int32), ("tile", ctypes.c_int32 * 3), ("sort_interval", ctypes.c_int32),
                ("guard", ctypes.c_int32), ("threads", ctypes.c_int32), ("interleave", ctypes.c_int32)]


_vp = ctypes.c_void_p


class FieldBufs(ctypes.Structure):
    _fields_ = [("E", _vp * 3), ("B", _vp * 3), ("J", _vp * 3)]


class SpeciesBufs(ctypes.Structure):
    _fields_ = [("q", ctypes.c_double), ("m", ctypes.c_double), ("capacity", ctypes.c_int64),
                ("cell", _vp), ("off", _vp * 3), ("u", _vp * 3), ("w", _vp), ("id", _vp)]


class Diag(ctypes.Structure):
    _fields_ = [("charge", ctypes.c_double), ("e_field", ctypes.c_double), ("e_kin", ctypes.c_double),
                ("max_abs_J", ctypes.c_double), ("n_particles", ctypes.c_int64), ("step", ctypes.c_int64)]


class LaserDesc(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("omega0", ctypes.c_double), ("waist", ctypes.c_double),
                ("fwhm", ctypes.c_double), ("t_peak", ctypes.c_double), ("t_end", ctypes.c_double),
                ("yc", ctypes.c_double), ("zc", ctypes.c_double), ("src_x", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class PlasmaDesc(ctypes.Structure):
    _fields_ = [("x_start", ctypes.c_double), ("ramp", ctypes.c_double), ("n_plateau", ctypes.c_double),
                ("ppc", ctypes.c_int32 * 3), ("pad_", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("sort_ms", ctypes.c_double), ("tile_ms", ctypes.c_double), ("loose_ms", ctypes.c_double),
                ("jpost_ms", ctypes.c_double), ("field_ms", ctypes.c_double), ("window_ms", ctypes.c_double),
                ("steps", ctypes.c_int64), ("sorts", ctypes.c_int64), ("tile_launches", ctypes.c_int64)]


class BeamDiag(ctypes.Structure):
    _fields_ = [("charge", ctypes.c_double), ("count", ctypes.c_int64), ("mean_ux", ctypes.c_double),
                ("eps_ny", ctypes.c_double), ("eps_nz", ctypes.c_double), ("mean_r", ctypes.c_double * 2),
                ("rms_r", ctypes.c_double * 2), ("rms_p", ctypes.c_double * 2)]


class PmlDesc(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int32), ("pad_", ctypes.c_int32), ("sigma_max", ctypes.c_double * 2),
                ("grade", ctypes.c_double)]


class Tiling(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32 * 3), ("guard", ctypes.c_int32), ("threads", ctypes.c_int32),
                ("interleave", ctypes.c_int32), ("sort_interval", ctypes.c_int32)]


# every symbol the header declares, with its ctypes signature
_SIGS = {
    "pic_set_tiling": (ctypes.c_int, [_vp, ctypes.POINTER(Tiling)]),
    "pic_pml_bytes": (ctypes.c_size_t, [ctypes.POINTER(GridDesc), ctypes.POINTER(PmlDesc)]),
    "pic_set_pml": (ctypes.c_int, [_vp, ctypes.POINTER(PmlDesc), _vp, ctypes.c_size_t]),
    "pic_axis_line": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "pic_accelerating_length": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]),
    "pic_spectrum": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "pic_beam_moments": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(BeamDiag)]),
    "pic_select_particles": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_double, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int64)]),
    "pic_field_moments": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "pic_checkpoint_bytes": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "pic_copy_out": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "pic_copy_in": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t]),
    "pic_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(Profile)]),
    "pic_set_laser": (ctypes.c_int, [_vp, ctypes.POINTER(LaserDesc)]),
    "pic_set_plasma": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(PlasmaDesc)]),
    "pic_inject_plasma": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pic_set_window": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "pic_window_state": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "pic_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(GridDesc), ctypes.c_int64]),
    "pic_validate_grid": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.c_char_p, ctypes.c_size_t]),
    "pic_init_grid": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(GridDesc), ctypes.POINTER(FieldBufs), _vp,
                                     ctypes.c_size_t, ctypes.c_int64, _vp]),
    "pic_init_species": (ctypes.c_int, [_vp, ctypes.POINTER(SpeciesBufs), ctypes.c_int64,
                                        ctypes.POINTER(ctypes.c_int32)]),
    "pic_gather_push": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_deposit": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_field_step": (ctypes.c_int, [_vp]),
    "pic_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_sort": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_species_view": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(SpeciesBufs),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "pic_continuity": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double)]),
    "pic_continuity_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_double)]),
    "pic_reduce": (ctypes.c_int, [_vp, ctypes.POINTER(Diag)]),
    "pic_sync": (ctypes.c_int, [_vp]),
    "pic_last_error": (ctypes.c_char_p, [_vp]),
    "pic_destroy": (None, [_vp]),
    "pic_denoiser_set": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float)]),
    "pic_current_filter": (ctypes.c_int, [_vp]),
    "pic_dn_trainer_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int32)]),
    "pic_dn_trainer_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_double), _vp, ctypes.c_size_t, _vp]),
    "pic_dn_trainer_set_params": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                                 ctypes.POINTER(ctypes.c_float)]),
    "pic_dn_trainer_get_params": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float),
                                                 ctypes.POINTER(ctypes.c_float)]),
    "pic_dn_trainer_step": (ctypes.c_int, [_vp, _vp * 3, _vp * 3, ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
    "pic_dn_trainer_grad": (ctypes.c_int, [_vp, _vp * 3, _vp * 3, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "pic_dn_trainer_step_batch": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                                 ctypes.c_float, ctypes.POINTER(ctypes.c_double)]),
    "pic_dn_trainer_eval": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                           ctypes.POINTER(ctypes.c_double)]),
    "pic_dn_trainer_freeze_biases": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_dn_trainer_last_error": (ctypes.c_char_p, [_vp]),
    "pic_dn_trainer_destroy": (None, [_vp]),
    "pic_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "pic_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32, _vp,
                                        ctypes.c_size_t, _vp]),
    "pic_batch_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_batch_sync": (ctypes.c_int, [_vp]),
    "pic_batch_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_batch_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(Profile)]),
    "pic_batch_last_error": (ctypes.c_char_p, [_vp]),
    "pic_batch_destroy": (None, [_vp]),
}

class CircDesc(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("nr", ctypes.c_int32), ("dz", ctypes.c_double), ("dr", ctypes.c_double),
                ("dt", ctypes.c_double), ("window_period", ctypes.c_int32), ("sort_interval", ctypes.c_int32),
                ("interleave", ctypes.c_int32), ("threads", ctypes.c_int32)]


class CircFieldBufs(ctypes.Structure):
    _fields_ = [("E", _vp * 9), ("B", _vp * 9), ("J", _vp * 9)]


class CircLaser(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("omega0", ctypes.c_double), ("waist", ctypes.c_double),
                ("fwhm", ctypes.c_double), ("t_peak", ctypes.c_double), ("t_end", ctypes.c_double),
                ("src_z", ctypes.c_int32), ("pad_", ctypes.c_int32)]


class CircPlasma(ctypes.Structure):
    _fields_ = [("z_start", ctypes.c_double), ("ramp", ctypes.c_double), ("n_plateau", ctypes.c_double),
                ("ppc", ctypes.c_int32), ("r_cells", ctypes.c_int32), ("seed", ctypes.c_uint64)]


_SIGS.update({
    "pic_circ_validate": (ctypes.c_int, [ctypes.POINTER(CircDesc), ctypes.c_char_p, ctypes.c_size_t]),
    "pic_circ_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(CircDesc), ctypes.c_int64]),
    "pic_circ_init": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.POINTER(CircDesc), ctypes.POINTER(CircFieldBufs), _vp,
                                     ctypes.c_size_t, ctypes.c_int64, _vp]),
    "pic_circ_init_species": (ctypes.c_int, [_vp, ctypes.POINTER(SpeciesBufs), ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "pic_circ_gather_push": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_circ_deposit": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_circ_field_step": (ctypes.c_int, [_vp]),
    "pic_circ_step": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_circ_set_laser": (ctypes.c_int, [_vp, ctypes.POINTER(CircLaser)]),
    "pic_circ_set_plasma": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(CircPlasma)]),
    "pic_circ_inject_plasma": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "pic_circ_set_window": (ctypes.c_int, [_vp, ctypes.c_int64]),
    "pic_circ_window_state": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "pic_circ_species_view": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(SpeciesBufs),
                                             ctypes.POINTER(ctypes.c_int64)]),
    "pic_circ_reduce": (ctypes.c_int, [_vp, ctypes.POINTER(Diag)]),
    "pic_circ_sync": (ctypes.c_int, [_vp]),
    "pic_circ_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "pic_circ_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(Profile)]),
    "pic_circ_last_error": (ctypes.c_char_p, [_vp]),
    "pic_circ_destroy": (None, [_vp]),
})

_lib = None


def lib():
    """Load libpic355.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1204_0838_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def make_desc(n, d, dt, solver="yee", bc_x=0, jpost="none", pd_variant=0, tile=(0, 0, 0), sort_interval=0,
              guard=-1, threads=0, interleave=0):
    g = GridDesc()
    for a in range(3):
        g.n[a] = int(n[a])
        g.d[a] = float(d[a])
        g.tile[a] = int(tile[a])
    g.dt = float(dt)
    g.solver = SOLVERS[solver] if isinstance(solver, str) else int(solver)
    g.bc_x = int(bc_x)
    g.jpost = JPOST[jpost] if isinstance(jpost, str) else int(jpost)
    g.pd_variant = int(pd_variant)
    g.sort_interval = int(sort_interval)
    g.guard = int(guard)
    g.threads = int(threads)
    g.interleave = int(interleave)
    return g


def validate(desc: GridDesc):
    """Host-only descriptor check: returns (status, message)."""
    buf = ctypes.create_string_buffer(256)
    st = lib().pic_validate_grid(ctypes.byref(desc), buf, 256)
    return st, buf.value.decode()


def workspace_bytes(desc: GridDesc, max_particles: int) -> int:
    return int(lib().pic_workspace_bytes(ctypes.byref(desc), int(max_particles)))


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Simulation:
    """A grid with its fields, workspace and species, driven through the C ABI.

    Fields are torch tensors ``E, B, J`` of shape [3, nz, ny, nx] (float32,
    x fastest) on ``device``; particles live in caller-owned torch tensors.
    """

    def __init__(self, n, d, dt, solver="yee", bc_x=0, jpost="none", pd_variant=0, tile=(0, 0, 0),
                 sort_interval=0, guard=-1, threads=0, interleave=0, max_particles=0, device="cuda:0", stream=None):
        self.desc = make_desc(n, d, dt, solver, bc_x, jpost, pd_variant, tile, sort_interval, guard, threads,
                              interleave)
        st, msg = validate(self.desc)
        if st != PIC_OK:
            raise PicError(st, msg)
        self.device = torch.device(device)
        self.n = tuple(int(v) for v in n)
        shape = (3, self.n[2], self.n[1], self.n[0])
        self.E = torch.zeros(shape, dtype=torch.float32, device=self.device)
        self.B = torch.zeros(shape, dtype=torch.float32, device=self.device)
        self.J = torch.zeros(shape, dtype=torch.float32, device=self.device)
        self.max_particles = int(max_particles)
        nbytes = workspace_bytes(self.desc, self.max_particles)
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "workspace size query failed")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        fb = FieldBufs()
        for a in range(3):
            fb.E[a] = self.E[a].data_ptr()
            fb.B[a] = self.B[a].data_ptr()
            fb.J[a] = self.J[a].data_ptr()
        h = ctypes.c_void_p()
        st = lib().pic_init_grid(ctypes.byref(h), ctypes.byref(self.desc), ctypes.byref(fb),
                                 ctypes.c_void_p(base + self._ws_off), nbytes, self.max_particles,
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if st != PIC_OK:
            raise PicError(st, "pic_init_grid failed")
        self.handle = h
        self.species = []

    # ------------------------------------------------------------ plumbing
    def _check(self, st):
        if st != PIC_OK:
            msg = lib().pic_last_error(self.handle)
            raise PicError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "handle", None):
            lib().pic_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ species
    def add_species(self, cell, off, u, w, ids, q=-1.0, m=1.0, capacity=None):
        """Register a species from host or device arrays (copied into new device tensors)."""
        n = int(len(cell))
        cap = int(capacity if capacity is not None else n)
        dev = self.device

        def buf(src, dtype):
            t = torch.zeros(cap, dtype=dtype, device=dev)
            if n:
                t[:n] = torch.as_tensor(np.asarray(src) if not torch.is_tensor(src) else src).to(dev, dtype)
            return t

        sp = {"cell": buf(cell, torch.int32), "off": [buf(off[a], torch.float32) for a in range(3)],
              "u": [buf(u[a], torch.float32) for a in range(3)], "w": buf(w, torch.float32),
              "id": buf(ids, torch.int32), "q": float(q), "m": float(m), "capacity": cap}
        sb = SpeciesBufs()
        sb.q, sb.m, sb.capacity = float(q), float(m), cap
        sb.cell = sp["cell"].data_ptr()
        for a in range(3):
            sb.off[a] = sp["off"][a].data_ptr()
            sb.u[a] = sp["u"][a].data_ptr()
        sb.w = sp["w"].data_ptr()
        sb.id = sp["id"].data_ptr()
        idx = ctypes.c_int32()
        self._check(lib().pic_init_species(self.handle, ctypes.byref(sb), n, ctypes.byref(idx)))
        self.species.append(sp)
        return idx.value

    def add_particles(self, p, capacity=None):
        """Register an ``inputs.Particles`` set."""
        return self.add_species(p.cell, p.off, p.u, p.w, p.id, p.q, p.m, capacity)

    def add_empty_species(self, capacity, q=-1.0, m=1.0):
        """Register a species with no particles yet (filled by plasma injection)."""
        z = np.zeros(0, np.int32)
        zf = np.zeros((3, 0), np.float32)
        return self.add_species(z, zf, zf, np.zeros(0, np.float32), z, q, m, capacity)

    # ------------------------------------------------------------ laser-wakefield boundaries
    def set_laser(self, a0, omega0, waist, fwhm, t_peak, t_end, yc, zc, src_x):
        L = LaserDesc(float(a0), float(omega0), float(waist), float(fwhm), float(t_peak), float(t_end), float(yc),
                      float(zc), int(src_x), 0)
        self._check(lib().pic_set_laser(self.handle, ctypes.byref(L)))

    def set_plasma(self, s, x_start, ramp, n_plateau, ppc=(2, 2, 2)):
        P = PlasmaDesc(float(x_start), float(ramp), float(n_plateau))
        for a in range(3):
            P.ppc[a] = int(ppc[a])
        self._check(lib().pic_set_plasma(self.handle, s, ctypes.byref(P)))

    def inject_plasma(self, s, x_begin, x_end):
        self._check(lib().pic_inject_plasma(self.handle, s, int(x_begin), int(x_end)))

    def set_window(self, start_step):
        self._check(lib().pic_set_window(self.handle, int(start_step)))

    def set_pml(self, layers=16, sigma_max=(0.0, 0.0), grade=0.0):
        """Transverse absorbing layer of `layers` cells (0 removes it); its
        device buffer is owned by this object.  sigma_max <= 0 and grade <= 0
        select the library's defaults."""
        P = PmlDesc(int(layers), 0)
        P.sigma_max[0], P.sigma_max[1] = float(sigma_max[0]), float(sigma_max[1])
        P.grade = float(grade)
        if int(layers) == 0:
            self._check(lib().pic_set_pml(self.handle, ctypes.byref(P), None, 0))
            self.pml_buffer = None
            return
        nbytes = int(lib().pic_pml_bytes(ctypes.byref(self.desc), ctypes.byref(P)))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, f"invalid absorbing layer of {layers} cells for this grid")
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = (buf.data_ptr() + 255) // 256 * 256
        self._check(lib().pic_set_pml(self.handle, ctypes.byref(P), ctypes.c_void_p(base), nbytes))
        self.pml_buffer = buf

    def window_state(self):
        sh, org = ctypes.c_int64(), ctypes.c_int32()
        self._check(lib().pic_window_state(self.handle, ctypes.byref(sh), ctypes.byref(org)))
        return sh.value, org.value

    def fields_window_order(self):
        """E, B, J as numpy arrays rolled so that x index 0 is the window's trailing cell."""
        _, org = self.window_state()
        return tuple(np.roll(t.cpu().numpy(), -org, axis=3) for t in (self.E, self.B, self.J))

    def set_tiling(self, tile=(0, 0, 0), guard=-1, threads=0, interleave=0, sort_interval=0):
        t = Tiling()
        for a in range(3):
            t.tile[a] = int(tile[a])
        t.guard, t.threads, t.interleave, t.sort_interval = int(guard), int(threads), int(interleave), \
            int(sort_interval)
        self._check(lib().pic_set_tiling(self.handle, ctypes.byref(t)))

    def profile_enable(self, on=True):
        self._check(lib().pic_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        p = Profile()
        self._check(lib().pic_profile_read(self.handle, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    # ------------------------------------------------------------ current post-processing
    def set_denoiser(self, params, scale):
        """params = (W1 [32,3,3,3,3], b1 [32], W2 [32,32,3,3,3], b2 [32], W3 [3,32,3,3,3], b3 [3])."""
        W1, b1, W2, b2, W3, b3 = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in params]
        assert W1.shape == (32, 3, 3, 3, 3) and W2.shape == (32, 32, 3, 3, 3) and W3.shape == (3, 32, 3, 3, 3)
        w = np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()]).astype(np.float32)
        b = np.concatenate([b1.ravel(), b2.ravel(), b3.ravel()]).astype(np.float32)
        sc = np.ascontiguousarray(np.asarray(scale, dtype=np.float32))
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().pic_denoiser_set(self.handle, w.ctypes.data_as(fp), b.ctypes.data_as(fp),
                                           sc.ctypes.data_as(fp)))

    def current_filter(self):
        self._check(lib().pic_current_filter(self.handle))

    # ------------------------------------------------------------ the cycle
    def gather_push(self, s=0):
        self._check(lib().pic_gather_push(self.handle, s))

    def deposit(self, s=0):
        self._check(lib().pic_deposit(self.handle, s))

    def field_step(self):
        self._check(lib().pic_field_step(self.handle))

    def step(self, nsteps=1):
        self._check(lib().pic_step(self.handle, int(nsteps)))

    def sort(self, s=0):
        self._check(lib().pic_sort(self.handle, s))

    def sync(self):
        self._check(lib().pic_sync(self.handle))

    def continuity(self, s=0):
        r, j = ctypes.c_double(), ctypes.c_double()
        self._check(lib().pic_continuity(self.handle, s, ctypes.byref(r), ctypes.byref(j)))
        return r.value, j.value

    def continuity_noalloc(self, s=0):
        """pic_continuity through the library's fixed scratch (no workspace density buffer)."""
        r, j = ctypes.c_double(), ctypes.c_double()
        self._check(lib().pic_continuity_noalloc(self.handle, s, ctypes.byref(r), ctypes.byref(j)))
        return r.value, j.value

    def reduce(self):
        d = Diag()
        self._check(lib().pic_reduce(self.handle, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    # ------------------------------------------------------------ run diagnostics
    def axis_line(self, comp=0, yc=None, zc=None):
        """Field component comp (0..5 = E_x..B_z) along x at (yc, zc) (default: the box's axis)."""
        yc = self.n[1] * self.desc.d[1] / 2 if yc is None else yc
        zc = self.n[2] * self.desc.d[2] / 2 if zc is None else zc
        out = np.zeros(self.n[0])
        self._check(lib().pic_axis_line(self.handle, int(comp), float(yc), float(zc),
                                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def accelerating_length(self, x_from, yc=None, zc=None):
        yc = self.n[1] * self.desc.d[1] / 2 if yc is None else yc
        zc = self.n[2] * self.desc.d[2] / 2 if zc is None else zc
        v = ctypes.c_double()
        self._check(lib().pic_accelerating_length(self.handle, float(yc), float(zc), float(x_from), ctypes.byref(v)))
        return v.value

    def spectrum(self, s=0, quantity=0, lo=0.0, hi=1.0, nbins=64):
        """(charge per bin, count per bin) over [lo, hi); quantity 0: gamma - 1, 1: u_x."""
        charge = np.zeros(int(nbins))
        count = np.zeros(int(nbins), dtype=np.int64)
        self._check(lib().pic_spectrum(self.handle, s, int(quantity), float(lo), float(hi), int(nbins),
                                       charge.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                       count.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return charge, count

    def beam_moments(self, s=0, ux_min=0.0):
        d = BeamDiag()
        self._check(lib().pic_beam_moments(self.handle, s, float(ux_min), ctypes.byref(d)))
        return {"charge": d.charge, "count": d.count, "mean_ux": d.mean_ux, "eps_ny": d.eps_ny, "eps_nz": d.eps_nz,
                "mean_r": tuple(d.mean_r), "rms_r": tuple(d.rms_r), "rms_p": tuple(d.rms_p)}

    def select_particles(self, s=0, ux_min=0.0, cap=1 << 20):
        """(ids, window x, u_x) of the particles with u_x > ux_min (at most cap), and how many qualify."""
        ids = np.zeros(int(cap), dtype=np.int32)
        x = np.zeros(int(cap))
        ux = np.zeros(int(cap), dtype=np.float32)
        n = ctypes.c_int64()
        self._check(lib().pic_select_particles(self.handle, s, float(ux_min), int(cap),
                                               ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                               x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ux.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(n)))
        k = min(n.value, int(cap))
        return ids[:k], x[:k], ux[:k], n.value

    def field_moments(self, transverse_only=False):
        out = np.zeros(3)
        self._check(lib().pic_field_moments(self.handle, 1 if transverse_only else 0,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return tuple(out)

    # ------------------------------------------------------------ checkpoint
    def copy_out(self) -> bytes:
        """Host checkpoint blob of the current state (synchronises)."""
        nb = ctypes.c_size_t()
        self._check(lib().pic_checkpoint_bytes(self.handle, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        self._check(lib().pic_copy_out(self.handle, ctypes.cast(buf, _vp), nb.value))
        return buf.raw

    def copy_in(self, blob: bytes):
        """Restore a checkpoint blob written by copy_out (synchronises)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(lib().pic_copy_in(self.handle, ctypes.cast(buf, _vp), len(blob)))

    # ------------------------------------------------------------ views
    def _tensor_at(self, ptr, n, dtype, s):
        """Tensor view of n elements at device address ptr (a species tensor or the workspace)."""
        sp = self.species[s]
        for t in [sp["cell"], sp["w"], sp["id"], *sp["off"], *sp["u"]]:
            if t.data_ptr() == ptr:
                return t[:n]
        base = self.workspace.data_ptr()
        off = ptr - base
        if not (0 <= off < self.workspace.numel()):
            raise PicError(PIC_EINVAL, "pointer outside the known buffers")
        esz = torch.empty(0, dtype=dtype).element_size()
        return self.workspace[off:off + n * esz].view(dtype)

    def particles(self, s=0):
        """Live-range device views of the species' current arrays (synchronises)."""
        sb = SpeciesBufs()
        n = ctypes.c_int64()
        self._check(lib().pic_species_view(self.handle, s, ctypes.byref(sb), ctypes.byref(n)))
        k = n.value
        return {"cell": self._tensor_at(sb.cell, k, torch.int32, s),
                "off": [self._tensor_at(sb.off[a], k, torch.float32, s) for a in range(3)],
                "u": [self._tensor_at(sb.u[a], k, torch.float32, s) for a in range(3)],
                "w": self._tensor_at(sb.w, k, torch.float32, s),
                "id": self._tensor_at(sb.id, k, torch.int32, s), "count": k}

    def particles_host(self, s=0):
        """Numpy copy of the live particles: dict(cell, off[3,n], u[3,n], w, id)."""
        v = self.particles(s)
        return {"cell": v["cell"].cpu().numpy(), "off": np.stack([t.cpu().numpy() for t in v["off"]]),
                "u": np.stack([t.cpu().numpy() for t in v["u"]]), "w": v["w"].cpu().numpy(),
                "id": v["id"].cpu().numpy()}


class Batch:
    """Lockstep driver of several Simulations (one launch per phase for all).

    Every member must use the same stream and have the same number of
    species; members stay usable on their own between batch calls.
    """

    def __init__(self, members):
        self.members = list(members)
        if not self.members:
            raise PicError(PIC_EINVAL, "empty batch")
        dev = self.members[0].device
        self.stream = self.members[0].stream
        n = len(self.members)
        nbytes = int(lib().pic_batch_workspace_bytes(n))
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        arr = (_vp * n)(*[m.handle.value for m in self.members])
        h = ctypes.c_void_p()
        st = lib().pic_batch_create(ctypes.byref(h), arr, n, ctypes.c_void_p(base + off), nbytes,
                                    ctypes.c_void_p(self.stream.cuda_stream))
        if st != PIC_OK:
            raise PicError(st, "pic_batch_create failed")
        self.handle = h

    def _check(self, st):
        if st != PIC_OK:
            msg = lib().pic_batch_last_error(self.handle)
            raise PicError(st, msg.decode() if msg else "")

    def step(self, nsteps=1):
        self._check(lib().pic_batch_step(self.handle, int(nsteps)))

    def sync(self):
        self._check(lib().pic_batch_sync(self.handle))

    def profile_enable(self, on=True):
        self._check(lib().pic_batch_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        p = Profile()
        self._check(lib().pic_batch_profile_read(self.handle, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().pic_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


N_WEIGHTS = 32 * 3 * 27 + 32 * 32 * 27 + 3 * 32 * 27
N_BIASES = 32 + 32 + 3


def pack_params(params):
    """(W1, b1, W2, b2, W3, b3) -> flat FP32 (weights, biases) in the pic_denoiser_set layout."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(a, dtype=np.float32) for a in params]
    w = np.ascontiguousarray(np.concatenate([W1.ravel(), W2.ravel(), W3.ravel()]), dtype=np.float32)
    b = np.ascontiguousarray(np.concatenate([b1.ravel(), b2.ravel(), b3.ravel()]), dtype=np.float32)
    return w, b


def unpack_params(w, b):
    n1, n2 = 32 * 3 * 27, 32 * 32 * 27
    return [w[:n1].reshape(32, 3, 3, 3, 3), b[:32], w[n1:n1 + n2].reshape(32, 32, 3, 3, 3), b[32:64],
            w[n1 + n2:].reshape(3, 32, 3, 3, 3), b[64:67]]


class DenoiserTrainer:
    """Adam training of the current denoiser on crops of ``crop`` = (nx, ny, nz) cells of size ``cell``."""

    def __init__(self, crop, cell=(1.0, 1.0, 1.0), device="cuda:0", stream=None):
        self.crop = tuple(int(v) for v in crop)
        self.device = torch.device(device)
        c = (ctypes.c_int32 * 3)(*self.crop)
        nbytes = int(lib().pic_dn_trainer_workspace_bytes(c))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "invalid crop")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        cd = (ctypes.c_double * 3)(*[float(v) for v in cell])
        st = lib().pic_dn_trainer_create(ctypes.byref(h), c, cd, ctypes.c_void_p(base + (-base) % 256), nbytes,
                                         ctypes.c_void_p(self.stream.cuda_stream))
        if st != PIC_OK:
            raise PicError(st, "pic_dn_trainer_create failed")
        self.handle = h

    def _check(self, st):
        if st != PIC_OK:
            msg = lib().pic_dn_trainer_last_error(self.handle)
            raise PicError(st, msg.decode() if msg else "")

    @staticmethod
    def _arr3(t):
        assert t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == 3
        return (_vp * 3)(*[t[a].data_ptr() for a in range(3)])

    def set_params(self, params, scale):
        w, b = pack_params(params)
        sc = np.ascontiguousarray(np.asarray(scale, dtype=np.float32))
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().pic_dn_trainer_set_params(self.handle, w.ctypes.data_as(fp), b.ctypes.data_as(fp),
                                                    sc.ctypes.data_as(fp)))

    def get_params(self):
        w = np.zeros(N_WEIGHTS, np.float32)
        b = np.zeros(N_BIASES, np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().pic_dn_trainer_get_params(self.handle, w.ctypes.data_as(fp), b.ctypes.data_as(fp)))
        return unpack_params(w, b)

    def step(self, inp, target, lr, want_loss=True):
        """inp, target: float32 tensors [3, nz, ny, nx] on the device."""
        loss = ctypes.c_double()
        self._check(lib().pic_dn_trainer_step(self.handle, self._arr3(inp), self._arr3(target), float(lr),
                                              ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    @staticmethod
    def _ptrs(ts):
        out = []
        for t in ts:
            assert t.dtype == torch.float32 and t.is_contiguous() and t.shape[0] == 3
            out += [t[a].data_ptr() for a in range(3)]
        return (_vp * len(out))(*out)

    def step_batch(self, inps, targets, lr, want_loss=True):
        """One Adam step on the mean gradient over lists of crops."""
        loss = ctypes.c_double()
        self._check(lib().pic_dn_trainer_step_batch(self.handle, len(inps), self._ptrs(inps), self._ptrs(targets),
                                                    float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def eval(self, inps, targets):
        """Mean loss over lists of crops."""
        loss = ctypes.c_double()
        self._check(lib().pic_dn_trainer_eval(self.handle, len(inps), self._ptrs(inps), self._ptrs(targets),
                                              ctypes.byref(loss)))
        return loss.value

    def freeze_biases(self, freeze=True):
        self._check(lib().pic_dn_trainer_freeze_biases(self.handle, 1 if freeze else 0))

    def grad(self, inp, target):
        loss = ctypes.c_double()
        gw = np.zeros(N_WEIGHTS, np.float32)
        gb = np.zeros(N_BIASES, np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        self._check(lib().pic_dn_trainer_grad(self.handle, self._arr3(inp), self._arr3(target), ctypes.byref(loss),
                                              gw.ctypes.data_as(fp), gb.ctypes.data_as(fp)))
        return loss.value, unpack_params(gw, gb)

    def close(self):
        if getattr(self, "handle", None):
            lib().pic_dn_trainer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
