"""Thin ctypes binding of the quasi-cylindrical C ABI (include/pic_circ.h).

Argument marshalling only: every step runs in the HIP library.  Field
planes are torch tensors E, B, J of shape [3 components (z, r, th),
3 channels (m 0, Re m 1, Im m 1), nr, nz] (z fastest); particles live in
caller-owned tensors with the pic_circ.h meaning of the species arrays.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .pic import (PIC_EINVAL, PIC_OK, CircDesc, CircFieldBufs, CircLaser, CircPlasma, Diag, PicError, Profile,
                  SpeciesBufs, lib)


def make_desc(nz, nr, dz, dr, dt, window_period=0, sort_interval=0, interleave=0, threads=0):
    return CircDesc(int(nz), int(nr), float(dz), float(dr), float(dt), int(window_period), int(sort_interval),
                    int(interleave), int(threads))


def validate(desc):
    buf = ctypes.create_string_buffer(256)
    st = lib().pic_circ_validate(ctypes.byref(desc), buf, 256)
    return st, buf.value.decode()


class CircSimulation:
    def __init__(self, nz, nr, dz, dr, dt, window_period=0, sort_interval=0, max_particles=0, device="cuda:0",
                 stream=None, interleave=0, threads=0):
        self.desc = make_desc(nz, nr, dz, dr, dt, window_period, sort_interval, interleave, threads)
        st, msg = validate(self.desc)
        if st != PIC_OK:
            raise PicError(st, msg)
        self.device = torch.device(device)
        self.nz, self.nr = int(nz), int(nr)
        shape = (3, 3, self.nr, self.nz)
        self.E = torch.zeros(shape, dtype=torch.float32, device=self.device)
        self.B = torch.zeros(shape, dtype=torch.float32, device=self.device)
        self.J = torch.zeros(shape, dtype=torch.float32, device=self.device)
        nbytes = int(lib().pic_circ_workspace_bytes(ctypes.byref(self.desc), int(max_particles)))
        if nbytes == 0:
            raise PicError(PIC_EINVAL, "workspace size query failed")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        fb = CircFieldBufs()
        for c in range(3):
            for ch in range(3):
                fb.E[3 * c + ch] = self.E[c, ch].data_ptr()
                fb.B[3 * c + ch] = self.B[c, ch].data_ptr()
                fb.J[3 * c + ch] = self.J[c, ch].data_ptr()
        h = ctypes.c_void_p()
        st = lib().pic_circ_init(ctypes.byref(h), ctypes.byref(self.desc), ctypes.byref(fb),
                                 ctypes.c_void_p(base + off), nbytes, int(max_particles),
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if st != PIC_OK:
            raise PicError(st, "pic_circ_init failed")
        self.handle = h
        self.species = []

    def _check(self, st):
        if st != PIC_OK:
            msg = lib().pic_circ_last_error(self.handle)
            raise PicError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "handle", None):
            lib().pic_circ_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ species and sources
    def add_species(self, cell, off, u, w, ids, q=-1.0, m=1.0, capacity=None):
        """cell = iz + nz jr; off = (z offset, x, y); u = (u_x, u_y, u_z); w charge weights."""
        n = int(len(cell))
        cap = int(capacity if capacity is not None else n)
        dev = self.device

        def buf(src, dtype):
            t = torch.zeros(cap, dtype=dtype, device=dev)
            if n:
                t[:n] = torch.as_tensor(np.asarray(src)).to(dev, dtype)
            return t

        sp = {"cell": buf(cell, torch.int32), "off": [buf(off[a], torch.float32) for a in range(3)],
              "u": [buf(u[a], torch.float32) for a in range(3)], "w": buf(w, torch.float32),
              "id": buf(ids, torch.int32)}
        sb = SpeciesBufs()
        sb.q, sb.m, sb.capacity = float(q), float(m), cap
        sb.cell = sp["cell"].data_ptr()
        for a in range(3):
            sb.off[a] = sp["off"][a].data_ptr()
            sb.u[a] = sp["u"][a].data_ptr()
        sb.w = sp["w"].data_ptr()
        sb.id = sp["id"].data_ptr()
        idx = ctypes.c_int32()
        self._check(lib().pic_circ_init_species(self.handle, ctypes.byref(sb), n, ctypes.byref(idx)))
        self.species.append(sp)
        return idx.value

    def add_empty_species(self, capacity, q=-1.0, m=1.0):
        z = np.zeros(0, np.int32)
        zf = np.zeros((3, 0), np.float32)
        return self.add_species(z, zf, zf, np.zeros(0, np.float32), z, q, m, capacity)

    def set_laser(self, a0, omega0, waist, fwhm, t_peak, t_end, src_z):
        L = CircLaser(float(a0), float(omega0), float(waist), float(fwhm), float(t_peak), float(t_end), int(src_z), 0)
        self._check(lib().pic_circ_set_laser(self.handle, ctypes.byref(L)))

    def set_plasma(self, s, z_start, ramp, n_plateau, ppc, r_cells, seed):
        P = CircPlasma(float(z_start), float(ramp), float(n_plateau), int(ppc), int(r_cells), int(seed))
        self._check(lib().pic_circ_set_plasma(self.handle, s, ctypes.byref(P)))

    def inject_plasma(self, s, z_begin, z_end):
        self._check(lib().pic_circ_inject_plasma(self.handle, s, int(z_begin), int(z_end)))

    def set_window(self, start_step):
        self._check(lib().pic_circ_set_window(self.handle, int(start_step)))

    def window_state(self):
        sh, org = ctypes.c_int64(), ctypes.c_int32()
        self._check(lib().pic_circ_window_state(self.handle, ctypes.byref(sh), ctypes.byref(org)))
        return sh.value, org.value

    # ------------------------------------------------------------ the cycle
    def gather_push(self, s=0):
        self._check(lib().pic_circ_gather_push(self.handle, s))

    def deposit(self, s=0):
        self._check(lib().pic_circ_deposit(self.handle, s))

    def field_step(self):
        self._check(lib().pic_circ_field_step(self.handle))

    def step(self, nsteps=1):
        self._check(lib().pic_circ_step(self.handle, int(nsteps)))

    def sync(self):
        self._check(lib().pic_circ_sync(self.handle))

    def reduce(self):
        d = Diag()
        self._check(lib().pic_circ_reduce(self.handle, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def profile_enable(self, on=True):
        self._check(lib().pic_circ_profile_enable(self.handle, 1 if on else 0))

    def profile_read(self):
        p = Profile()
        self._check(lib().pic_circ_profile_read(self.handle, ctypes.byref(p)))
        return {k: getattr(p, k) for k, _ in Profile._fields_}

    # ------------------------------------------------------------ views
    def particles_host(self, s=0):
        """Numpy copy of the species' arrays (count entries, removed ones included as cell < 0)."""
        sb = SpeciesBufs()
        n = ctypes.c_int64()
        self._check(lib().pic_circ_species_view(self.handle, s, ctypes.byref(sb), ctypes.byref(n)))
        k = n.value
        base = self.workspace.data_ptr()
        sp = self.species[s]

        def view(ptr, dtype):
            for t in [sp["cell"], sp["w"], sp["id"], *sp["off"], *sp["u"]]:
                if t.data_ptr() == ptr:
                    return t[:k].cpu().numpy()
            esz = torch.empty(0, dtype=dtype).element_size()
            o = ptr - base
            return self.workspace[o:o + k * esz].view(dtype).cpu().numpy()

        return {"cell": view(sb.cell, torch.int32), "off": np.stack([view(sb.off[a], torch.float32) for a in range(3)]),
                "u": np.stack([view(sb.u[a], torch.float32) for a in range(3)]), "w": view(sb.w, torch.float32),
                "id": view(sb.id, torch.int32)}

    def fields_complex(self):
        """(E, B, J) as complex128 [2 modes, 3 components, nr, nz] in window order."""
        _, org = self.window_state()
        out = []
        for T in (self.E, self.B, self.J):
            a = np.roll(T.cpu().numpy().astype(np.float64), -org, axis=3)
            out.append(np.stack([a[:, 0] + 0j, a[:, 1] + 1j * a[:, 2]]))
        return tuple(out)
