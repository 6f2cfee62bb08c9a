"""Python binding of libpicstep.so (include/picstep.h): argument marshalling
only.  Every step of the particle path runs in the HIP kernels of the library;
torch provides the device buffers and the stream.  There is no CPU fallback:
a missing library raises.
"""
import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libpicstep.so")

PIC_OK, PIC_E_ARG, PIC_E_RANGE, PIC_E_STATE, PIC_E_HIP, PIC_E_CAPACITY, PIC_E_UNSUPPORTED = range(7)
PIC_DEVERR_NONFINITE, PIC_DEVERR_SORT_MOVE = 1, 2
STATUS = {0: "PIC_OK", 1: "PIC_E_ARG", 2: "PIC_E_RANGE", 3: "PIC_E_STATE", 4: "PIC_E_HIP",
          5: "PIC_E_CAPACITY", 6: "PIC_E_UNSUPPORTED"}
GEOM = {"cart": 0, "sph": 1, "qsph": 2}
PREC = {"f32": 0, "f64": 1}
MAXSP = 8
NG = 2


class GridDesc(C.Structure):
    _fields_ = [("geom", C.c_int32), ("dim", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("r0", C.c_double),
                ("vartheta", C.c_double), ("periodic", C.c_int32 * 3), ("rho0", C.c_double),
                ("prec", C.c_int32), ("fp64_axis_cells", C.c_int32), ("sort_every", C.c_int32),
                ("reserved", C.c_int32), ("max_particles", C.c_uint64)]


class Sizes(C.Structure):
    _fields_ = [("fields_bytes", C.c_uint64), ("current_bytes", C.c_uint64),
                ("particle_set_bytes", C.c_uint64), ("prev_bytes", C.c_uint64),
                ("scratch_bytes", C.c_uint64), ("checkpoint_bytes", C.c_uint64),
                ("field_points", C.c_uint64), ("np", C.c_int32 * 3), ("elem_bytes", C.c_int32)]


class Buffers(C.Structure):
    _fields_ = [("fields", C.c_void_p), ("current", C.c_void_p), ("particles", C.c_void_p * 2),
                ("prev", C.c_void_p), ("scratch", C.c_void_p)]


class Layout(C.Structure):
    _fields_ = [("cell", C.c_uint64), ("offs", C.c_uint64 * 3), ("u", C.c_uint64 * 3),
                ("w", C.c_uint64), ("phi", C.c_uint64), ("capacity", C.c_uint64),
                ("species_offset", C.c_uint64 * MAXSP), ("species_capacity", C.c_uint64 * MAXSP),
                ("species_count", C.c_uint64 * MAXSP), ("nspecies", C.c_int32),
                ("active_set", C.c_int32), ("shift2", C.c_int32), ("shift3", C.c_int32),
                ("prev_cell", C.c_uint64), ("prev_offs", C.c_uint64 * 3), ("id", C.c_uint64)]


class Timing(C.Structure):
    _fields_ = [("push_launches", C.c_int64), ("push_ms", C.c_double), ("sort_calls", C.c_int64),
                ("sort_ms", C.c_double), ("adjoint_launches", C.c_int64), ("adjoint_ms", C.c_double),
                ("push_blocks", C.c_int64), ("push_global_particles", C.c_int64),
                ("sort_brick_calls", C.c_int64)]


class AdjointBuffers(C.Structure):
    _fields_ = [("lam_u", C.c_void_p), ("lam_offs", C.c_void_p), ("dEB", C.c_void_p),
                ("lamJ_work", C.c_void_p)]


class ParticleView(C.Structure):
    _fields_ = [("n", C.c_uint64), ("cell", C.POINTER(C.c_int32)), ("offs", C.POINTER(C.c_double)),
                ("u", C.POINTER(C.c_double)), ("w", C.POINTER(C.c_double)),
                ("phi", C.POINTER(C.c_double)), ("alive", C.POINTER(C.c_int32)),
                ("cell_prev", C.POINTER(C.c_int32)), ("offs_prev", C.POINTER(C.c_double)),
                ("perm", C.POINTER(C.c_int32)), ("id", C.POINTER(C.c_int32))]


_LIB = None


def lib():
    """Load libpicstep.so; raises if it was not built (no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with "
                               "`python -m paper_2511_17710_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIBPATH)
        vp, i32, u64, dbl = C.c_void_p, C.c_int32, C.c_uint64, C.c_double
        sig = {
            "pic_grid_init": [C.POINTER(GridDesc), C.POINTER(vp)],
            "pic_grid_destroy": [vp],
            "pic_query_sizes": [vp, C.POINTER(Sizes)],
            "pic_bind_buffers": [vp, C.POINTER(Buffers)],
            "pic_set_stream": [vp, vp],
            "pic_timestep_from_cfl": [vp, dbl, C.POINTER(dbl)],
            "pic_species_add": [vp, dbl, dbl, u64, C.POINTER(i32)],
            "pic_species_set_pusher": [vp, i32, i32, dbl, dbl],
            "pic_fields_set": [vp, vp, i32, i32],
            "pic_fields_fill_ghosts": [vp],
            "pic_particles_load": [vp, i32, u64, vp, vp, vp, vp, vp],
            "pic_sort": [vp],
            "pic_sort_static": [vp],
            "pic_push_deposit": [vp, dbl, i32],
            "pic_fields_advance_b": [vp, dbl],
            "pic_fields_advance_e": [vp, dbl, dbl],
            "pic_current_filter": [vp, i32, vp],
            "pic_step_full": [vp, dbl, i32, i32, dbl, vp],
            "pic_current_get": [vp, vp, i32],
            "pic_fields_get": [vp, vp, i32],
            "pic_particles_get": [vp, i32, C.POINTER(ParticleView)],
            "pic_particle_layout": [vp, C.POINTER(Layout)],
            "pic_step_count": [vp, C.POINTER(C.c_int64)],
            "pic_adjoint_workspace": [vp, i32, i32, C.POINTER(u64)],
            "pic_forward_checkpointed": [vp, dbl, i32, i32, vp],
            "pic_backward": [vp, dbl, i32, i32, vp, vp, vp, vp, vp],
            "pic_checkpointed_order": [vp, vp, vp],
            "pic_checkpoint_save": [vp, vp],
            "pic_checkpoint_load": [vp, vp],
            "pic_adjoint_step": [vp, dbl, vp, C.POINTER(AdjointBuffers)],
            "pic_last_error": [vp],
            "pic_timing_enable": [vp, i32],
            "pic_timing_read": [vp, C.POINTER(Timing)],
            "pic_device_errors": [vp, C.POINTER(C.c_int32), i32],
            "pic_particles_modified": [vp],
            "pic_debug_serial": [vp, i32],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name == "pic_grid_destroy" else (
                C.c_char_p if name == "pic_last_error" else C.c_int)
        _LIB = L
    return _LIB


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """One library context with its torch-allocated device buffers."""

    def __init__(self, geom, dim, n, lo, hi, r0=0.0, vartheta=0.0, periodic=(1, 1, 1),
                 rho0=1.0, prec="f32", fp64_axis_cells=2, sort_every=20, max_particles=1,
                 device="cuda"):
        d = GridDesc()
        d.geom = GEOM[geom] if isinstance(geom, str) else int(geom)
        d.dim = int(dim)
        n = list(n) + [1] * (3 - len(n))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        for a in range(3):
            d.n[a], d.lo[a], d.hi[a], d.periodic[a] = int(n[a]), float(lo[a]), float(hi[a]), int(periodic[a])
        d.r0, d.vartheta, d.rho0 = float(r0), float(vartheta), float(rho0)
        d.prec = PREC[prec]
        d.fp64_axis_cells = int(fp64_axis_cells)
        d.sort_every = int(sort_every)
        d.max_particles = int(max_particles)
        self.desc = d
        self.prec = prec
        self.dtype = torch.float32 if prec == "f32" else torch.float64
        self.device = device
        self.dim = d.dim
        self.geom = d.geom
        self.n = tuple(n)
        h = C.c_void_p()
        st = lib().pic_grid_init(C.byref(d), C.byref(h))
        if st != PIC_OK:
            raise PicError(st, "pic_grid_init rejected the grid description")
        self.h = h
        self.bufs = None
        self.species = []

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().pic_grid_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -------------------------------------------------------------- helpers
    def _check(self, st, what):
        if st != PIC_OK:
            msg = lib().pic_last_error(self.h)
            raise PicError(st, f"{what}: {msg.decode() if msg else ''}")

    def sizes(self):
        s = Sizes()
        self._check(lib().pic_query_sizes(self.h, C.byref(s)), "query_sizes")
        return s

    def layout(self):
        L = Layout()
        self._check(lib().pic_particle_layout(self.h, C.byref(L)), "particle_layout")
        return L

    def padded_shape(self):
        s = self.sizes()
        return (s.np[2], s.np[1], s.np[0])

    # -------------------------------------------------------------- setup
    def species_add(self, q, m, capacity):
        sid = C.c_int32()
        self._check(lib().pic_species_add(self.h, float(q), float(m), int(capacity), C.byref(sid)),
                    "species_add")
        self.species.append((q, m, capacity))
        return sid.value

    def species_set_pusher(self, s, pusher="boris", gca=False, e_ovr=0.9, larmor_max=0.0):
        """pusher "boris" or "vay"; gca=True adds the guiding-centre hybrid."""
        code = {"boris": 0, "vay": 1}[pusher] | (2 if gca else 0)
        self._check(lib().pic_species_set_pusher(self.h, int(s), code, float(e_ovr),
                                                 float(larmor_max)), "species_set_pusher")

    def bind(self, stream=None):
        """Allocate every device buffer with torch and register it."""
        s = self.sizes()

        def alloc(nb):
            return torch.empty(max(int(nb), 256), dtype=torch.uint8, device=self.device)

        self.bufs = dict(fields=alloc(s.fields_bytes), current=alloc(s.current_bytes),
                         p0=alloc(s.particle_set_bytes), p1=alloc(s.particle_set_bytes),
                         prev=alloc(s.prev_bytes), scratch=alloc(s.scratch_bytes))
        b = Buffers()
        b.fields = self.bufs["fields"].data_ptr()
        b.current = self.bufs["current"].data_ptr()
        b.particles[0] = self.bufs["p0"].data_ptr()
        b.particles[1] = self.bufs["p1"].data_ptr()
        b.prev = self.bufs["prev"].data_ptr()
        b.scratch = self.bufs["scratch"].data_ptr()
        self.set_stream(stream)
        self._check(lib().pic_bind_buffers(self.h, C.byref(b)), "bind_buffers")

    def set_stream(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.stream = st
        self._check(lib().pic_set_stream(self.h, C.c_void_p(st.cuda_stream)), "set_stream")

    def timestep_from_cfl(self, cfl):
        dt = C.c_double()
        self._check(lib().pic_timestep_from_cfl(self.h, float(cfl), C.byref(dt)), "timestep")
        return dt.value

    def fields_set(self, EB, basis="tetrad", includes_ghosts=0):
        EB = np.ascontiguousarray(EB, dtype=np.float64)
        self._check(lib().pic_fields_set(self.h, _ptr(EB), 1 if basis == "tetrad" else 0,
                                         int(includes_ghosts)), "fields_set")

    def fields_fill_ghosts(self):
        self._check(lib().pic_fields_fill_ghosts(self.h), "fields_fill_ghosts")

    def particles_load(self, s, cell, offs, u, w, phi=None):
        n = int(np.asarray(cell).shape[0])
        D = self.dim
        cell = np.ascontiguousarray(np.asarray(cell)[:, :D], dtype=np.int32)
        offs = np.ascontiguousarray(np.asarray(offs)[:, :D], dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        phi = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
        self._check(lib().pic_particles_load(self.h, int(s), n, _ptr(cell), _ptr(offs), _ptr(u),
                                             _ptr(w), _ptr(phi)), "particles_load")

    # -------------------------------------------------------------- the step
    def sort(self):
        self._check(lib().pic_sort(self.h), "sort")

    def sort_static(self):
        """pic_sort with the radix temporaries in the library's static device
        array (no allocation; at most 2^22 particles per species)."""
        self._check(lib().pic_sort_static(self.h), "sort_static")

    def debug_serial(self, on=True):
        """Debug launch mode: the fused step kernel one block at a time."""
        self._check(lib().pic_debug_serial(self.h, int(bool(on))), "debug_serial")

    def particles_modified(self):
        """The particle arrays were written through the bound buffers."""
        self._check(lib().pic_particles_modified(self.h), "particles_modified")

    def device_errors(self, clear=True):
        """The sticky device error word (PIC_DEVERR_* bits); waits for the stream."""
        v = C.c_int32(0)
        self._check(lib().pic_device_errors(self.h, C.byref(v), int(bool(clear))), "device_errors")
        return int(v.value)

    def push_deposit(self, dt, n_steps):
        self._check(lib().pic_push_deposit(self.h, float(dt), int(n_steps)), "push_deposit")

    # -------------------------------------------------------------- field solver
    def _work(self):
        w = getattr(self, "_jwork", None)
        if w is None:
            w = torch.empty(max(int(self.sizes().current_bytes), 256), dtype=torch.uint8,
                            device=self.device)
            self._jwork = w
        return C.c_void_p(w.data_ptr())

    def fields_advance_b(self, f):
        """Faraday: B -= f curl E / sqrt(h)."""
        self._check(lib().pic_fields_advance_b(self.h, float(f)), "fields_advance_b")

    def fields_advance_e(self, dt, coupling=4 * np.pi):
        """Ampere with the bound current: E += dt (curl B - coupling J) / sqrt(h)."""
        self._check(lib().pic_fields_advance_e(self.h, float(dt), float(coupling)),
                    "fields_advance_e")

    def current_filter(self, passes):
        self._check(lib().pic_current_filter(self.h, int(passes), self._work()), "current_filter")

    def step_full(self, dt, n_steps, filter_passes=0, coupling=4 * np.pi):
        """n_steps of the whole loop (fields evolved with the particles)."""
        w = self._work() if filter_passes > 0 else None
        self._check(lib().pic_step_full(self.h, float(dt), int(n_steps), int(filter_passes),
                                        float(coupling), w), "step_full")

    def step_count(self):
        v = C.c_int64()
        self._check(lib().pic_step_count(self.h, C.byref(v)), "step_count")
        return v.value

    # -------------------------------------------------------------- adjoint
    def adjoint_workspace(self, K, m):
        nb = C.c_uint64()
        self._check(lib().pic_adjoint_workspace(self.h, int(K), int(m), C.byref(nb)),
                    "adjoint_workspace")
        return nb.value

    def forward_checkpointed(self, dt, K, m):
        """K steps as push_deposit runs them (sorts included); the state is
        kept every m steps, with every sort's permutation, in a
        torch-allocated workspace for backward()."""
        nb = self.adjoint_workspace(K, m)
        ws = getattr(self, "_ws", None)
        if ws is None or ws.numel() < nb:
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            self._ws = ws
        self._check(lib().pic_forward_checkpointed(self.h, float(dt), int(K), int(m),
                                                   C.c_void_p(ws.data_ptr())), "forward_checkpointed")
        self.forward_generation = getattr(self, "forward_generation", 0) + 1
        return self.forward_generation

    def backward(self, dt, K, m, lamJ=None, lam_u=None):
        """dL/d(fields) [6, np3, np2, np1] and dL/du0 [3, capacity] for
        L = sum(lamJ * J_K) + sum(lam_u * u_K)."""
        cap = self.layout().capacity
        dEB = torch.empty((6,) + self.padded_shape(), dtype=self.dtype, device=self.device)
        du0 = torch.empty((3, cap), dtype=self.dtype, device=self.device)

        def ptr(t, shape):
            if t is None:
                return None
            t = t.to(device=self.device, dtype=self.dtype).contiguous()
            assert tuple(t.shape) == tuple(shape), (t.shape, shape)
            keep.append(t)
            return C.c_void_p(t.data_ptr())

        keep = []
        pJ = ptr(lamJ, (3,) + self.padded_shape())
        pu = ptr(lam_u, (3, cap))
        self._check(lib().pic_backward(self.h, float(dt), int(K), int(m),
                                       C.c_void_p(self._ws.data_ptr()), pJ, pu,
                                       C.c_void_p(dEB.data_ptr()), C.c_void_p(du0.data_ptr())),
                    "backward")
        torch.cuda.current_stream(self.device).synchronize()
        return dEB, du0

    # -------------------------------------------------------------- low-level adjoint
    def checkpoint_slot(self):
        """A torch device buffer for one particle-state checkpoint."""
        return torch.empty(max(int(self.sizes().checkpoint_bytes), 256), dtype=torch.uint8,
                           device=self.device)

    def checkpoint_save(self, slot):
        self._check(lib().pic_checkpoint_save(self.h, C.c_void_p(slot.data_ptr())),
                    "checkpoint_save")

    def checkpoint_load(self, slot):
        self._check(lib().pic_checkpoint_load(self.h, C.c_void_p(slot.data_ptr())),
                    "checkpoint_load")

    def adjoint_step(self, dt, lam_u, lam_offs, dEB, lamJ=None, work=None):
        """Reverse of one step from the current state: lam_u, lam_offs
        ([3, capacity]) are updated in place, dEB ([6, np3, np2, np1]) is
        accumulated; lamJ ([3, np3, np2, np1]) needs a work buffer of the same
        shape."""
        b = AdjointBuffers()
        b.lam_u = lam_u.data_ptr()
        b.lam_offs = lam_offs.data_ptr()
        b.dEB = dEB.data_ptr()
        pJ = None
        if lamJ is not None:
            if work is None:
                work = torch.empty_like(lamJ)
            b.lamJ_work = work.data_ptr()
            pJ = C.c_void_p(lamJ.data_ptr())
        self._check(lib().pic_adjoint_step(self.h, float(dt), pJ, C.byref(b)), "adjoint_step")

    def checkpointed_order(self):
        """int32 [capacity]: for each particle slot at step K of the last
        forward_checkpointed, its slot at step 0."""
        out = np.zeros(self.layout().capacity, dtype=np.int32)
        self._check(lib().pic_checkpointed_order(self.h, C.c_void_p(self._ws.data_ptr()),
                                                 out.ctypes.data_as(C.c_void_p)),
                    "checkpointed_order")
        return out

    def timing_enable(self, on=True):
        self._check(lib().pic_timing_enable(self.h, 1 if on else 0), "timing_enable")

    def timing_read(self):
        t = Timing()
        self._check(lib().pic_timing_read(self.h, C.byref(t)), "timing_read")
        return {k: getattr(t, k) for k, _ in Timing._fields_}

    # -------------------------------------------------------------- views / readback
    def _view(self, buf, byte_off, count, dtype):
        esz = torch.tensor([], dtype=dtype).element_size()
        return self.bufs[buf][byte_off:byte_off + count * esz].view(dtype)

    def current(self):
        """Device view [3, np3, np2, np1] of the current buffer."""
        s = self.sizes()
        return self._view("current", 0, 3 * s.field_points, self.dtype).view((3,) + self.padded_shape())

    def fields(self):
        """Device view [6, np3, np2, np1] of the contravariant field buffer."""
        s = self.sizes()
        return self._view("fields", 0, 6 * s.field_points, self.dtype).view((6,) + self.padded_shape())

    def particle_arrays(self):
        """Device views of the active particle set (whole capacity).  They are
        writable, so the library is told that the arrays may change behind its
        back (the next sort assumes nothing about the moves since the last)."""
        self._check(lib().pic_particles_modified(self.h), "particles_modified")
        L = self.layout()
        buf = "p1" if L.active_set else "p0"
        cap = L.capacity
        none = (1 << 64) - 1
        out = dict(cell=self._view(buf, L.cell, cap, torch.int32),
                   u=[self._view(buf, L.u[a], cap, self.dtype) for a in range(3)],
                   offs=[self._view(buf, L.offs[a], cap, self.dtype) for a in range(self.dim)],
                   w=self._view(buf, L.w, cap, self.dtype),
                   id=self._view(buf, L.id, cap, torch.int32))
        if L.phi != none:
            out["phi"] = self._view(buf, L.phi, cap, self.dtype)
        return out

    def particles_get(self, s):
        L = self.layout()
        n = int(L.species_count[s])
        out = dict(cell=np.zeros((n, 3), np.int32), offs=np.zeros((n, 3)), u=np.zeros((n, 3)),
                   w=np.zeros(n), phi=np.zeros(n) if self.geom != 0 else None,
                   alive=np.zeros(n, np.int32), cell_prev=np.zeros((n, 3), np.int32),
                   offs_prev=np.zeros((n, 3)), perm=np.zeros(n, np.int32), id=np.zeros(n, np.int32))
        v = ParticleView()
        v.n = n
        for k in ("cell", "alive", "cell_prev", "perm", "id"):
            setattr(v, k, out[k].ctypes.data_as(C.POINTER(C.c_int32)))
        for k in ("offs", "u", "w", "offs_prev"):
            setattr(v, k, out[k].ctypes.data_as(C.POINTER(C.c_double)))
        if out["phi"] is not None:
            v.phi = out["phi"].ctypes.data_as(C.POINTER(C.c_double))
        self._check(lib().pic_particles_get(self.h, int(s), C.byref(v)), "particles_get")
        return out

    def current_host(self):
        J = np.zeros((3,) + self.padded_shape(),
                     dtype=np.float32 if self.prec == "f32" else np.float64)
        self._check(lib().pic_current_get(self.h, _ptr(J), 0), "current_get")
        return J

    def fields_host(self):
        F = np.zeros((6,) + self.padded_shape(),
                     dtype=np.float32 if self.prec == "f32" else np.float64)
        self._check(lib().pic_fields_get(self.h, _ptr(F), 0), "fields_get")
        return F


def from_workload(wl, prec="f32", device="cuda", sort_every=None, fp64_axis_cells=2,
                  capacity_slack=0):
    """Context for a workloads.Workload: grid, species, fields and particles loaded."""
    caps = [s["cell"].shape[0] + capacity_slack for s in wl.species]
    ctx = Context(wl.geom, wl.dim, wl.n, wl.lo, wl.hi, r0=wl.r0, vartheta=wl.vartheta,
                  periodic=wl.periodic, rho0=wl.rho0, prec=prec, fp64_axis_cells=fp64_axis_cells,
                  sort_every=wl.sort_every if sort_every is None else sort_every,
                  max_particles=sum(caps), device=device)
    for i, (s, cap) in enumerate(zip(wl.species, caps)):
        ctx.species_add(s["q"], s["m"], cap)
        code = int(s.get("pusher", 0))
        if code:
            ctx.species_set_pusher(i, "vay" if code & 1 else "boris", gca=bool(code & 2),
                                   e_ovr=s.get("e_ovr", 0.9), larmor_max=s.get("larmor_max", 0.0))
    ctx.bind()
    ctx.fields_set(wl.fields_tetrad, "tetrad", wl.fields_includes_ghosts)
    for i, s in enumerate(wl.species):
        ctx.particles_load(i, s["cell"], s["offs"], s["u"], s["w"], s.get("phi"))
    return ctx
