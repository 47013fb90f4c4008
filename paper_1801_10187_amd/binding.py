"""ctypes binding of libmpcd (include/mpcd.h): argument marshalling only.

Every step of the SRD path runs in the library's HIP kernels; this module
converts numpy arrays (or torch device tensors) to pointers and status codes
to exceptions. It raises at import of the library if libmpcd.so has not been
built; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB_PATH = os.path.join(HERE, "libmpcd.so")
HEADER = os.path.join(ROOT, "include", "mpcd.h")

MPCD_OK, MPCD_EINVAL, MPCD_ENOMEM, MPCD_EHIP, MPCD_ERANGE, MPCD_ESTATE = range(6)
FP64, FP32 = 0, 1
SRD, AT = 0, 1
FLAG_TIGHT_SLABS = 1
FLAG_MD_SOLUTE = 2
# tile shapes (bits 8-10 of flags; absent: chosen by density)
TILE_SHAPES = {"4x4x2": 1, "4x4x4": 2, "8x4x4": 3, "8x8x4": 4}


def tile_flag(shape):
    """flags bits of a tile shape name (None: the density rule)."""
    return 0 if shape is None else TILE_SHAPES[shape] << 8
NOALLOC_MAX_SHIFTS = 8192
STATUS_NAMES = {0: "MPCD_OK", 1: "MPCD_EINVAL", 2: "MPCD_ENOMEM", 3: "MPCD_EHIP",
                4: "MPCD_ERANGE", 5: "MPCD_ESTATE"}


class MpcdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int32 * 3),
                ("a", ctypes.c_double),
                ("alpha", ctypes.c_double),
                ("dt", ctypes.c_double),
                ("kT", ctypes.c_double),
                ("seed", ctypes.c_uint64),
                ("solvent_mass", ctypes.c_double),
                ("precision", ctypes.c_int32),
                ("thermostat", ctypes.c_int32),
                ("grid_shift", ctypes.c_int32),
                ("flags", ctypes.c_int32),
                ("collision", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def load():
    """Load libmpcd.so (built by paper_1801_10187_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run "
                          "`python -m paper_1801_10187_amd.build` first")
    # torch ships its own HIP runtime under the same soname as the system's.
    # Whichever is loaded first is the one the library links to; with torch
    # imported first, the library and torch share that one runtime (two
    # runtimes in one process leave torch without a device).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "mpcd_create": (st, [ctypes.POINTER(Params), ctypes.c_int64, _P, _P, ctypes.c_int64,
                              _P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
        "mpcd_stream": (st, [_P]),
        "mpcd_bin": (st, [_P]),
        "mpcd_collide": (st, [_P]),
        "mpcd_step": (st, [_P, ctypes.c_int64]),
        "mpcd_step_noalloc": (st, [_P, ctypes.c_int64]),
        "mpcd_get_state": (st, [_P, _P, _P, ctypes.c_int32]),
        "mpcd_get_cells": (st, [_P, _P, _P, ctypes.c_int32]),
        "mpcd_get_cell_props": (st, [_P, _P, _P, _P, ctypes.c_int32]),
        "mpcd_get_cell_draws": (st, [_P, _P, _P, ctypes.c_int32]),
        "mpcd_get_shift": (st, [_P, ctypes.c_uint64, _P]),
        "mpcd_get_step": (st, [_P, ctypes.POINTER(ctypes.c_uint64)]),
        "mpcd_set_step": (st, [_P, ctypes.c_uint64]),
        "mpcd_totals": (st, [_P, _P, _D, _D]),
        "mpcd_sync": (st, [_P]),
        "mpcd_get_sizes": (st, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_md_verlet_chains": (st, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int32, _P]),
        "mpcd_debug_fail_allocs": (st, [ctypes.c_int64, ctypes.c_int64]),
        "mpcd_handover_stats": (st, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_set_graph": (st, [ctypes.c_void_p, ctypes.c_int32]),
        "mpcd_graph_stats": (st, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_footprint": (st, [ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_get_layout": (st, [_P, _P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_profile_enable": (st, [_P, ctypes.c_int32]),
        "mpcd_profile_read": (st, [_P, ctypes.c_int32, _D, ctypes.POINTER(ctypes.c_int64)]),
        "mpcd_destroy": (None, [_P]),
        "mpcd_last_error": (ctypes.c_char_p, []),
        "mpcd_philox4x32_10": (st, [_P, ctypes.c_int64, ctypes.c_uint64, _P]),
        "mpcd_copy_kernel": (st, [_P, _P, ctypes.c_int64, _P]),
        "mpcd_copy_kernel_unrolled": (st, [_P, _P, ctypes.c_int64, _P]),
        "mpcd_create_batch": (st, [ctypes.c_int32, ctypes.POINTER(Params), _P, _P, _P,
                                   ctypes.c_int32, _P, ctypes.POINTER(_P)]),
        "mpcd_get_n_boxes": (st, [_P, ctypes.POINTER(ctypes.c_int32)]),
        "mpcd_get_box": (st, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64), _P, ctypes.c_uint64]),
        "mpcd_box_totals": (st, [_P, _P, _P, _P]),
        "mpcd_get_velocity_field": (st, [_P, _P, _P, ctypes.c_int32]),
        "mpcd_get_embedded": (st, [_P, _P, _P, ctypes.c_int32]),
        "mpcd_set_embedded": (st, [_P, _P, _P, ctypes.c_int32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols():
    """Entry points declared in include/mpcd.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mpcd_[a-z0-9_]+)\s*\(", text)))


def _check(status):
    if status != MPCD_OK:
        raise MpcdError(status, load().mpcd_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_params(n_cells, a=1.0, alpha=130.0 * math.pi / 180.0, dt=0.1, kT=1.0,
                seed=1, solvent_mass=1.0, precision=FP64, thermostat=False,
                grid_shift=True, flags=0, collision=0, tile=None):
    p = Params()
    n = [int(x) for x in np.broadcast_to(np.asarray(n_cells), (3,))]
    p.n_cells[:] = n
    p.a, p.alpha, p.dt, p.kT = float(a), float(alpha), float(dt), float(kT)
    p.seed = int(seed)
    p.solvent_mass = float(solvent_mass)
    p.precision = int(precision)
    p.thermostat = int(bool(thermostat)) if thermostat in (0, 1, True, False) else int(thermostat)
    p.grid_shift = int(bool(grid_shift)) if grid_shift in (0, 1, True, False) else int(grid_shift)
    p.flags = int(flags) | tile_flag(tile)
    p.collision = int(collision)
    return p


class Sim:
    """One SRD-MPCD system on the GPU (a thin owner of an mpcd_ctx)."""

    def __init__(self, pos, vel, n_cells, a=1.0, alpha=130.0 * math.pi / 180.0,
                 dt=0.1, kT=1.0, seed=1, solvent_mass=1.0, precision=FP64,
                 thermostat=False, grid_shift=True, emb_pos=None, emb_vel=None,
                 emb_mass=None, hip_stream=None, flags=0, collision=0, tile=None):
        lib = load()
        self.params = make_params(n_cells, a, alpha, dt, kT, seed, solvent_mass,
                                  precision, thermostat, grid_shift, flags, collision, tile)
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        n_emb = 0
        ep = ev = em = None
        if emb_pos is not None:
            ep = np.ascontiguousarray(emb_pos, dtype=np.float64).reshape(-1, 3)
            ev = np.ascontiguousarray(emb_vel, dtype=np.float64).reshape(-1, 3)
            em = np.ascontiguousarray(emb_mass, dtype=np.float64).reshape(-1)
            n_emb = ep.shape[0]
        ctx = ctypes.c_void_p()
        _check(lib.mpcd_create(ctypes.byref(self.params), pos.shape[0], _ptr(pos), _ptr(vel),
                               n_emb, _ptr(ep), _ptr(ev), _ptr(em), 0,
                               None if hip_stream is None else ctypes.c_void_p(hip_stream),
                               ctypes.byref(ctx)))
        self._ctx = ctx
        self.n_solvent = pos.shape[0]
        self.n_embedded = n_emb
        self.n_total = pos.shape[0] + n_emb
        self.ncells = int(np.prod([int(x) for x in self.params.n_cells]))

    # -- steps
    def stream(self):
        _check(load().mpcd_stream(self._ctx))

    def bin(self):
        _check(load().mpcd_bin(self._ctx))

    def collide(self):
        _check(load().mpcd_collide(self._ctx))

    def step(self, nsteps=1):
        _check(load().mpcd_step(self._ctx, int(nsteps)))

    def step_noalloc(self, nsteps=1):
        """mpcd_step_noalloc: the same steps without any allocation."""
        _check(load().mpcd_step_noalloc(self._ctx, int(nsteps)))

    def sync(self):
        _check(load().mpcd_sync(self._ctx))

    # -- readback
    def get_state(self):
        pos = np.empty((self.n_total, 3))
        vel = np.empty((self.n_total, 3))
        _check(load().mpcd_get_state(self._ctx, _ptr(pos), _ptr(vel), 0))
        return pos, vel

    def get_cells(self):
        cells = np.empty(self.n_total, dtype=np.int32)
        counts = np.empty(self.ncells, dtype=np.int32)
        _check(load().mpcd_get_cells(self._ctx, _ptr(cells), _ptr(counts), 0))
        return cells, counts

    def get_cell_props(self):
        mass = np.empty(self.ncells)
        mom = np.empty((self.ncells, 3))
        ek = np.empty(self.ncells)
        _check(load().mpcd_get_cell_props(self._ctx, _ptr(mass), _ptr(mom), _ptr(ek), 0))
        return mass, mom, ek

    def get_cell_draws(self):
        axis = np.empty((self.ncells, 3))
        xi = np.empty(self.ncells)
        _check(load().mpcd_get_cell_draws(self._ctx, _ptr(axis), _ptr(xi), 0))
        return axis, xi

    def get_embedded(self):
        """Positions and velocities (n_embedded, 3) of the embedded particles."""
        pos = np.empty((self.n_embedded, 3))
        vel = np.empty((self.n_embedded, 3))
        _check(load().mpcd_get_embedded(self._ctx, _ptr(pos), _ptr(vel), 0))
        return pos, vel

    def set_embedded(self, pos, vel):
        """Hand the embedded particles' state (from an MD integrator) over."""
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        vel = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1, 3)
        _check(load().mpcd_set_embedded(self._ctx, _ptr(pos), _ptr(vel), 0))

    def get_embedded_device(self, pos_ptr, vel_ptr):
        """get_embedded into device buffers of n_embedded x 3 doubles each."""
        _check(load().mpcd_get_embedded(self._ctx, ctypes.c_void_p(pos_ptr),
                                        ctypes.c_void_p(vel_ptr), 1))

    def set_embedded_device(self, pos_ptr, vel_ptr):
        """set_embedded from device buffers of n_embedded x 3 doubles each."""
        _check(load().mpcd_set_embedded(self._ctx, ctypes.c_void_p(pos_ptr),
                                        ctypes.c_void_p(vel_ptr), 1))

    def velocity_field(self):
        """Mass-weighted mean velocity (n_cells, 3) and mass (n_cells) per
        cell of the unshifted grid."""
        u = np.empty((self.ncells, 3))
        mass = np.empty(self.ncells)
        _check(load().mpcd_get_velocity_field(self._ctx, _ptr(u), _ptr(mass), 0))
        return u, mass

    def shift(self, n):
        s = np.empty(3)
        _check(load().mpcd_get_shift(self._ctx, int(n), _ptr(s)))
        return s

    @property
    def step_count(self):
        n = ctypes.c_uint64()
        _check(load().mpcd_get_step(self._ctx, ctypes.byref(n)))
        return n.value

    @step_count.setter
    def step_count(self, n):
        _check(load().mpcd_set_step(self._ctx, int(n)))

    def totals(self):
        p = np.empty(3)
        ke = ctypes.c_double()
        kT = ctypes.c_double()
        _check(load().mpcd_totals(self._ctx, _ptr(p), ctypes.byref(ke), ctypes.byref(kT)))
        return p, ke.value, kT.value

    def layout(self):
        """(tile size in cells, number of tiles, slots per tile, regrows)."""
        tile = (ctypes.c_int32 * 3)()
        nt, cap, rg = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(load().mpcd_get_layout(self._ctx, ctypes.cast(tile, ctypes.c_void_p), ctypes.byref(nt),
                                      ctypes.byref(cap), ctypes.byref(rg)))
        return tuple(tile), nt.value, cap.value, rg.value

    def handover_stats(self):
        """(kept, given up): solute handovers into a prepared binning."""
        k, g = ctypes.c_int64(), ctypes.c_int64()
        _check(load().mpcd_handover_stats(self._ctx, ctypes.byref(k), ctypes.byref(g)))
        return k.value, g.value

    # -- launch mode
    def set_graph(self, on=True):
        """Launch each stepping call's kernels as one HIP graph (mpcd_set_graph)."""
        _check(load().mpcd_set_graph(self._ctx, int(bool(on))))

    def graph_stats(self):
        """(instantiations, in-place updates) of the context's executable graph."""
        i, u = ctypes.c_int64(), ctypes.c_int64()
        _check(load().mpcd_graph_stats(self._ctx, ctypes.byref(i), ctypes.byref(u)))
        return i.value, u.value

    # -- timing
    def profile(self, on=True, every=1):
        """Time launches with HIP events: the first of each kind, then one in
        every `every` (mpcd_profile_enable)."""
        _check(load().mpcd_profile_enable(self._ctx, int(every) if on else 0))

    def profile_read(self, which=0):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().mpcd_profile_read(self._ctx, int(which), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_ctx", None):
            load().mpcd_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch(Sim):
    """Several independent SRD boxes stepped together (one mpcd_ctx made by
    mpcd_create_batch). `boxes` is a list of dicts with the keys pos, vel,
    n_cells and optionally a, alpha, dt, kT, seed, solvent_mass and tile (a
    TILE_SHAPES name); precision, thermostat, grid_shift and flags are common
    to all boxes. Every method of
    Sim works on all boxes at once; get_state/get_cells return the boxes one
    after the other (see box())."""

    def __init__(self, boxes, precision=FP64, thermostat=False, grid_shift=True,
                 hip_stream=None, flags=0, collision=0):
        lib = load()
        nb = len(boxes)
        arr = (Params * nb)()
        counts = np.empty(nb, dtype=np.int64)
        pos_l, vel_l = [], []
        for b, bx in enumerate(boxes):
            arr[b] = make_params(bx["n_cells"], bx.get("a", 1.0),
                                 bx.get("alpha", 130.0 * math.pi / 180.0), bx.get("dt", 0.1),
                                 bx.get("kT", 1.0), bx.get("seed", 1 + b),
                                 bx.get("solvent_mass", 1.0), precision, thermostat,
                                 grid_shift, flags, collision, bx.get("tile"))
            pos_l.append(np.asarray(bx["pos"], dtype=np.float64).reshape(-1, 3))
            vel_l.append(np.asarray(bx["vel"], dtype=np.float64).reshape(-1, 3))
            counts[b] = pos_l[-1].shape[0]
        pos = np.ascontiguousarray(np.concatenate(pos_l)) if nb else np.empty((0, 3))
        vel = np.ascontiguousarray(np.concatenate(vel_l)) if nb else np.empty((0, 3))
        ctx = ctypes.c_void_p()
        _check(lib.mpcd_create_batch(nb, arr, _ptr(counts), _ptr(pos), _ptr(vel), 0,
                                     None if hip_stream is None else ctypes.c_void_p(hip_stream),
                                     ctypes.byref(ctx)))
        self._ctx = ctx
        self.params = arr[0]
        self.box_params = arr
        self.n_boxes = nb
        self.n_solvent = int(counts.sum())
        self.n_embedded = 0
        self.n_total = self.n_solvent
        nt, nc = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.mpcd_get_sizes(ctx, ctypes.byref(nt), ctypes.byref(nc)))
        self.ncells = nc.value

    def box(self, b, step=0):
        """(first tag, particles, first cell, cells, shift of `step`) of box b."""
        t, n, c, nc = (ctypes.c_int64() for _ in range(4))
        s = np.empty(3)
        _check(load().mpcd_get_box(self._ctx, int(b), ctypes.byref(t), ctypes.byref(n),
                                   ctypes.byref(c), ctypes.byref(nc), _ptr(s), int(step)))
        return t.value, n.value, c.value, nc.value, s

    def box_totals(self):
        """Per box: momentum (n_boxes, 3), kinetic energy, temperature."""
        p = np.empty((self.n_boxes, 3))
        ke = np.empty(self.n_boxes)
        kT = np.empty(self.n_boxes)
        _check(load().mpcd_box_totals(self._ctx, _ptr(p), _ptr(ke), _ptr(kT)))
        return p, ke, kT


def md_verlet_chains(pos_ptr, vel_ptr, mass_ptr, n_chains, chain_len, box, dt, nsteps,
                     k_bond=30.0, bond_length=0.97, hip_stream=None):
    """mpcd_md_verlet_chains on device arrays (pointers): nsteps velocity-
    Verlet steps of harmonic bead chains, in place, enqueued on hip_stream."""
    b = (ctypes.c_double * 3)(*[float(x) for x in np.broadcast_to(np.asarray(box, float), (3,))])
    _check(load().mpcd_md_verlet_chains(ctypes.c_void_p(pos_ptr), ctypes.c_void_p(vel_ptr),
                                        ctypes.c_void_p(mass_ptr), int(n_chains), int(chain_len), b,
                                        float(k_bond), float(bond_length), float(dt), int(nsteps),
                                        None if hip_stream is None else ctypes.c_void_p(hip_stream)))


def debug_fail_allocs(after, count=1):
    """Test hook: after `after` more device allocations, `count` fail
    (mpcd_debug_fail_allocs; after < 0 turns it off)."""
    _check(load().mpcd_debug_fail_allocs(int(after), int(count)))


def footprint(n_cells, n_particles, nsteps=1, precision=FP32, host_arrays=True, **kw):
    """mpcd_footprint: (peak, held) device bytes of a one-box context."""
    p = make_params(n_cells, precision=precision, **kw)
    peak, held = ctypes.c_int64(), ctypes.c_int64()
    _check(load().mpcd_footprint(ctypes.byref(p), int(n_particles), int(nsteps), int(bool(host_arrays)),
                                 ctypes.byref(peak), ctypes.byref(held)))
    return peak.value, held.value


def philox(ctr, key):
    """Philox4x32-10 on the GPU: ctr (n, 4) uint32, key 64-bit int."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    _check(load().mpcd_philox4x32_10(_ptr(ctr), ctr.shape[0], int(key), _ptr(out)))
    return out


def copy_kernel(src_ptr, dst_ptr, nbytes, hip_stream=None, unrolled=False):
    """Device copy with the library's streaming kernel (device pointers);
    `unrolled` selects the four-vectors-per-thread variant."""
    fn = load().mpcd_copy_kernel_unrolled if unrolled else load().mpcd_copy_kernel
    _check(fn(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
              None if hip_stream is None else ctypes.c_void_p(hip_stream)))
