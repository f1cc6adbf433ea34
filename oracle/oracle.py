"""ctypes wrapper of the FP64 CPU oracle (oracle/lbm_oracle.cpp).

Test infrastructure only: imported by tests/, by the package smoke check and by
the CPU-baseline leg of bench.py. The product path never imports this module.

Moment arrays use the layout [block][moment][node]; moments are
(rho-1, ux, uy, uz, Sxx, Syy, Szz, Sxy, Sxz, Syz), node index x + 8y + 64z,
blocks listed in increasing Morton order of their block coordinates.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")

PERIODIC, INFLOW, OUTFLOW, WALL, OUTFLOW_CONV = 0, 1, 2, 3, 4
R_INTERIOR, R_GHOST, R_IU, R_SOLID, R_INFLOW, R_OUTFLOW = range(6)


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("n", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("uin", ctypes.c_double * 3),
        ("tau0", ctypes.c_double),
        ("force", ctypes.c_double * 3),
        ("rescale", ctypes.c_int32),
        ("storage", ctypes.c_int32),
        ("scale", ctypes.c_double * 10),
        ("inflow_profile", ctypes.c_int32),
        ("inflow_axis", ctypes.c_int32),
        ("inflow_beta", ctypes.c_double),
        ("inflow_h0", ctypes.c_double),
    ]


def _set_log_inflow(c, log_inflow):
    """log_inflow = (axis, beta, h0): inflow velocity uin * ln(1 + beta (h - h0)) at
    height h (fine units) along axis, zero at or below h0; None: uniform uin."""
    if log_inflow is None:
        c.inflow_profile = 0
        return
    axis, beta, h0 = log_inflow
    c.inflow_profile = 1
    c.inflow_axis = int(axis)
    c.inflow_beta = float(beta)
    c.inflow_h0 = float(h0)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from oracle.build import build
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.oc_create.restype = vp
        L.oc_create.argtypes = [ctypes.POINTER(_Cfg), vp, vp, i64]
        L.oc_destroy.argtypes = [vp]
        L.oc_last_error.restype = ctypes.c_char_p
        L.oc_num_blocks.restype = i64
        L.oc_num_blocks.argtypes = [vp, i32]
        L.oc_block_keys.argtypes = [vp, i32, vp]
        L.oc_set_block_moments.restype = i32
        L.oc_set_block_moments.argtypes = [vp, i32, vp, vp, i64]
        L.oc_get_block_moments.argtypes = [vp, i32, vp, vp]
        L.oc_set_coupling.restype = i32
        L.oc_set_coupling.argtypes = [vp, vp, vp, i64]
        L.oc_scalar_set.restype = i32
        L.oc_scalar_set.argtypes = [vp, vp, vp, i64]
        L.oc_scalar_get.argtypes = [vp, vp]
        L.oc_scalar_advance.argtypes = [vp, ctypes.c_double, ctypes.c_double, vp]
        L.oc_get_roles.argtypes = [vp, i32, vp]
        L.oc_step.restype = i32
        L.oc_step.argtypes = [vp, i32]
        L.oc_step_finest.restype = i32
        L.oc_step_finest.argtypes = [vp, i32]
        L.oc_finest_phase.restype = i32
        L.oc_finest_phase.argtypes = [vp]
        L.oc_remesh.restype = i32
        L.oc_remesh.argtypes = [vp, vp, i64]
        L.oc_advance_particles.argtypes = [vp, i64, vp]
        L.oc_reduce.argtypes = [vp, i32, vp, vp, vp]
        L.oc_level_params.argtypes = [vp, vp, vp, vp]
        L.oc_lattice.argtypes = [vp, vp]
        L.oc_reconstruct.argtypes = [vp, vp]
        L.oc_collide.argtypes = [vp, ctypes.c_double, vp, vp]
        L.oc_num_threads.restype = ctypes.c_int
        L.oc_set_num_threads.argtypes = [ctypes.c_int]
        L.oc_loss_ke.restype = ctypes.c_double
        L.oc_loss_ke.argtypes = [vp, i32, vp, vp]
        L.occ_create.restype = vp
        L.occ_create.argtypes = [ctypes.POINTER(_Cfg), vp, vp, i64]
        L.occ_destroy.argtypes = [vp]
        L.occ_set_block_moments.restype = i32
        L.occ_set_block_moments.argtypes = [vp, i32, vp, vp, vp, i64]
        L.occ_step.restype = i32
        L.occ_step.argtypes = [vp, i32]
        L.occ_loss_ke.argtypes = [vp, i32, vp, vp, vp]
        L.occ_remesh.restype = i32
        L.occ_remesh.argtypes = [vp, vp, i64]
        L.oc_store_round.restype = ctypes.c_double
        L.oc_store_round.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_double]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleSim:
    """One simulation held by the oracle."""

    def __init__(self, levels, n, bc, tau0, uin=(0.0, 0.0, 0.0), force=(0.0, 0.0, 0.0),
                 solid=None, particles=None, rescale="ce", storage="exact", scale=None, log_inflow=None):
        c = _Cfg()
        _set_log_inflow(c, log_inflow)
        c.levels = levels
        for a in range(3):
            c.n[a] = int(n[a])
            c.uin[a] = float(uin[a])
            c.force[a] = float(force[a])
        for f in range(6):
            c.bc[f] = int(bc[f])
        c.tau0 = float(tau0)
        c.rescale = {"ce": 0, "printed": 1}[rescale]
        c.storage = {"exact": 0, "bf16": 1, "f16": 2}[storage]
        sc = [1.0] * 10 if scale is None else list(scale)
        for m in range(10):
            c.scale[m] = float(sc[m])
        self.levels = levels
        self.n = tuple(int(v) for v in n)
        self._solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        p = None if particles is None else np.ascontiguousarray(particles, dtype=np.float32)
        np_ = 0 if p is None else p.shape[0]
        h = lib().oc_create(ctypes.byref(c), _ptr(self._solid), _ptr(p), np_)
        if not h:
            raise ValueError(lib().oc_last_error().decode())
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().oc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def scalar_set(self, keys, phi):
        """Powder-snow volume fraction of finest-level blocks `keys`: phi [nb, 512]."""
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        f = np.ascontiguousarray(phi, dtype=np.float64)
        assert f.shape == (len(keys), 512)
        if lib().oc_scalar_set(self.h, _ptr(keys), _ptr(f), len(keys)) != 0:
            raise ValueError(lib().oc_last_error().decode())

    def scalar_get(self):
        """phi of every finest-level block, [nb, 512] in key order."""
        out = np.empty((self.num_blocks(0), 512))
        lib().oc_scalar_get(self.h, _ptr(out))
        return out

    def scalar_advance(self, dt, D, source=None):
        src = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
        lib().oc_scalar_advance(self.h, float(dt), float(D), _ptr(src))

    def set_coupling(self, keys, fields):
        """Finest-level coupling fields of blocks `keys`: fields [nb, 4, 512] = (eps, Fx, Fy, Fz),
        eps the fluid fraction (tau scaled to eps tau), F the force density."""
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        f = np.ascontiguousarray(fields, dtype=np.float64)
        assert f.shape == (len(keys), 4, 512)
        if lib().oc_set_coupling(self.h, _ptr(keys), _ptr(f), len(keys)) != 0:
            raise ValueError(lib().oc_last_error().decode())

    def num_blocks(self, level):
        return int(lib().oc_num_blocks(self.h, level))

    def block_keys(self, level):
        k = np.empty(self.num_blocks(level), dtype=np.int64)
        lib().oc_block_keys(self.h, level, _ptr(k))
        return k

    def set_block_moments(self, level, keys, vals):
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        vals = np.ascontiguousarray(vals, dtype=np.float64)
        assert vals.shape == (keys.shape[0], 10, 512)
        if lib().oc_set_block_moments(self.h, level, _ptr(keys), _ptr(vals), keys.shape[0]) != 0:
            raise ValueError(lib().oc_last_error().decode())

    def get_block_moments(self, level):
        nb = self.num_blocks(level)
        k = np.empty(nb, dtype=np.int64)
        v = np.empty((nb, 10, 512), dtype=np.float64)
        lib().oc_get_block_moments(self.h, level, _ptr(k), _ptr(v))
        return k, v

    def roles(self, level):
        r = np.empty((self.num_blocks(level), 512), dtype=np.uint8)
        lib().oc_get_roles(self.h, level, _ptr(r))
        return r

    def step(self, n=1):
        if lib().oc_step(self.h, n) != 0:
            raise RuntimeError(lib().oc_last_error().decode())

    def step_finest(self, n=1):
        """n finest-level steps (Alg. 1 walked up to the end of each finest step)."""
        if lib().oc_step_finest(self.h, int(n)) != 0:
            raise RuntimeError(lib().oc_last_error().decode())

    def finest_phase(self):
        return int(lib().oc_finest_phase(self.h))

    def remesh(self, particles):
        p = np.ascontiguousarray(particles, dtype=np.float32)
        if lib().oc_remesh(self.h, _ptr(p), p.shape[0]) != 0:
            raise RuntimeError(lib().oc_last_error().decode())

    def reduce(self, level, lo=(0, 0, 0), hi=None):
        hi = self.n if hi is None else hi
        lo_ = np.array(lo, dtype=np.int32)
        hi_ = np.array(hi, dtype=np.int32)
        out = np.empty(5, dtype=np.float64)
        lib().oc_reduce(self.h, level, _ptr(lo_), _ptr(hi_), _ptr(out))
        return out

    def kinetic_energy(self, level, lo, hi):
        lo_ = np.array(lo, dtype=np.int32)
        hi_ = np.array(hi, dtype=np.int32)
        return float(lib().oc_loss_ke(self.h, level, _ptr(lo_), _ptr(hi_)))

    def level_params(self):
        t = np.empty(self.levels)
        u = np.empty(self.levels)
        d = np.empty(self.levels)
        lib().oc_level_params(self.h, _ptr(t), _ptr(u), _ptr(d))
        return t, u, d


class OracleSimComplex:
    """The same oracle on std::complex<double>, for complex-step derivatives: set
    moments with an imaginary part h*d, step, read the imaginary part of the loss."""

    def __init__(self, levels, n, bc, tau0, particles=None, solid=None, uin=(0.0, 0.0, 0.0), rescale="ce",
                 log_inflow=None):
        self._real = OracleSim(levels, n, bc, tau0, uin=uin, solid=solid, particles=particles, rescale=rescale,
                               log_inflow=log_inflow)
        c = _Cfg()
        _set_log_inflow(c, log_inflow)
        c.levels = levels
        for a in range(3):
            c.n[a] = int(n[a])
            c.uin[a] = float(uin[a])
        for f in range(6):
            c.bc[f] = int(bc[f])
        c.tau0 = float(tau0)
        c.rescale = {"ce": 0, "printed": 1}[rescale]
        self.levels = levels
        p = None if particles is None else np.ascontiguousarray(particles, dtype=np.float32)
        self._solid = None if solid is None else np.ascontiguousarray(solid, dtype=np.uint8)
        h = lib().occ_create(ctypes.byref(c), _ptr(self._solid), _ptr(p), 0 if p is None else p.shape[0])
        if not h:
            raise ValueError(lib().oc_last_error().decode())
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().occ_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def block_keys(self, level):
        return self._real.block_keys(level)

    def set_block_moments(self, level, keys, re, im=None):
        keys = np.ascontiguousarray(keys, dtype=np.int64)
        re = np.ascontiguousarray(re, dtype=np.float64)
        im = None if im is None else np.ascontiguousarray(im, dtype=np.float64)
        if lib().occ_set_block_moments(self.h, level, _ptr(keys), _ptr(re), _ptr(im), keys.shape[0]) != 0:
            raise ValueError(lib().oc_last_error().decode())

    def step(self, n=1):
        if lib().occ_step(self.h, n) != 0:
            raise RuntimeError(lib().oc_last_error().decode())

    def remesh(self, particles):
        """Grid update of both the complex instance and the real one that names its blocks."""
        p = np.ascontiguousarray(particles, dtype=np.float32)
        if lib().occ_remesh(self.h, _ptr(p), p.shape[0]) < 0:
            raise RuntimeError(lib().oc_last_error().decode())
        self._real.remesh(p)

    def kinetic_energy(self, level, lo, hi):
        lo_ = np.array(lo, dtype=np.int32)
        hi_ = np.array(hi, dtype=np.int32)
        out = np.empty(2)
        lib().occ_loss_ke(self.h, level, _ptr(lo_), _ptr(hi_), _ptr(out))
        return complex(out[0], out[1])


def advance_particles(p, d):
    """p += d in float32 (in place), the same rounding as the GPU path."""
    assert p.dtype == np.float32 and p.flags.c_contiguous
    dd = np.asarray(d, dtype=np.float32)
    lib().oc_advance_particles(_ptr(p), p.shape[0], _ptr(dd))


def store_round(v, storage, scale):
    """The oracle's emulation of one 16-bit stored value ('bf16' or 'f16')."""
    return float(lib().oc_store_round(float(v), {"bf16": 1, "f16": 2}[storage], float(scale)))


def num_threads():
    """OpenMP threads the oracle runs with."""
    return int(lib().oc_num_threads())


def set_num_threads(n):
    """OpenMP threads of the oracle's parallel loops."""
    lib().oc_set_num_threads(int(n))


def lattice():
    c = np.empty((27, 3), dtype=np.int32)
    w = np.empty(27)
    lib().oc_lattice(_ptr(c), _ptr(w))
    return c, w


def reconstruct(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    f = np.empty(27)
    lib().oc_reconstruct(_ptr(q), _ptr(f))
    return f


def collide(q, omega, force=(0.0, 0.0, 0.0)):
    q = np.ascontiguousarray(q, dtype=np.float64)
    F = np.ascontiguousarray(force, dtype=np.float64)
    out = np.empty(10)
    lib().oc_collide(_ptr(q), float(omega), _ptr(F), _ptr(out))
    return out
