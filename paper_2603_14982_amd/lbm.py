"""Python binding of the C ABI in include/lbm.h (argument marshalling only).

Device memory comes from torch (the pool and table buffers, particles, solid
field, moment arrays); every step of the method runs in the HIP kernels of
liblbmx.so on torch's current stream. There is no CPU fallback: if the HIP
library is missing this module raises.
"""
import ctypes
import os

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbmx.so")

PERIODIC, INFLOW, OUTFLOW, WALL = 0, 1, 2, 3
F32, BF16, F16 = 0, 1, 2
STORAGE = {"f32": F32, "bf16": BF16, "f16": F16}
ROLE_COMPUTED, ROLE_GHOST, ROLE_IU, ROLE_SOLID, ROLE_INFLOW, ROLE_OUTFLOW = range(6)

_STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_ECAPACITY", -4: "LBM_EDEVICE",
           -5: "LBM_ENAN", -6: "LBM_ESTATE"}


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class LBMConfig(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32),
        ("fine_extent", ctypes.c_int32 * 3),
        ("bc", ctypes.c_int32 * 6),
        ("inflow_u", ctypes.c_float * 3),
        ("tau0", ctypes.c_double),
        ("storage", ctypes.c_int32),
        ("rescale", ctypes.c_int32),
        ("scale", ctypes.c_float * 10),
        ("max_blocks", ctypes.c_int64),
        ("pool", ctypes.c_void_p),
        ("meta", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("inflow_profile", ctypes.c_int32),
        ("inflow_axis", ctypes.c_int32),
        ("inflow_beta", ctypes.c_float),
        ("inflow_h0", ctypes.c_float),
        ("coupling", ctypes.c_int32),
        ("scalar", ctypes.c_int32),
    ]


EXPORTS = ["lbm_pool_bytes", "lbm_meta_bytes", "lbm_create", "lbm_destroy", "lbm_num_blocks", "lbm_block_keys",
           "lbm_set_block_moments", "lbm_step", "lbm_advance_particles", "lbm_remesh", "lbm_get_moments",
           "lbm_get_roles", "lbm_reduce_f64", "lbm_reduce_f64_noalloc", "lbm_step_finest", "lbm_finest_phase", "lbm_step_remesh", "lbm_record_work_bytes", "lbm_record_begin", "lbm_record_end", "lbm_check_finite", "lbm_set_profiling", "lbm_set_profiling_phases", "lbm_get_profile",
           "lbm_state_bytes", "lbm_save", "lbm_load", "lbm_adjoint_work_bytes", "lbm_adjoint_step", "lbm_adjoint_steps",
           "lbm_step_record", "lbm_adjoint_reverse",
           "lbm_loss_ke_grad", "lbm_set_option", "lbm_set_coupling",
           "lbm_scalar_set", "lbm_scalar_get", "lbm_scalar_advance", "lbm_last_error"]
_SIZE_QUERIES = ("lbm_pool_bytes", "lbm_meta_bytes", "lbm_state_bytes", "lbm_adjoint_work_bytes", "lbm_last_error")
PROFILE_PHASES = ["sc0", "sc1", "sc2", "sc3", "sc4", "down", "up", "outflow", "remesh", "sc_pair",
                  "adj_sc", "adj_sc_fused", "adj"]
OPTIONS = {"tile_min_blocks": 0, "fuse_substeps": 1, "graphs": 2, "pair_run": 3}

_lib = None


def lib():
    """Loads liblbmx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_14982_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        cfgp = ctypes.POINTER(LBMConfig)
        L.lbm_pool_bytes.restype = sz
        L.lbm_pool_bytes.argtypes = [cfgp]
        L.lbm_meta_bytes.restype = sz
        L.lbm_meta_bytes.argtypes = [cfgp]
        L.lbm_create.argtypes = [cfgp, vp, vp, i64, ctypes.POINTER(vp)]
        L.lbm_destroy.argtypes = [vp]
        L.lbm_num_blocks.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.lbm_block_keys.argtypes = [vp, i32, vp]
        L.lbm_set_block_moments.argtypes = [vp, i32, vp, vp, i64]
        L.lbm_step.argtypes = [vp, i32]
        L.lbm_step_finest.argtypes = [vp, i32]
        L.lbm_step_remesh.argtypes = [vp, i32, vp, i64, vp]
        L.lbm_record_work_bytes.restype = sz
        L.lbm_record_work_bytes.argtypes = [vp, i32, i32]
        L.lbm_record_begin.argtypes = [vp, vp, sz]
        L.lbm_record_end.argtypes = [vp]
        L.lbm_finest_phase.argtypes = [vp, ctypes.POINTER(i32)]
        L.lbm_advance_particles.argtypes = [vp, vp, i64, vp]
        L.lbm_remesh.argtypes = [vp, vp, i64]
        L.lbm_get_moments.argtypes = [vp, i32, vp, vp]
        L.lbm_get_roles.argtypes = [vp, i32, vp]
        L.lbm_reduce_f64.argtypes = [vp, i32, vp, vp, vp]
        L.lbm_reduce_f64_noalloc.argtypes = [vp, i32, vp, vp, vp]
        L.lbm_check_finite.argtypes = [vp]
        L.lbm_set_profiling.argtypes = [vp, i32]
        L.lbm_set_profiling_phases.argtypes = [vp, ctypes.c_uint32]
        L.lbm_get_profile.argtypes = [vp, vp, vp]
        L.lbm_state_bytes.restype = sz
        L.lbm_state_bytes.argtypes = [vp]
        L.lbm_save.argtypes = [vp, vp, sz]
        L.lbm_load.argtypes = [vp, vp, sz]
        L.lbm_adjoint_work_bytes.restype = sz
        L.lbm_adjoint_work_bytes.argtypes = [vp, i32]
        L.lbm_adjoint_step.argtypes = [vp, vp, sz, vp, vp, vp, sz]
        L.lbm_adjoint_steps.argtypes = [vp, vp, sz, i32, vp, vp, vp, sz]
        L.lbm_step_record.argtypes = [vp, i32, vp, sz]
        L.lbm_adjoint_reverse.argtypes = [vp, vp, vp, vp, sz]
        L.lbm_loss_ke_grad.argtypes = [vp, i32, vp, vp, vp]
        L.lbm_set_option.argtypes = [vp, i32, i64]
        L.lbm_set_coupling.argtypes = [vp, vp, vp, i64]
        L.lbm_scalar_set.argtypes = [vp, vp, vp, i64]
        L.lbm_scalar_get.argtypes = [vp, vp, vp]
        L.lbm_scalar_advance.argtypes = [vp, ctypes.c_float, ctypes.c_float, vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_last_error.argtypes = [vp]
        for name in EXPORTS:
            if name not in _SIZE_QUERIES:
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def make_config(levels, n, bc, tau0, uin=(0.0, 0.0, 0.0), storage="f32", scale=None, rescale="ce",
                max_blocks=1, log_inflow=None, coupling=False, scalar=False):
    """log_inflow = (axis, beta, h0): inflow velocity uin * ln(1 + beta (h - h0)) at
    height h (fine nodes) along axis, zero at or below h0; None: uniform uin."""
    c = LBMConfig()
    c.coupling = 1 if coupling else 0
    c.scalar = 1 if scalar else 0
    if log_inflow is not None:
        c.inflow_profile = 1
        c.inflow_axis = int(log_inflow[0])
        c.inflow_beta = float(log_inflow[1])
        c.inflow_h0 = float(log_inflow[2])
    c.levels = int(levels)
    for a in range(3):
        c.fine_extent[a] = int(n[a])
        c.inflow_u[a] = float(uin[a])
    for f in range(6):
        c.bc[f] = int(bc[f])
    c.tau0 = float(tau0)
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.rescale = {"ce": 0, "printed": 1}[rescale]
    sc = [1.0] * 10 if scale is None else list(scale)
    for m in range(10):
        c.scale[m] = float(sc[m])
    c.max_blocks = int(max_blocks)
    return c


def _dptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


class Sim:
    """One block-adaptive simulation on a GPU; buffers are torch tensors."""

    def __init__(self, levels, n, bc, tau0, uin=(0.0, 0.0, 0.0), storage="f32", scale=None, rescale="ce",
                 max_blocks=None, solid=None, particles=None, device="cuda", log_inflow=None, coupling=False,
                 scalar=False):
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.levels = int(levels)
        self.n = tuple(int(v) for v in n)
        if max_blocks is None:
            max_blocks = sum((n[0] >> l) // 8 * ((n[1] >> l) // 8) * ((n[2] >> l) // 8) for l in range(levels))
            max_blocks = min(max_blocks, 1 << 16)
        self.cfg = make_config(levels, n, bc, tau0, uin, storage, scale, rescale, max_blocks, log_inflow, coupling,
                               scalar)
        L = lib()
        pool_bytes = L.lbm_pool_bytes(ctypes.byref(self.cfg))
        meta_bytes = L.lbm_meta_bytes(ctypes.byref(self.cfg))
        if pool_bytes == 0 or meta_bytes == 0:
            raise LBMError(-1, "invalid configuration")
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=self.device)
        self.meta = torch.empty(meta_bytes, dtype=torch.uint8, device=self.device)
        self.cfg.pool = self.pool.data_ptr()
        self.cfg.meta = self.meta.data_ptr()
        self.cfg.stream = torch.cuda.current_stream(self.device).cuda_stream
        self.solid = None
        if solid is not None:
            self.solid = torch.as_tensor(np.ascontiguousarray(solid, dtype=np.uint8)).to(self.device).contiguous()
        p = self._particles(particles)
        h = ctypes.c_void_p()
        st = L.lbm_create(ctypes.byref(self.cfg), _dptr(self.solid), _dptr(p), 0 if p is None else p.shape[0],
                          ctypes.byref(h))
        if st != 0:
            raise LBMError(st, L.lbm_last_error(None).decode())
        self.h = h

    def _particles(self, particles):
        if particles is None:
            return None
        if isinstance(particles, torch.Tensor):
            assert particles.dtype == torch.float32 and particles.is_contiguous() and particles.device == self.device
            return particles
        return torch.as_tensor(np.ascontiguousarray(particles, dtype=np.float32)).to(self.device)

    def _check(self, st):
        if st != 0:
            raise LBMError(st, lib().lbm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_blocks(self, level):
        out = ctypes.c_int64()
        self._check(lib().lbm_num_blocks(self.h, level, ctypes.byref(out)))
        return int(out.value)

    def block_keys(self, level):
        k = torch.empty(self.num_blocks(level), dtype=torch.int64, device=self.device)
        if k.numel():
            self._check(lib().lbm_block_keys(self.h, level, _dptr(k)))
        return k

    def set_block_moments(self, level, keys, vals):
        keys = torch.as_tensor(np.asarray(keys) if not isinstance(keys, torch.Tensor) else keys,
                               dtype=torch.int64).to(self.device).contiguous()
        vals = torch.as_tensor(vals if isinstance(vals, torch.Tensor) else np.asarray(vals),
                               dtype=torch.float32).to(self.device).contiguous()
        assert vals.shape == (keys.shape[0], 10, 512)
        self._check(lib().lbm_set_block_moments(self.h, level, _dptr(keys), _dptr(vals), keys.shape[0]))

    def step(self, n=1):
        self._check(lib().lbm_step(self.h, int(n)))

    def step_finest(self, n=1):
        """n finest-level steps (Alg. 1 stopped after each finest stream-collide)."""
        self._check(lib().lbm_step_finest(self.h, int(n)))

    def finest_phase(self):
        """Finest steps taken since the last coarse-step boundary."""
        v = ctypes.c_int32()
        self._check(lib().lbm_finest_phase(self.h, ctypes.byref(v)))
        return v.value

    def step_remesh(self, n, particles, d):
        """n times: step(1), advance_particles(particles, d), remesh(particles), the particle
        work overlapped with the step on a second stream."""
        dd = (ctypes.c_float * 3)(*[float(v) for v in d])
        self._check(lib().lbm_step_remesh(self.h, int(n), _dptr(particles), particles.shape[0], dd))

    def advance_particles(self, particles, d):
        dd = (ctypes.c_float * 3)(*[float(v) for v in d])
        self._check(lib().lbm_advance_particles(self.h, _dptr(particles), particles.shape[0], dd))

    def remesh(self, particles):
        p = self._particles(particles)
        self._check(lib().lbm_remesh(self.h, _dptr(p), 0 if p is None else p.shape[0]))

    def get_moments(self, level):
        nb = self.num_blocks(level)
        k = torch.empty(nb, dtype=torch.int64, device=self.device)
        v = torch.empty((nb, 10, 512), dtype=torch.float32, device=self.device)
        if nb:
            self._check(lib().lbm_get_moments(self.h, level, _dptr(k), _dptr(v)))
        return k, v

    def roles(self, level):
        nb = self.num_blocks(level)
        r = torch.empty((nb, 512), dtype=torch.uint8, device=self.device)
        if nb:
            self._check(lib().lbm_get_roles(self.h, level, _dptr(r)))
        return r

    def reduce(self, level, lo=(0, 0, 0), hi=None):
        hi = self.n if hi is None else hi
        lo_ = (ctypes.c_int32 * 3)(*lo)
        hi_ = (ctypes.c_int32 * 3)(*hi)
        out = (ctypes.c_double * 5)()
        self._check(lib().lbm_reduce_f64(self.h, level, lo_, hi_, out))
        return np.array(list(out))

    def reduce_noalloc(self, level, out, lo=(0, 0, 0), hi=None):
        """The sums of reduce() into out (device float64 tensor of 5), asynchronously,
        with the partials in the library's static device array."""
        hi = self.n if hi is None else hi
        assert out.dtype == torch.float64 and out.is_cuda and out.numel() >= 5 and out.is_contiguous()
        lo_ = (ctypes.c_int32 * 3)(*lo)
        hi_ = (ctypes.c_int32 * 3)(*hi)
        self._check(lib().lbm_reduce_f64_noalloc(self.h, level, lo_, hi_, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_coupling(self, keys, fields):
        """Finest-level coupling fields (needs coupling=True): keys of level-0 blocks and
        fields [nb, 4, 512] = (eps, Fx, Fy, Fz) per node (fluid fraction, force density)."""
        k = torch.as_tensor(np.asarray(keys, dtype=np.int64) if not torch.is_tensor(keys) else keys,
                            dtype=torch.int64, device=self.device).contiguous()
        f = torch.as_tensor(fields, dtype=torch.float32, device=self.device).contiguous()
        if tuple(f.shape) != (k.numel(), 4, 512):
            raise ValueError("fields must be [nb, 4, 512]")
        self._check(lib().lbm_set_coupling(self.h, _dptr(k), _dptr(f), k.numel()))

    def scalar_set(self, keys, phi):
        """Powder-snow volume fraction of finest-level blocks (needs scalar=True): phi [nb, 512]."""
        k = torch.as_tensor(np.asarray(keys, dtype=np.int64) if not torch.is_tensor(keys) else keys,
                            dtype=torch.int64, device=self.device).contiguous()
        f = torch.as_tensor(phi, dtype=torch.float32, device=self.device).contiguous()
        if tuple(f.shape) != (k.numel(), 512):
            raise ValueError("phi must be [nb, 512]")
        self._check(lib().lbm_scalar_set(self.h, _dptr(k), _dptr(f), k.numel()))

    def scalar_get(self):
        """(keys [nb], phi [nb, 512]) of every finest-level block, key order."""
        nb = self.num_blocks(0)
        keys = torch.empty(nb, dtype=torch.int64, device=self.device)
        phi = torch.empty((nb, 512), dtype=torch.float32, device=self.device)
        self._check(lib().lbm_scalar_get(self.h, _dptr(keys), _dptr(phi)))
        return keys, phi

    def scalar_advance(self, dt, D, source=None):
        src = None if source is None else torch.as_tensor(source, dtype=torch.float32, device=self.device).contiguous()
        self._check(lib().lbm_scalar_advance(self.h, float(dt), float(D), _dptr(src)))

    def set_option(self, name, value):
        """Execution options: "tile_min_blocks" (blocks a level needs for the tiled
        stream-collide, default 16384) and "fuse_substeps" (2: the finest level's two
        substeps per parent step in one sweep where allowed (default), 1: the same
        with FP32 storage only, 0: always two sweeps) and "graphs" (1: coarse steps
        replayed as HIP graphs outside profiling and recording, 0: every kernel
        launched by itself (default))."""
        self._check(lib().lbm_set_option(self.h, OPTIONS[name], int(value)))

    def set_profiling(self, on=True, phases=None):
        """Phase timers on or off; with `phases` (names from PROFILE_PHASES) only those
        phases are timed (each timed launch costs two event records on the stream)."""
        if phases is None:
            self._check(lib().lbm_set_profiling(self.h, 1 if on else 0))
        else:
            mask = 0
            for name in phases:
                mask |= 1 << PROFILE_PHASES.index(name)
            self._check(lib().lbm_set_profiling_phases(self.h, mask if on else 0))

    def profile(self):
        """Summed ms and launch counts per phase since the last call (synchronises)."""
        ms = (ctypes.c_double * len(PROFILE_PHASES))()
        cnt = (ctypes.c_int64 * len(PROFILE_PHASES))()
        self._check(lib().lbm_get_profile(self.h, ms, cnt))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROFILE_PHASES)}

    def check_finite(self):
        st = lib().lbm_check_finite(self.h)
        if st == -5:
            return False
        self._check(st)
        return True

    # ---- states and the adjoint ----
    def total_blocks(self):
        return sum(self.num_blocks(l) for l in range(self.levels))

    def state_bytes(self):
        return int(lib().lbm_state_bytes(self.h))

    def save(self, out=None):
        """The current state (all levels' current time level) as a device uint8 tensor."""
        n = self.state_bytes()
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=self.device)
        self._check(lib().lbm_save(self.h, _dptr(out), out.numel()))
        return out

    def load(self, state):
        self._check(lib().lbm_load(self.h, _dptr(state), state.numel()))

    def get_all_moments(self):
        """Moments of every level, concatenated in level order: [sum nb, 10, 512]."""
        return torch.cat([self.get_moments(l)[1] for l in range(self.levels)])

    def set_all_moments(self, x):
        off = 0
        for l in range(self.levels):
            keys = self.block_keys(l)
            n = keys.shape[0]
            if n:
                self.set_block_moments(l, keys, x[off:off + n])
            off += n
        assert off == x.shape[0]

    def adjoint_work(self, n_steps=1):
        n = int(lib().lbm_adjoint_work_bytes(self.h, int(n_steps)))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def adjoint_step(self, state, lam_next, lam_out=None, work=None, n_steps=1):
        """dLoss/d(state) from dLoss/d(state n_steps coarse steps later); leaves the
        simulation at `state`."""
        if lam_out is None:
            lam_out = torch.empty_like(lam_next)
        if work is None:
            work = self.adjoint_work(n_steps)
        assert lam_next.dtype == torch.float32 and lam_next.is_contiguous()
        assert lam_next.shape == (self.total_blocks(), 10, 512) and lam_out.shape == lam_next.shape
        self._check(lib().lbm_adjoint_steps(self.h, _dptr(state), state.numel(), int(n_steps), _dptr(lam_next),
                                            _dptr(lam_out), _dptr(work), work.numel()))
        return lam_out

    def step_record(self, n_steps, work):
        """`n_steps` coarse steps that keep their undo log in `work` (adjoint_work(n_steps))."""
        self._rec_blocks = self.total_blocks()
        self._check(lib().lbm_step_record(self.h, int(n_steps), _dptr(work), work.numel()))

    def record_work(self, n_steps, n_updates):
        """A work buffer for a recording of n_steps coarse steps and n_updates grid updates."""
        nbytes = int(lib().lbm_record_work_bytes(self.h, int(n_steps), int(n_updates)))
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def record_begin(self, work):
        """Opens a recording (steps and grid updates) for adjoint_reverse."""
        self._rec_blocks = self.total_blocks()
        self._check(lib().lbm_record_begin(self.h, _dptr(work), work.numel()))

    def record_end(self):
        self._check(lib().lbm_record_end(self.h))

    def adjoint_reverse(self, lam_next, lam_out=None, work=None):
        """Adjoint through the recorded steps (and grid updates); returns the simulation
        to the state (and hierarchy) before them. lam_out has the block count of that
        hierarchy."""
        nb0 = getattr(self, "_rec_blocks", None) or self.total_blocks()
        if lam_out is None:
            lam_out = torch.empty((nb0, 10, 512), dtype=torch.float32, device=self.device)
        assert lam_next.dtype == torch.float32 and lam_next.is_contiguous()
        assert lam_next.shape == (self.total_blocks(), 10, 512) and lam_out.shape[1:] == (10, 512)
        self._check(lib().lbm_adjoint_reverse(self.h, _dptr(lam_next), _dptr(lam_out), _dptr(work), work.numel()))
        return lam_out

    def loss_ke_grad(self, level, lo, hi):
        """d(1/2 sum rho |u|^2 over the level's owned nodes in [lo, hi))/d(moments), all-level layout."""
        lam = torch.empty((self.total_blocks(), 10, 512), dtype=torch.float32, device=self.device)
        lo_ = (ctypes.c_int32 * 3)(*lo)
        hi_ = (ctypes.c_int32 * 3)(*hi)
        self._check(lib().lbm_loss_ke_grad(self.h, level, lo_, hi_, _dptr(lam)))
        return lam


class _RolloutTaped(torch.autograd.Function):
    """x0 -> moments after `steps` coarse steps, keeping the whole undo log of the
    forward pass on the device; the backward pass is one reverse sweep."""

    @staticmethod
    def forward(ctx, x0, sim, steps):
        sim.set_all_moments(x0.detach())
        work = sim.adjoint_work(steps)
        sim.step_record(steps, work)
        out = sim.get_all_moments()
        ctx.sim, ctx.work = sim, work
        ctx.final = sim.save()
        return out

    @staticmethod
    def backward(ctx, grad):
        sim = ctx.sim
        lam = grad.detach().to(torch.float32).contiguous().clone()
        sim.adjoint_reverse(lam, lam, ctx.work)
        sim.load(ctx.final)
        ctx.work = None
        return lam, None, None


class _Rollout(torch.autograd.Function):
    """x0 (all-level moments) -> moments after `steps` coarse steps. Checkpoints
    every `every` steps; the backward pass hands each segment, last first, to the
    library's multi-step adjoint (one replay with the undo log, one reverse sweep).
    The forward pass records the last segment's undo log itself (in the work buffer
    the backward pass needs anyway), so that segment is not replayed unless the
    simulation changed in between (the library then refuses the recording and the
    segment is replayed from its checkpoint)."""

    @staticmethod
    def forward(ctx, x0, sim, steps, every):
        sim.set_all_moments(x0.detach())
        ckpts = []
        last = (steps - 1) // every * every
        work = sim.adjoint_work(min(every, steps))
        for k in range(0, last, every):
            ckpts.append((k, sim.save()))
            sim.step(min(every, last - k))
        ckpts.append((last, sim.save()))
        sim.step_record(steps - last, work)
        out = sim.get_all_moments()
        ctx.sim, ctx.steps, ctx.every, ctx.ckpts, ctx.work = sim, steps, every, ckpts, work
        ctx.final = sim.save()
        return out

    @staticmethod
    def backward(ctx, grad):
        sim = ctx.sim
        lam = grad.detach().to(torch.float32).contiguous().clone()
        work = ctx.work
        ckpts = list(ctx.ckpts)
        k0, ck = ckpts.pop()
        try:
            sim.adjoint_reverse(lam, lam, work)
        except LBMError as e:
            if e.status != -6:  # LBM_ESTATE: the recording no longer matches the simulation
                raise
            sim.adjoint_step(ck, lam, lam, work, n_steps=ctx.steps - k0)
        for k0, ck in reversed(ckpts):
            k1 = min(k0 + ctx.every, ctx.steps)
            sim.adjoint_step(ck, lam, lam, work, n_steps=k1 - k0)
        sim.load(ctx.final)
        ctx.work = None
        return lam, None, None, None


def rollout(sim, x0, steps, checkpoint_every=20):
    """Differentiable `steps` coarse steps from the all-level moments x0 ([sum nb, 10, 512],
    device f32); returns the all-level moments after them. The hierarchy stays fixed.
    checkpoint_every > 0: states are kept every that many steps and each segment is
    replayed in the backward pass; 0: the forward pass keeps its whole undo log
    (lbm_adjoint_work_bytes(steps) of device memory) and nothing is replayed."""
    if int(checkpoint_every) == 0:
        return _RolloutTaped.apply(x0, sim, int(steps))
    return _Rollout.apply(x0, sim, int(steps), int(checkpoint_every))
