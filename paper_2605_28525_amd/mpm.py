"""ctypes binding of ``libmpm.so`` (the C ABI declared in include/mpm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Particle arrays are torch CUDA tensors (device memory); their ``data_ptr()``
and the raw HIP stream handle are passed straight through.  If the library is
not built, importing this module raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int, c_uint32, c_uint64, c_void_p

import numpy as np
# torch is imported before the library is loaded: it ships its own HIP runtime
# under the same soname as the system one, the first one loaded serves the
# whole process, and torch's device memory and streams need torch's own.
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmpm.so")

MPM_OK, MPM_ERR_ARG, MPM_ERR_HIP, MPM_ERR_NOMEM = 0, 1, 2, 3
MPM_ERR_OVERFLOW, MPM_ERR_DOMAIN, MPM_ERR_INVERTED, MPM_ERR_NAN, MPM_ERR_STATE = 4, 5, 6, 7, 8
MPM_FLAG_OVERFLOW, MPM_FLAG_DOMAIN, MPM_FLAG_INVERTED, MPM_FLAG_NAN = 1, 2, 4, 8
MPM_BC = {"none": 0, "sticky": 1, "slip": 2, "separate": 3}
MPM_MODEL = {"elastic": 0, "dp": 1}
MPM_GRID_SPARSE, MPM_GRID_DENSE = 0, 1
MPM_FLAG_SYNC_REBUILD = 1
MPM_FLAG_ADJOINT = 2
MPM_FLAG_FULL_SORT = 4
MPM_FLAG_DETERMINISTIC_ORDER = 8
MPM_FLAG_SCAN_BUILD = 16


class mpm_instance(ctypes.Structure):
    _fields_ = [
        ("E", c_float),
        ("nu", c_float),
        ("friction_deg", c_float),
        ("dt", c_float),
        ("p_mass", c_float),
        ("p_vol0", c_float),
    ]


class mpm_params(ctypes.Structure):
    _fields_ = [
        ("dim", c_int),
        ("dx", c_double),
        ("cells", c_int * 3),
        ("gravity", c_float * 3),
        ("dt", c_float),
        ("bound", c_int),
        ("bc", (c_int * 2) * 3),
        ("heightmap", POINTER(c_float)),
        ("mu_terrain", c_float),
        ("model", c_int),
        ("E", c_float),
        ("nu", c_float),
        ("friction_deg", c_float),
        ("p_mass", c_float),
        ("p_vol0", c_float),
        ("max_particles", c_int),
        ("block_capacity", c_int),
        ("hash_capacity_log2", c_int),
        ("grid_mode", c_int),
        ("flags", c_int),
        ("n_instances", c_int),
        ("instances", POINTER(mpm_instance)),
    ]


class mpm_particles(ctypes.Structure):
    _fields_ = [
        ("n", c_int),
        ("x", c_void_p),
        ("v", c_void_p),
        ("C", c_void_p),
        ("F", c_void_p),
        ("tau", c_void_p),
        ("id", c_void_p),
        ("inst", c_void_p),
    ]


_PCTX = c_void_p
_SIGS = {
    "mpm_create": (c_int, [POINTER(mpm_params), POINTER(_PCTX)]),
    "mpm_destroy": (c_int, [_PCTX]),
    "mpm_status_string": (ctypes.c_char_p, [c_int]),
    "mpm_sparse_build": (c_int, [_PCTX, POINTER(mpm_particles), c_void_p]),
    "mpm_p2g": (c_int, [_PCTX, POINTER(mpm_particles), c_void_p]),
    "mpm_grid_update": (c_int, [_PCTX, c_void_p]),
    "mpm_g2p": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), c_void_p]),
    "mpm_step": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), c_int, c_void_p]),
    "mpm_get_status": (c_int, [_PCTX, c_void_p, POINTER(c_uint32)]),
    "mpm_clear_status": (c_int, [_PCTX, c_void_p]),
    "mpm_active_count": (c_int, [_PCTX, c_void_p, POINTER(c_int), POINTER(c_int)]),
    "mpm_get_active": (c_int, [_PCTX, c_void_p, c_void_p, c_int, c_void_p]),
    "mpm_scan_active": (c_int, [_PCTX, POINTER(mpm_particles), c_void_p, c_void_p, c_int, POINTER(c_int), c_void_p]),
    "mpm_scan_active_static": (c_int, [_PCTX, POINTER(mpm_particles), c_void_p, c_void_p, c_int, POINTER(c_int),
                                       c_void_p]),
    "mpm_get_grid": (c_int, [_PCTX, c_void_p, c_int, c_void_p]),
    "mpm_get_order": (c_int, [_PCTX, c_void_p, c_int, c_void_p]),
    "mpm_set_material": (c_int, [_PCTX, c_float, c_float, c_float, c_float]),
    "mpm_g2p_adj": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), POINTER(mpm_particles),
                            c_void_p, c_void_p]),
    "mpm_grid_update_adj": (c_int, [_PCTX, c_void_p]),
    "mpm_p2g_adj": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), c_void_p]),
    "mpm_step_adj": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), POINTER(mpm_particles),
                             c_void_p, c_void_p]),
    "mpm_tape_reserve": (c_int, [_PCTX, c_int]),
    "mpm_tape_forward": (c_int, [_PCTX, POINTER(mpm_particles), c_int, c_void_p]),
    "mpm_tape_adjoint": (c_int, [_PCTX, POINTER(mpm_particles), c_int, POINTER(mpm_particles),
                                 POINTER(mpm_particles), c_void_p, c_void_p]),
    "mpm_graph_capture": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), c_int, c_void_p]),
    "mpm_graph_launch": (c_int, [_PCTX, c_int, c_void_p]),
    "mpm_graph_release": (c_int, [_PCTX]),
    "mpm_set_tuning": (c_int, [_PCTX, c_int, c_int, c_int, c_int]),
    "mpm_autotune": (c_int, [_PCTX, POINTER(mpm_particles), POINTER(mpm_particles), POINTER(c_int), c_void_p]),
}


def _load():
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built; run `python -m paper_2605_28525_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class MPMError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {lib.mpm_status_string(code).decode()}")


def _check(rc: int, where: str):
    if rc != MPM_OK:
        raise MPMError(rc, where)


def _stream(stream):
    if stream is None:
        import torch
        return c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# same names as the C ABI
def mpm_create(params: mpm_params) -> c_void_p:
    ctx = _PCTX()
    _check(lib.mpm_create(ctypes.byref(params), ctypes.byref(ctx)), "mpm_create")
    return ctx


def mpm_destroy(ctx):
    _check(lib.mpm_destroy(ctx), "mpm_destroy")


def mpm_sparse_build(ctx, p: mpm_particles, stream=None):
    _check(lib.mpm_sparse_build(ctx, ctypes.byref(p), _stream(stream)), "mpm_sparse_build")


def mpm_p2g(ctx, p: mpm_particles, stream=None):
    _check(lib.mpm_p2g(ctx, ctypes.byref(p), _stream(stream)), "mpm_p2g")


def mpm_grid_update(ctx, stream=None):
    _check(lib.mpm_grid_update(ctx, _stream(stream)), "mpm_grid_update")


def mpm_g2p(ctx, pin: mpm_particles, pout: mpm_particles, stream=None):
    _check(lib.mpm_g2p(ctx, ctypes.byref(pin), ctypes.byref(pout), _stream(stream)), "mpm_g2p")


def mpm_step(ctx, a: mpm_particles, b: mpm_particles, n_steps: int, stream=None):
    _check(lib.mpm_step(ctx, ctypes.byref(a), ctypes.byref(b), int(n_steps), _stream(stream)), "mpm_step")


def mpm_get_status(ctx, stream=None):
    """Returns (return code, flags); synchronises the stream."""
    f = c_uint32(0)
    rc = lib.mpm_get_status(ctx, _stream(stream), ctypes.byref(f))
    if rc in (MPM_ERR_ARG, MPM_ERR_HIP):
        raise MPMError(rc, "mpm_get_status")
    return rc, int(f.value)


def mpm_clear_status(ctx, stream=None):
    _check(lib.mpm_clear_status(ctx, _stream(stream)), "mpm_clear_status")


def mpm_active_count(ctx, stream=None):
    nb, nt = c_int(0), c_int(0)
    _check(lib.mpm_active_count(ctx, _stream(stream), ctypes.byref(nb), ctypes.byref(nt)), "mpm_active_count")
    return int(nb.value), int(nt.value)


def mpm_get_active(ctx, keys, masks, capacity: int, stream=None):
    _check(lib.mpm_get_active(ctx, c_void_p(keys.data_ptr()), c_void_p(masks.data_ptr()), int(capacity),
                              _stream(stream)), "mpm_get_active")


def mpm_scan_active(ctx, particles, keys, masks, capacity: int, stream=None) -> int:
    """Scan-based active set of `particles` (keys and masks written to the first
    min(count, capacity) entries of the device tensors); returns the count."""
    nb = c_int(0)
    _check(lib.mpm_scan_active(ctx, ctypes.byref(particles), c_void_p(keys.data_ptr() if capacity else 0),
                               c_void_p(masks.data_ptr() if capacity else 0), int(capacity), ctypes.byref(nb),
                               _stream(stream)), "mpm_scan_active")
    return nb.value


def mpm_scan_active_static(ctx, particles, keys, masks, capacity: int, stream=None) -> int:
    """mpm_scan_active with the library's static scratch (allocates nothing);
    returns the count."""
    nb = c_int(0)
    _check(lib.mpm_scan_active_static(ctx, ctypes.byref(particles), c_void_p(keys.data_ptr() if capacity else 0),
                                      c_void_p(masks.data_ptr() if capacity else 0), int(capacity),
                                      ctypes.byref(nb), _stream(stream)), "mpm_scan_active_static")
    return nb.value


def mpm_get_grid(ctx, out, capacity_blocks: int, stream=None):
    _check(lib.mpm_get_grid(ctx, c_void_p(out.data_ptr()), int(capacity_blocks), _stream(stream)), "mpm_get_grid")


def mpm_get_order(ctx, order, n: int, stream=None):
    _check(lib.mpm_get_order(ctx, c_void_p(order.data_ptr()), int(n), _stream(stream)), "mpm_get_order")


def mpm_set_material(ctx, E: float, nu: float, friction_deg: float, dt: float):
    _check(lib.mpm_set_material(ctx, E, nu, friction_deg, dt), "mpm_set_material")


def mpm_g2p_adj(ctx, pin: mpm_particles, out_bar: mpm_particles, in_bar: mpm_particles, param_bar, stream=None):
    _check(lib.mpm_g2p_adj(ctx, ctypes.byref(pin), ctypes.byref(out_bar), ctypes.byref(in_bar),
                           c_void_p(param_bar.data_ptr()), _stream(stream)), "mpm_g2p_adj")


def mpm_grid_update_adj(ctx, stream=None):
    _check(lib.mpm_grid_update_adj(ctx, _stream(stream)), "mpm_grid_update_adj")


def mpm_p2g_adj(ctx, pin: mpm_particles, in_bar: mpm_particles, stream=None):
    _check(lib.mpm_p2g_adj(ctx, ctypes.byref(pin), ctypes.byref(in_bar), _stream(stream)), "mpm_p2g_adj")


def mpm_step_adj(ctx, pin: mpm_particles, out_bar: mpm_particles, in_bar: mpm_particles, param_bar, stream=None):
    _check(lib.mpm_step_adj(ctx, ctypes.byref(pin), ctypes.byref(out_bar), ctypes.byref(in_bar),
                            c_void_p(param_bar.data_ptr()), _stream(stream)), "mpm_step_adj")


def mpm_tape_reserve(ctx, n_slots: int):
    _check(lib.mpm_tape_reserve(ctx, int(n_slots)), "mpm_tape_reserve")


def _particle_array(states):
    arr = (mpm_particles * len(states))()
    for i, st in enumerate(states):
        arr[i] = st
    return arr


def mpm_tape_forward(ctx, states, stream=None):
    """states: list of n_steps + 1 mpm_particles views; runs len(states) - 1 steps."""
    arr = _particle_array(states)
    _check(lib.mpm_tape_forward(ctx, arr, len(states) - 1, _stream(stream)), "mpm_tape_forward")


def mpm_tape_adjoint(ctx, states, bar: mpm_particles, spare: mpm_particles, param_bar, stream=None):
    arr = _particle_array(states)
    _check(lib.mpm_tape_adjoint(ctx, arr, len(states) - 1, ctypes.byref(bar), ctypes.byref(spare),
                                c_void_p(param_bar.data_ptr()), _stream(stream)), "mpm_tape_adjoint")


def mpm_graph_capture(ctx, a: mpm_particles, b: mpm_particles, n_steps: int, stream=None):
    _check(lib.mpm_graph_capture(ctx, ctypes.byref(a), ctypes.byref(b), int(n_steps), _stream(stream)),
           "mpm_graph_capture")


def mpm_graph_launch(ctx, times: int = 1, stream=None):
    _check(lib.mpm_graph_launch(ctx, int(times), _stream(stream)), "mpm_graph_launch")


def mpm_graph_release(ctx):
    _check(lib.mpm_graph_release(ctx), "mpm_graph_release")


def mpm_set_tuning(ctx, chunk: int = 0, g2p_block: int = 0, p2g_workgroups: int = 0, g2p_workgroups: int = 0):
    _check(lib.mpm_set_tuning(ctx, int(chunk), int(g2p_block), int(p2g_workgroups), int(g2p_workgroups)),
           "mpm_set_tuning")


def mpm_autotune(ctx, a: mpm_particles, b: mpm_particles, stream=None):
    """Returns the chosen (chunk, g2p_block, p2g_workgroups, g2p_workgroups)."""
    out = (c_int * 4)()
    _check(lib.mpm_autotune(ctx, ctypes.byref(a), ctypes.byref(b), out, _stream(stream)), "mpm_autotune")
    return tuple(int(v) for v in out)


# ---------------------------------------------------------------------------
# marshalling helpers
def params_from_workload(w, *, max_particles=None, grid_mode=MPM_GRID_SPARSE, block_capacity=0,
                         hash_capacity_log2=0, flags=0):
    """Build an ``mpm_params`` from a workload description.  The returned object
    keeps the heightmap array alive until mpm_create has copied it."""
    p = mpm_params()
    p.dim = w.dim
    p.dx = float(w.dx)
    for a in range(3):
        p.cells[a] = int(w.cells[a]) if a < w.dim else 0
        p.gravity[a] = float(w.gravity[a])
        for s in range(2):
            p.bc[a][s] = MPM_BC[w.bc[a][s]] if a < w.dim else 0
    p.dt = float(w.dt)
    p.bound = int(w.bound)
    if w.heightmap is not None:
        hm = np.ascontiguousarray(w.heightmap, dtype=np.float32)
        p._hm_keepalive = hm
        p.heightmap = hm.ctypes.data_as(POINTER(c_float))
    p.mu_terrain = float(w.mu_terrain)
    p.model = MPM_MODEL[w.model]
    p.E, p.nu, p.friction_deg = float(w.E), float(w.nu), float(w.friction_deg)
    p.p_mass, p.p_vol0 = float(w.p_mass), float(w.p_vol0)
    p.max_particles = int(max_particles or w.n)
    p.block_capacity = int(block_capacity)
    p.hash_capacity_log2 = int(hash_capacity_log2)
    p.grid_mode = int(grid_mode)
    p.flags = int(flags)
    p.n_instances = 0
    return p


def params_from_ensemble(ens, *, max_particles=None, block_capacity=0, hash_capacity_log2=0, flags=0):
    """``mpm_params`` of an ensemble: the shared grid, walls and model from its
    first member, one ``mpm_instance`` per member.  The returned object keeps
    the instance table alive until mpm_create has copied it."""
    m0 = ens.members[0]
    p = params_from_workload(m0, max_particles=max_particles or ens.n, block_capacity=block_capacity,
                             hash_capacity_log2=hash_capacity_log2, flags=flags)
    table = (mpm_instance * len(ens.members))()
    for i, m in enumerate(ens.members):
        table[i] = mpm_instance(float(m.E), float(m.nu), float(m.friction_deg), float(m.dt), float(m.p_mass),
                                float(m.p_vol0))
    p._inst_keepalive = table
    p.n_instances = len(ens.members)
    p.instances = ctypes.cast(table, POINTER(mpm_instance))
    return p


class ParticleSet:
    """Device SoA particle state as torch tensors plus its ``mpm_particles`` view."""

    def __init__(self, dim: int, n: int, device="cuda", with_inst: bool = False, zero: bool = True):
        import torch
        d = dim
        make = torch.zeros if zero else torch.empty
        self.dim, self.n = dim, n
        self.inst = make((n,), dtype=torch.int32, device=device) if with_inst else None
        self.x = make((d, n), dtype=torch.float32, device=device)
        self.v = make((d, n), dtype=torch.float32, device=device)
        self.C = make((d * d, n), dtype=torch.float32, device=device)
        self.F = make((d * d, n), dtype=torch.float32, device=device)
        self.tau = make((3 if d == 2 else 6, n), dtype=torch.float32, device=device)
        self.id = make((n,), dtype=torch.int32, device=device)

    @classmethod
    def from_arrays(cls, st: dict, ids=None, device="cuda", inst=None):
        import torch
        d, n = st["x"].shape
        ps = cls(d, n, device, with_inst=inst is not None)
        for k in ("x", "v", "C", "F", "tau"):
            getattr(ps, k).copy_(torch.from_numpy(np.ascontiguousarray(st[k], dtype=np.float32)))
        ids = np.arange(n, dtype=np.int32) if ids is None else np.asarray(ids, dtype=np.int32)
        ps.id.copy_(torch.from_numpy(ids))
        if inst is not None:
            ps.inst.copy_(torch.from_numpy(np.asarray(inst).astype(np.int32)))
        return ps

    def copy_(self, other: "ParticleSet"):
        for k in ("x", "v", "C", "F", "tau", "id", "inst"):
            if getattr(self, k) is not None:
                getattr(self, k).copy_(getattr(other, k))
        return self

    def insts(self) -> np.ndarray:
        return self.inst.detach().cpu().numpy().view(np.uint32)

    def zero_(self):
        for k in ("x", "v", "C", "F", "tau"):
            getattr(self, k).zero_()
        return self

    def to_arrays(self) -> dict:
        return {k: getattr(self, k).detach().cpu().numpy() for k in ("x", "v", "C", "F", "tau")}

    def ids(self) -> np.ndarray:
        return self.id.detach().cpu().numpy().view(np.uint32)

    def view(self, with_id: bool = True) -> mpm_particles:
        """The ``mpm_particles`` of this set; without the id array the library
        carries no identities (the order from mpm_get_order still holds)."""
        p = mpm_particles()
        p.n = self.n
        p.x, p.v, p.C = self.x.data_ptr(), self.v.data_ptr(), self.C.data_ptr()
        p.F, p.tau = self.F.data_ptr(), self.tau.data_ptr()
        p.id = self.id.data_ptr() if with_id else None
        p.inst = self.inst.data_ptr() if self.inst is not None else None
        return p


class Simulation:
    """A context plus two particle buffers it ping-pongs between."""

    def __init__(self, w, *, grid_mode=MPM_GRID_SPARSE, block_capacity=0, hash_capacity_log2=0, flags=0,
                 device="cuda"):
        self.w = w
        inst = getattr(w, "inst", None)
        if inst is not None:   # an ensemble
            self.params = params_from_ensemble(w, block_capacity=block_capacity,
                                               hash_capacity_log2=hash_capacity_log2, flags=flags)
            dim = w.members[0].dim
        else:
            self.params = params_from_workload(w, grid_mode=grid_mode, block_capacity=block_capacity,
                                               hash_capacity_log2=hash_capacity_log2, flags=flags)
            dim = w.dim
        self.ctx = mpm_create(self.params)
        self.carry_id = True   # pass the id arrays to the library (particles keep their identity)
        self.a = ParticleSet.from_arrays(w.state(), device=device, inst=inst)
        self.b = ParticleSet(dim, w.n, device, with_inst=inst is not None)

    def set_state(self, st: dict, ids=None):
        import torch
        for k in ("x", "v", "C", "F", "tau"):
            getattr(self.a, k).copy_(torch.from_numpy(np.ascontiguousarray(st[k], dtype=np.float32)))
        ids = np.arange(self.a.n, dtype=np.int32) if ids is None else np.asarray(ids, dtype=np.int32)
        self.a.id.copy_(torch.from_numpy(ids))

    def step(self, n_steps: int = 1, stream=None):
        mpm_step(self.ctx, self.a.view(self.carry_id), self.b.view(self.carry_id), n_steps, stream)
        if n_steps % 2 == 1:
            self.a, self.b = self.b, self.a

    def status(self):
        return mpm_get_status(self.ctx)

    def close(self):
        if self.ctx:
            mpm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
