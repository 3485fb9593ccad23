"""ctypes binding of ``libfpdlbm.so`` (the C ABI in ``include/fpdlbm.h``).

Argument marshalling only: every step of the method runs in the library's HIP kernels.
Functions keep the C names; :class:`Simulation` is a small convenience wrapper.  The
library is loaded from this package directory and a missing library is an error (there
is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FPD_LIBRARY may name another build of the same library (A/B timing of kernel variants)
LIB_PATH = os.environ.get("FPD_LIBRARY") or os.path.join(HERE, "libfpdlbm.so")

FPD_OK, FPD_EINVAL, FPD_ENOMEM, FPD_EUNSTABLE, FPD_EDEVICE, FPD_ESTATE = 0, -1, -2, -3, -4, -5
FPD_F64, FPD_F32, FPD_F16DEV, FPD_BF16DEV = 0, 1, 2, 3
FPD_INIT_REST, FPD_INIT_LINEAR_COUETTE = 0, 1
FPD_WALLS, FPD_PERIODIC = 0, 1
FPD_FLAG_CLAMP_PHI, FPD_FLAG_NO_GRAPH, FPD_FLAG_TIME_KERNELS, FPD_FLAG_NO_SPLIT = 0x1, 0x2, 0x4, 0x8
FPD_HEALTH_NAN, FPD_HEALTH_STRAIN, FPD_HEALTH_MACH, FPD_HEALTH_WALL, FPD_HEALTH_SUPPORT = (
    0x1, 0x2, 0x4, 0x8, 0x10)
FPD_MAX_BEADS = 256

STORAGE = {"f64": FPD_F64, "f32": FPD_F32, "f16dev": FPD_F16DEV, "bf16dev": FPD_BF16DEV}


class fpd_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("u_wall", ctypes.c_double), ("nu_f", ctypes.c_double),
        ("eta_ratio", ctypes.c_double), ("xi", ctypes.c_double),
        ("n_beads", ctypes.c_int32),
        ("radius", ctypes.c_double), ("l0", ctypes.c_double),
        ("k_s", ctypes.c_double), ("k_b", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_q_fixed", ctypes.c_double), ("cutoff", ctypes.c_double),
        ("storage", ctypes.c_int32), ("init_flow", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("boundary", ctypes.c_int32),
        ("f_ext", ctypes.c_double * 2), ("g_body", ctypes.c_double * 2),
        ("n_chains", ctypes.c_int32),
        ("ev_k", ctypes.c_double), ("ev_range", ctypes.c_double),
    ]


class fpd_launch(ctypes.Structure):
    _fields_ = [
        ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
        ("rows_per_thread", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
        ("graph_chunk", ctypes.c_int32),
    ]


_D = ctypes.POINTER(ctypes.c_double)
_SIM = ctypes.c_void_p

# (name, restype, argtypes) for every exported function of include/fpdlbm.h
SIGNATURES = [
    ("fpd_params_default", None, [ctypes.POINTER(fpd_params)]),
    ("fpd_params_from_physical", ctypes.c_int,
     [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
      ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
      ctypes.POINTER(fpd_params)]),
    ("fpd_population_bytes", ctypes.c_size_t, [ctypes.POINTER(fpd_params)]),
    ("fpd_create", ctypes.c_int,
     [ctypes.POINTER(fpd_params), ctypes.c_void_p, ctypes.POINTER(_SIM)]),
    ("fpd_create_with_buffers", ctypes.c_int,
     [ctypes.POINTER(fpd_params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_size_t, ctypes.POINTER(_SIM)]),
    ("fpd_init_fiber", ctypes.c_int, [_SIM, _D]),
    ("fpd_init_fiber_line", ctypes.c_int, [_SIM, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    ("fpd_step", ctypes.c_int, [_SIM, ctypes.c_int64]),
    ("fpd_capture", ctypes.c_int, [_SIM, ctypes.c_int64]),
    ("fpd_sync", ctypes.c_int, [_SIM]),
    ("fpd_health", ctypes.c_int, [_SIM, ctypes.POINTER(ctypes.c_uint32), _D]),
    ("fpd_clear_health", ctypes.c_int, [_SIM]),
    ("fpd_step_count", ctypes.c_int, [_SIM, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_destroy", None, [_SIM]),
    ("fpd_last_error", ctypes.c_char_p, []),
    ("fpd_read_fields", ctypes.c_int, [_SIM, _D, _D, _D, _D]),
    ("fpd_read_populations", ctypes.c_int, [_SIM, _D]),
    ("fpd_write_populations", ctypes.c_int, [_SIM, _D]),
    ("fpd_read_beads", ctypes.c_int, [_SIM, _D, _D, _D]),
    ("fpd_particle_stats", ctypes.c_int, [_SIM, ctypes.c_int32, _D]),
    ("fpd_set_static_phi", ctypes.c_int, [_SIM, _D]),
    ("fpd_record_start", ctypes.c_int, [_SIM, ctypes.c_int32, ctypes.c_int64]),
    ("fpd_record_stop", ctypes.c_int, [_SIM]),
    ("fpd_record_read", ctypes.c_int, [_SIM, _D, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_set_launch", ctypes.c_int, [_SIM, ctypes.POINTER(fpd_launch)]),
    ("fpd_get_launch", ctypes.c_int, [_SIM, ctypes.POINTER(fpd_launch)]),
    ("fpd_set_flags", ctypes.c_int, [_SIM, ctypes.c_uint32]),
    ("fpd_split_active", ctypes.c_int, [_SIM, ctypes.POINTER(ctypes.c_int32)]),
    ("fpd_kernel_times", ctypes.c_int,
     [_SIM, _D, ctypes.POINTER(ctypes.c_int64), _D, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_reset_kernel_times", ctypes.c_int, [_SIM]),
    ("fpd_copy_probe", ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, _D]),
    ("fpd_save", ctypes.c_int, [_SIM, ctypes.c_char_p]),
    ("fpd_load", ctypes.c_int, [_SIM, ctypes.c_char_p]),
    ("fpd_static_scratch_need", ctypes.c_size_t, [ctypes.POINTER(fpd_params)]),
    ("fpd_run_static", ctypes.c_int,
     [ctypes.POINTER(fpd_params), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
      ctypes.c_int64]),
    ("fpd_sim_footprint", ctypes.c_size_t, [ctypes.POINTER(fpd_params)]),
    ("fpd_batch_create", ctypes.c_int,
     [ctypes.c_size_t, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(_SIM)]),
    ("fpd_batch_set_launch", ctypes.c_int, [_SIM, ctypes.POINTER(fpd_launch)]),
    ("fpd_batch_add", ctypes.c_int,
     [_SIM, ctypes.POINTER(fpd_params), _D, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_batch_run", ctypes.c_int, [_SIM, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_batch_launch", ctypes.c_int, [_SIM, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_batch_wait", ctypes.c_int, [_SIM]),
    ("fpd_batch_poll", ctypes.c_int,
     [_SIM, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
      ctypes.POINTER(ctypes.c_int32)]),
    ("fpd_batch_read_beads", ctypes.c_int, [_SIM, ctypes.c_int64, _D, _D, _D]),
    ("fpd_batch_read_populations", ctypes.c_int, [_SIM, ctypes.c_int64, _D]),
    ("fpd_batch_read_fields", ctypes.c_int, [_SIM, ctypes.c_int64, _D, _D, _D, _D]),
    ("fpd_batch_particle_stats", ctypes.c_int, [_SIM, ctypes.c_int64, ctypes.c_int32, _D]),
    ("fpd_batch_set_static_phi", ctypes.c_int, [_SIM, ctypes.c_int64, _D]),
    ("fpd_batch_record_start", ctypes.c_int, [_SIM, ctypes.c_int64, ctypes.c_int32, ctypes.c_int64]),
    ("fpd_batch_record_read", ctypes.c_int, [_SIM, ctypes.c_int64, _D, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64)]),
    ("fpd_batch_sim_info", ctypes.c_int,
     [_SIM, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
      ctypes.POINTER(ctypes.c_uint32)]),
    ("fpd_batch_release", ctypes.c_int, [_SIM, ctypes.c_int64]),
    ("fpd_batch_stats", ctypes.c_int,
     [_SIM, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
      ctypes.POINTER(ctypes.c_size_t)]),
    ("fpd_batch_destroy", None, [_SIM]),
]

FPD_SIM_ACTIVE, FPD_SIM_DONE, FPD_SIM_FAILED = 0, 1, 2

_lib = None


class FpdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fpd error {code}: {msg}")
        self.code = code


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                " or `python paper_2212_14153_amd/build.py`")
        # torch ships its own HIP runtime.  Loading it first makes the library bind to that
        # runtime (the same soname) in a process that also uses torch; loaded the other way
        # round, the process would hold two HIP runtimes and torch's would find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int) -> int:
    if rc != FPD_OK:
        raise FpdError(rc, lib().fpd_last_error().decode())
    return rc


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


# ------------------------------------------------------------ thin C-name wrappers ---

def fpd_params_default() -> fpd_params:
    p = fpd_params()
    lib().fpd_params_default(ctypes.byref(p))
    return p


def fpd_params_from_physical(re_ps, confinement, kappa, n_beads, radius, eta_ratio, xi,
                             u_wall, nx_over_ny) -> fpd_params:
    p = fpd_params()
    check(lib().fpd_params_from_physical(re_ps, confinement, kappa, n_beads, radius,
                                         eta_ratio, xi, u_wall, nx_over_ny, ctypes.byref(p)))
    return p


def fpd_population_bytes(p: fpd_params) -> int:
    return int(lib().fpd_population_bytes(ctypes.byref(p)))


def fpd_copy_probe(stream, nbytes: int, iters: int) -> float:
    out = ctypes.c_double()
    check(lib().fpd_copy_probe(stream, nbytes, iters, ctypes.byref(out)))
    return out.value


FPD_STATIC_SCRATCH_BYTES = 8388608


def fpd_static_scratch_need(p: fpd_params) -> int:
    return int(lib().fpd_static_scratch_need(ctypes.byref(p)))


def fpd_run_static(p: fpd_params, stream, f_a, f_b, bytes_each: int, init_populations: bool,
                   R_in, R_out, health, n_steps: int):
    """fpd_run_static on device addresses (integers or objects with data_ptr(), e.g. torch
    tensors; R_in, R_out and health may be None)."""
    def addr(x):
        if x is None:
            return None
        return x.data_ptr() if hasattr(x, "data_ptr") else int(x)
    check(lib().fpd_run_static(ctypes.byref(p), stream, addr(f_a), addr(f_b), int(bytes_each),
                               1 if init_populations else 0, addr(R_in), addr(R_out),
                               addr(health), int(n_steps)))


def params_from_mapping(m, storage=None, **over) -> fpd_params:
    """Build fpd_params from a mapping with the same field names (extra keys ignored)."""
    p = fpd_params_default()
    d = dict(m)
    d.update(over)
    for name, _ in fpd_params._fields_:
        if name in d and name != "storage":
            v = d[name]
            setattr(p, name, tuple(v) if name in ("f_ext", "g_body") else v)
    st = storage if storage is not None else d.get("storage", "f32")
    p.storage = STORAGE[st] if isinstance(st, str) else int(st)
    return p


@dataclass
class LaunchConfig:
    block_x: int = 64
    block_y: int = 4
    rows_per_thread: int = 1
    xcd_remap: int = 2
    graph_chunk: int = 64


def buffer_args(buffers):
    """(a, b) or (a, b, nbytes) -> the two device addresses and the usable size of each:
    objects with data_ptr() (e.g. torch tensors) give their address and size, integers are
    addresses whose size must be given."""
    a, b = buffers[0], buffers[1]
    if len(buffers) > 2:
        nbytes = int(buffers[2])
    else:
        sizes = [x.numel() * x.element_size() if hasattr(x, "element_size") else None
                 for x in (a, b)]
        if None in sizes:
            raise ValueError("integer buffer addresses need their size in bytes")
        nbytes = min(sizes)
    pa, pb = (x.data_ptr() if hasattr(x, "data_ptr") else int(x) for x in (a, b))
    return pa, pb, nbytes


class Simulation:
    """One simulation on the current HIP device, driven through the C ABI."""

    def __init__(self, params: fpd_params, stream=None, buffers=None):
        """buffers: None (the library allocates), or (a, b) or (a, b, nbytes) with two device
        buffers of at least fpd_population_bytes(params) bytes each, 16-byte aligned, given
        as objects with data_ptr() (e.g. torch tensors, whose sizes are then read) or as
        integer addresses (nbytes required).  The simulation keeps a reference to them."""
        self.p = params
        self._buffers = None
        h = _SIM()
        if buffers is None:
            check(lib().fpd_create(ctypes.byref(params), stream, ctypes.byref(h)))
        else:
            pa, pb, nbytes = buffer_args(buffers)
            check(lib().fpd_create_with_buffers(ctypes.byref(params), stream, pa, pb, nbytes,
                                                ctypes.byref(h)))
            self._buffers = tuple(buffers[:2])  # the owners outlive the simulation's use
        self.h = h
        self.nx, self.ny, self.n = params.nx, params.ny, params.n_beads

    # lifecycle
    def close(self):
        if self.h:
            lib().fpd_destroy(self.h)
            self.h = _SIM()
        self._buffers = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def init_fiber(self, R):
        R = np.ascontiguousarray(R, dtype=np.float64).reshape(self.n, 2)
        check(lib().fpd_init_fiber(self.h, _ptr(R)))

    def init_fiber_line(self, cx, cy, theta):
        check(lib().fpd_init_fiber_line(self.h, cx, cy, theta))

    def step(self, n: int):
        check(lib().fpd_step(self.h, int(n)))

    def capture(self, n: int):
        """Capture the graph that step(n) replays, without running a step."""
        check(lib().fpd_capture(self.h, int(n)))

    def sync(self):
        check(lib().fpd_sync(self.h))

    def health(self):
        f = ctypes.c_uint32()
        s = ctypes.c_double()
        check(lib().fpd_health(self.h, ctypes.byref(f), ctypes.byref(s)))
        return f.value, s.value

    def clear_health(self):
        check(lib().fpd_clear_health(self.h))

    @property
    def steps(self) -> int:
        v = ctypes.c_int64()
        check(lib().fpd_step_count(self.h, ctypes.byref(v)))
        return v.value

    # data
    def populations(self) -> np.ndarray:
        f = np.empty((9, self.ny, self.nx))
        check(lib().fpd_read_populations(self.h, _ptr(f)))
        return f

    def write_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        check(lib().fpd_write_populations(self.h, _ptr(f)))

    def fields(self):
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        check(lib().fpd_read_fields(self.h, *[_ptr(o) for o in out]))
        return tuple(out)

    def set_static_phi(self, phi):
        """Fixed profile phi_s(y) [ny] added to sum_i phi_i in Eq. (1); None removes it."""
        if phi is None:
            check(lib().fpd_set_static_phi(self.h, None))
            return
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.ny)
        check(lib().fpd_set_static_phi(self.h, _ptr(phi)))

    def record_start(self, every: int = 1, capacity: int = 1 << 16):
        """Record each fiber's end-to-end vector and centroid every `every` steps."""
        check(lib().fpd_record_start(self.h, int(every), int(capacity)))

    def record_stop(self):
        check(lib().fpd_record_stop(self.h))

    def record(self) -> np.ndarray:
        """[records, 1 + 4 fibers]: step, then (ex, ey, cx, cy) per fiber, oldest first."""
        return _read_record(lambda out, cap, n: lib().fpd_record_read(self.h, out, cap, n),
                            self.p.n_chains)

    STATS_FIELDS = ("A", "V0x", "V0y", "eps_v", "Fvisc_x", "Fvisc_y", "Fpres_x", "Fpres_y")

    def particle_stats(self, bead: int = 0) -> dict:
        """Driven-particle diagnostics of one bead on the current state (fpd_particle_stats):
        A, the phi-weighted velocity V0, eps_v (Eq. 15), viscous and pressure forces."""
        out = np.empty(8)
        check(lib().fpd_particle_stats(self.h, int(bead), _ptr(out)))
        return dict(zip(self.STATS_FIELDS, out.tolist()))

    def beads(self):
        R = np.empty((max(self.n, 0), 2))
        V = np.empty_like(R)
        F = np.empty_like(R)
        if self.n:
            check(lib().fpd_read_beads(self.h, _ptr(R), _ptr(V), _ptr(F)))
        return R, V, F

    # tuning / timing
    def set_launch(self, cfg: LaunchConfig | dict):
        d = cfg if isinstance(cfg, dict) else cfg.__dict__
        c = fpd_launch(*(int(d.get(k, 0)) for k, _ in fpd_launch._fields_))
        check(lib().fpd_set_launch(self.h, ctypes.byref(c)))

    def set_flags(self, flags: int):
        check(lib().fpd_set_flags(self.h, int(flags)))

    def split_active(self) -> bool:
        on = ctypes.c_int32(0)
        check(lib().fpd_split_active(self.h, ctypes.byref(on)))
        return bool(on.value)

    def get_launch(self) -> LaunchConfig:
        c = fpd_launch()
        check(lib().fpd_get_launch(self.h, ctypes.byref(c)))
        return LaunchConfig(c.block_x, c.block_y, c.rows_per_thread, c.xcd_remap, c.graph_chunk)

    def kernel_times(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        na, nb = ctypes.c_int64(), ctypes.c_int64()
        check(lib().fpd_kernel_times(self.h, ctypes.byref(a), ctypes.byref(na), ctypes.byref(b),
                                     ctypes.byref(nb)))
        return a.value, na.value, b.value, nb.value

    def reset_kernel_times(self):
        check(lib().fpd_reset_kernel_times(self.h))

    def save(self, path: str):
        check(lib().fpd_save(self.h, path.encode()))

    def load(self, path: str):
        check(lib().fpd_load(self.h, path.encode()))


def simulation_from_workload(w, storage=None, stream=None, flags=0, **over) -> Simulation:
    """Create a Simulation for a workload (lattice parameters + straight fiber)."""
    p = params_from_mapping(w.params(), storage=storage if storage else w.storage, flags=flags,
                            **over)
    sim = Simulation(p, stream=stream)
    if p.n_beads > 0:
        sim.init_fiber(w.beads())
    return sim


def fpd_sim_footprint(p: fpd_params) -> int:
    return int(lib().fpd_sim_footprint(ctypes.byref(p)))


def _read_record(call, n_chains: int) -> np.ndarray:
    width = 1 + 4 * max(int(n_chains), 1)
    n = ctypes.c_int64()
    check(call(None, 0, ctypes.byref(n)))
    out = np.empty((n.value, width))
    if n.value:
        check(call(_ptr(out), n.value, ctypes.byref(n)))
    return out


class Batch:
    """A batch of independent simulations advanced together (C ABI fpd_batch_*)."""

    def __init__(self, hbm_budget: int, max_slots: int, storage="f32", stream=None):
        h = _SIM()
        st = STORAGE[storage] if isinstance(storage, str) else int(storage)
        check(lib().fpd_batch_create(int(hbm_budget), int(max_slots), st, stream,
                                     ctypes.byref(h)))
        self.h = h
        self.storage = st
        self.shapes = {}
        self.chains = {}

    def close(self):
        if self.h:
            lib().fpd_batch_destroy(self.h)
            self.h = _SIM()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_launch(self, cfg):
        d = cfg if isinstance(cfg, dict) else cfg.__dict__
        c = fpd_launch(*(int(d.get(k, 0)) for k, _ in fpd_launch._fields_))
        check(lib().fpd_batch_set_launch(self.h, ctypes.byref(c)))

    def add(self, params: fpd_params, R, n_steps: int) -> int:
        """Admit a simulation; raises FpdError (code FPD_ENOMEM) when it does not fit."""
        sid = ctypes.c_int64()
        Rp = None
        if params.n_beads > 0:
            R = np.ascontiguousarray(R, dtype=np.float64).reshape(params.n_beads, 2)
            Rp = _ptr(R)
        check(lib().fpd_batch_add(self.h, ctypes.byref(params), Rp, int(n_steps),
                                  ctypes.byref(sid)))
        self.shapes[sid.value] = (params.nx, params.ny, params.n_beads)
        self.chains[sid.value] = max(int(params.n_chains), 1)
        return sid.value

    def try_add(self, params: fpd_params, R, n_steps: int):
        try:
            return self.add(params, R, n_steps)
        except FpdError as e:
            if e.code == FPD_ENOMEM:
                return None
            raise

    def run(self, max_steps: int) -> int:
        adv = ctypes.c_int64()
        check(lib().fpd_batch_run(self.h, int(max_steps), ctypes.byref(adv)))
        return adv.value

    def launch(self, max_steps: int) -> int:
        """Enqueue the steps run() would take without waiting (wait() completes them)."""
        adv = ctypes.c_int64()
        check(lib().fpd_batch_launch(self.h, int(max_steps), ctypes.byref(adv)))
        return adv.value

    def wait(self):
        check(lib().fpd_batch_wait(self.h))

    def poll(self, cap: int = 4096):
        ids = (ctypes.c_int64 * cap)()
        st = (ctypes.c_int32 * cap)()
        n = ctypes.c_int32()
        check(lib().fpd_batch_poll(self.h, ids, st, cap, ctypes.byref(n)))
        return [(ids[i], st[i]) for i in range(n.value)]

    def beads(self, sid: int):
        nx, ny, n = self.shapes[sid]
        R, V, F = (np.empty((n, 2)) for _ in range(3))
        if n:
            check(lib().fpd_batch_read_beads(self.h, sid, _ptr(R), _ptr(V), _ptr(F)))
        return R, V, F

    def record_start(self, sid: int, every: int = 1, capacity: int = 1 << 16):
        check(lib().fpd_batch_record_start(self.h, int(sid), int(every), int(capacity)))

    def record(self, sid: int) -> np.ndarray:
        chains = self.chains.get(sid, 1)
        return _read_record(lambda out, cap, n: lib().fpd_batch_record_read(self.h, int(sid), out,
                                                                             cap, n), chains)

    def set_static_phi(self, sid: int, phi):
        """Fixed profile phi_s(y) for one simulation of the batch (None removes it)."""
        if phi is None:
            check(lib().fpd_batch_set_static_phi(self.h, int(sid), None))
            return
        arr = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.shapes[sid][1])
        check(lib().fpd_batch_set_static_phi(self.h, int(sid), _ptr(arr)))

    def particle_stats(self, sid: int, bead: int = 0) -> dict:
        out = np.empty(8)
        check(lib().fpd_batch_particle_stats(self.h, int(sid), int(bead), _ptr(out)))
        return dict(zip(Simulation.STATS_FIELDS, out.tolist()))

    def populations(self, sid: int):
        nx, ny, n = self.shapes[sid]
        f = np.empty((9, ny, nx))
        check(lib().fpd_batch_read_populations(self.h, sid, _ptr(f)))
        return f

    def fields(self, sid: int):
        nx, ny, n = self.shapes[sid]
        out = [np.empty((ny, nx)) for _ in range(4)]
        check(lib().fpd_batch_read_fields(self.h, sid, *[_ptr(o) for o in out]))
        return tuple(out)

    def info(self, sid: int):
        steps, status, health = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_uint32()
        check(lib().fpd_batch_sim_info(self.h, sid, ctypes.byref(steps), ctypes.byref(status),
                                       ctypes.byref(health)))
        return steps.value, status.value, health.value

    def release(self, sid: int):
        check(lib().fpd_batch_release(self.h, sid))
        self.shapes.pop(sid, None)

    def stats(self):
        a, h, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_size_t()
        check(lib().fpd_batch_stats(self.h, ctypes.byref(a), ctypes.byref(h), ctypes.byref(b)))
        return a.value, h.value, b.value
