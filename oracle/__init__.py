"""Python access to the FP64 CPU oracle (``fpd_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, single-threaded FP64 reference of
the FPD fiber time step (arXiv:2212.14153, Sec. II) that the GPU library is checked
against.  Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

Arrays use the oracle's own layout: populations ``f[9, ny, nx]`` (k-major), beads
``R[N, 2]``, per-node fields ``[ny, nx]``; all float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpd_oracle.c")
_LIB = os.path.join(_HERE, "libfpd_oracle.so")

# The oracle is compiled without FMA contraction or fast-math so that every
# operation rounds as written.
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c99"]


def build() -> str:
    """Compile the oracle with gcc into ``oracle/libfpd_oracle.so``."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("u_wall", ctypes.c_double), ("nu_f", ctypes.c_double),
        ("eta_ratio", ctypes.c_double), ("xi", ctypes.c_double),
        ("n_beads", ctypes.c_int),
        ("radius", ctypes.c_double), ("l0", ctypes.c_double),
        ("k_s", ctypes.c_double), ("k_b", ctypes.c_double),
        ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_q_fixed", ctypes.c_double),
        ("clamp_phi", ctypes.c_int),
        ("periodic_y", ctypes.c_int),
        ("fx_ext", ctypes.c_double), ("fy_ext", ctypes.c_double),
        ("gx_body", ctypes.c_double), ("gy_body", ctypes.c_double),
        ("phi_static", ctypes.POINTER(ctypes.c_double)),
        ("n_chains", ctypes.c_int),
        ("ev_k", ctypes.c_double), ("ev_range", ctypes.c_double),
    ]


@dataclass
class OracleParams:
    """Lattice-unit parameters of one simulation (oracle's own mirror of them)."""
    nx: int
    ny: int
    u_wall: float = 0.0
    nu_f: float = 1.0 / 6.0
    eta_ratio: float = 50.0
    xi: float = 1.0
    n_beads: int = 0
    radius: float = 2.0
    l0: float = 4.0
    k_s: float = 0.0
    k_b: float = 0.0
    s_e: float = 1.64
    s_eps: float = 1.54
    s_q_fixed: float = 0.0
    clamp_phi: int = 0
    periodic_y: int = 0       # 1: no walls (the single-particle box of Sec. III.B)
    fx_ext: float = 0.0       # external force on every bead
    fy_ext: float = 0.0
    gx_body: float = 0.0      # uniform body force density on every node
    gy_body: float = 0.0
    phi_static: object = None  # None or [ny]: fixed profile phi_s(y) added in Eq. (1)
    n_chains: int = 1          # fibers of n_beads / n_chains consecutive beads each
    ev_k: float = 0.0          # excluded volume between fibers (0: none)
    ev_range: float = 0.0      # its range d (<= 0: 2a)

    def c(self) -> _Params:
        ps = None
        if self.phi_static is not None:
            self._phi_keep = np.ascontiguousarray(self.phi_static, dtype=np.float64)
            assert self._phi_keep.shape == (self.ny,)
            ps = self._phi_keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return _Params(self.nx, self.ny, self.u_wall, self.nu_f, self.eta_ratio, self.xi,
                       self.n_beads, self.radius, self.l0, self.k_s, self.k_b, self.s_e,
                       self.s_eps, self.s_q_fixed, self.clamp_phi, self.periodic_y,
                       self.fx_ext, self.fy_ext, self.gx_body, self.gy_body, ps,
                       self.n_chains, self.ev_k, self.ev_range)

    @classmethod
    def from_mapping(cls, m) -> "OracleParams":
        names = {f for f in cls.__dataclass_fields__}
        return cls(**{k: v for k, v in dict(m).items() if k in names})


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load the compiled oracle, building it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Params)
        L.orc_bead_forces.argtypes = [P, _D, _D]
        L.orc_phi.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        L.orc_phi.restype = ctypes.c_double
        L.orc_fields.argtypes = [P, _D, _D, _D, _D, _D, _D]
        L.orc_meq.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, _D]
        L.orc_moments.argtypes = [_D, _D]
        L.orc_inverse_moments.argtypes = [_D, _D]
        L.orc_collide.argtypes = [_D] + [ctypes.c_double] * 6 + [_D]
        L.orc_stream.argtypes = [P, _D, _D]
        L.orc_lbm_step_fields.argtypes = [P, _D, _D, _D, _D]
        L.orc_bare_velocity.argtypes = [P, _D, _D, _D, _D]
        L.orc_step.argtypes = [P, _D, _D, _D, _D]
        L.orc_run.argtypes = [P, _D, _D, ctypes.c_long, _D, _D, _D]
        L.orc_init.argtypes = [P, ctypes.c_int, _D]
        L.orc_macro.argtypes = [P, _D, _D, _D, _D, _D, _D]
        L.orc_iso_gradient.argtypes = [P, _D, _D, _D]
        L.orc_particle_stats.argtypes = [P, _D, _D, ctypes.c_int, _D]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# --------------------------------------------------------------------- wrappers ---

def bead_forces(p: OracleParams, R) -> np.ndarray:
    """F_i of Eqs. (10)-(12) for bead positions R[N, 2]."""
    R = _f64(R, (p.n_beads, 2))
    F = np.zeros_like(R)
    lib().orc_bead_forces(ctypes.byref(p.c()), _p(R), _p(F))
    return F


def phi(p: OracleParams, Rx: float, Ry: float, i: int, j: int) -> float:
    """Eq. (2) at node (i, j) for a bead at (Rx, Ry)."""
    return lib().orc_phi(ctypes.byref(p.c()), Rx, Ry, i, j)


def fields(p: OracleParams, R):
    """Step (1): returns (A[N], F[N,2], eta[ny,nx], fx[ny,nx], fy[ny,nx])."""
    N = p.n_beads
    R = _f64(R, (max(N, 0), 2)) if N else np.zeros((1, 2))
    A = np.zeros(max(N, 1))
    F = np.zeros((max(N, 1), 2))
    eta = np.zeros((p.ny, p.nx))
    fx = np.zeros((p.ny, p.nx))
    fy = np.zeros((p.ny, p.nx))
    lib().orc_fields(ctypes.byref(p.c()), _p(R), _p(A), _p(F), _p(eta), _p(fx), _p(fy))
    return A[:N], F[:N], eta, fx, fy


def meq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_meq(rho, ux, uy, _p(out))
    return out


def moments(f) -> np.ndarray:
    f = _f64(f, (9,))
    out = np.zeros(9)
    lib().orc_moments(_p(f), _p(out))
    return out


def inverse_moments(m) -> np.ndarray:
    m = _f64(m, (9,))
    out = np.zeros(9)
    lib().orc_inverse_moments(_p(m), _p(out))
    return out


def collide(f, s_nu, s_e, s_eps, s_q, Fx=0.0, Fy=0.0) -> np.ndarray:
    """One MRT collision with Guo forcing at a single node."""
    f = _f64(f, (9,))
    out = np.zeros(9)
    lib().orc_collide(_p(f), s_nu, s_e, s_eps, s_q, Fx, Fy, _p(out))
    return out


def stream(p: OracleParams, fpost) -> np.ndarray:
    fpost = _f64(fpost, (9, p.ny, p.nx))
    out = np.zeros_like(fpost)
    lib().orc_stream(ctypes.byref(p.c()), _p(fpost), _p(out))
    return out


def lbm_step_fields(p: OracleParams, f, s_nu, fx, fy) -> np.ndarray:
    """One LBM collide+stream with prescribed per-node s_nu and force density; returns a new array."""
    f = _f64(f, (9, p.ny, p.nx)).copy()
    s_nu = _f64(np.broadcast_to(s_nu, (p.ny, p.nx)))
    fx = _f64(np.broadcast_to(fx, (p.ny, p.nx)))
    fy = _f64(np.broadcast_to(fy, (p.ny, p.nx)))
    lib().orc_lbm_step_fields(ctypes.byref(p.c()), _p(f), _p(s_nu), _p(fx), _p(fy))
    return f


def bare_velocity(p: OracleParams, f):
    f = _f64(f, (9, p.ny, p.nx))
    rho = np.zeros((p.ny, p.nx)); vx = np.zeros_like(rho); vy = np.zeros_like(rho)
    lib().orc_bare_velocity(ctypes.byref(p.c()), _p(f), _p(rho), _p(vx), _p(vy))
    return rho, vx, vy


def init(p: OracleParams, init_flow: int) -> np.ndarray:
    """Equilibrium populations at rest (0) or on the linear Couette profile (1)."""
    f = np.zeros((9, p.ny, p.nx))
    lib().orc_init(ctypes.byref(p.c()), int(init_flow), _p(f))
    return f


@dataclass
class OracleState:
    p: OracleParams
    f: np.ndarray
    R: np.ndarray
    V: np.ndarray = field(default=None)
    F: np.ndarray = field(default=None)
    steps: int = 0


def make_state(p: OracleParams, init_flow: int, R=None) -> OracleState:
    N = p.n_beads
    R = _f64(R, (N, 2)).copy() if N else np.zeros((0, 2))
    return OracleState(p, init(p, init_flow), R, np.zeros((N, 2)), np.zeros((N, 2)))


def run(st: OracleState, n_steps: int, trajectory: bool = False):
    """Advance the state by n_steps full steps in place; optionally return R after each step."""
    p = st.p
    N = p.n_beads
    Rb = st.R if N else np.zeros((1, 2))
    Vb = st.V if N else np.zeros((1, 2))
    Fb = st.F if N else np.zeros((1, 2))
    traj = np.zeros((n_steps, max(N, 1), 2)) if (trajectory and n_steps > 0) else None
    lib().orc_run(ctypes.byref(p.c()), _p(st.f), _p(Rb), int(n_steps), _p(Vb), _p(Fb),
                  _p(traj) if traj is not None else None)
    st.steps += int(n_steps)
    if traj is not None:
        return traj[:, :N, :]
    return None


def macro(p: OracleParams, f, R):
    """(rho, ux, uy, eta) with u = (j + f/2)/rho at the current bead state."""
    N = p.n_beads
    f = _f64(f, (9, p.ny, p.nx))
    Rb = _f64(R, (N, 2)) if N else np.zeros((1, 2))
    rho = np.zeros((p.ny, p.nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
    eta = np.zeros_like(rho)
    lib().orc_macro(ctypes.byref(p.c()), _p(f), _p(Rb), _p(rho), _p(ux), _p(uy), _p(eta))
    return rho, ux, uy, eta


def iso_gradient(p: OracleParams, q):
    """Isotropic D2Q9 gradient (gx, gy) of a node field q[ny, nx]."""
    q = _f64(q, (p.ny, p.nx))
    gx = np.zeros_like(q)
    gy = np.zeros_like(q)
    lib().orc_iso_gradient(ctypes.byref(p.c()), _p(q), _p(gx), _p(gy))
    return gx, gy


STATS_FIELDS = ("A", "V0x", "V0y", "eps_v", "Fvisc_x", "Fvisc_y", "Fpres_x", "Fpres_y")


def particle_stats(p: OracleParams, f, R, bead: int = 0) -> dict:
    """Single-particle diagnostics of Sec. III.B for one bead on the current state:
    A, the phi-weighted velocity V0, eps_v (Eq. 15) and the viscous and pressure forces
    of Eq. (17) in diffuse-interface form."""
    f = _f64(f, (9, p.ny, p.nx))
    Rb = _f64(R, (p.n_beads, 2))
    out = np.zeros(8)
    lib().orc_particle_stats(ctypes.byref(p.c()), _p(f), _p(Rb), int(bead), _p(out))
    return dict(zip(STATS_FIELDS, out.tolist()))
