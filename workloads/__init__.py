"""Seeded synthetic workloads for the FPD fiber solver (arXiv:2212.14153, Sec. IV).

This module only states *inputs*: lattice sizes, physical groups turned into lattice
units, straight initial fibers, and seeded random perturbations.  It holds none of the
method's arithmetic (no equilibria, no collision, no forces), so both the GPU library
and the CPU oracle can be fed from it.

The paper runs its own simulations and uses no public dataset.  The configurations
below re-create its workloads synthetically: a straight fiber of N beads centred in a
confined Couette channel (Sec. IV.A), with the dimensionless groups of Eq. (18)
mapped to lattice units:

    shear rate        gamma = 2 U / H                      (Fig. 1 caption)
    Reynolds number   Re_ps = gamma l_c^2 / (4 nu_f)       (Eq. 18, rho = 1)
    stiffness         K     = 2 k_b / (eta_f gamma l_c^2)  (Eq. 18)
    confinement       C     = l_c / H                      (Eq. 18)

The stretching constant is not taken from the paper's K_s = 3.33e6, which is unstable
for explicit coupling in lattice units; k_s / l_0^2 = 0.1 * pi * a^2 is used instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict, replace

import numpy as np

S_E_DEFAULT = 1.64
S_EPS_DEFAULT = 1.54


@dataclass(frozen=True)
class Workload:
    """One simulation in lattice units plus its initial fiber."""
    name: str
    nx: int
    ny: int
    u_wall: float
    nu_f: float
    eta_ratio: float
    xi: float
    n_beads: int
    radius: float
    l0: float
    k_s: float
    k_b: float
    theta0: float            # initial fiber angle in radians
    cx: float                # fiber centroid
    cy: float
    steps: int
    storage: str = "f64"     # "f64" | "f32" | "f16dev" | "bf16dev"
    init_flow: int = 1       # 0 rest, 1 linear Couette
    s_e: float = S_E_DEFAULT
    s_eps: float = S_EPS_DEFAULT
    s_q_fixed: float = 0.0
    kappa: float = float("nan")
    re_ps: float = float("nan")
    confinement: float = float("nan")
    boundary: int = 0                    # 0 moving walls, 1 periodic box (no walls)
    f_ext: tuple = (0.0, 0.0)            # external force on every bead
    g_body: tuple = (0.0, 0.0)           # uniform body force density on every node
    n_chains: int = 1                    # fibers of n_beads / n_chains consecutive beads
    centres: tuple = ()                  # several fibers: ((cx, cy, theta), ...)
    ev_k: float = 0.0                    # excluded volume between fibers (0: none)
    ev_range: float = 0.0                # its range (<= 0: 2a)

    def params(self) -> dict:
        """Lattice parameters as a plain mapping (both sides read what they need; the
        boundary and the two forces are also given under the oracle's names)."""
        d = {k: v for k, v in asdict(self).items()}
        d.update(periodic_y=int(self.boundary == 1), fx_ext=self.f_ext[0],
                 fy_ext=self.f_ext[1], gx_body=self.g_body[0], gy_body=self.g_body[1])
        return d

    def beads(self) -> np.ndarray:
        if self.n_chains > 1:
            L = self.n_beads // self.n_chains
            return np.concatenate([straight_fiber(L, self.l0, th, x, y)
                                   for (x, y, th) in self.centres])
        return straight_fiber(self.n_beads, self.l0, self.theta0, self.cx, self.cy)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)

    @property
    def sites(self) -> int:
        return self.nx * self.ny


def straight_fiber(n: int, l0: float, theta: float, cx: float, cy: float) -> np.ndarray:
    """R_i = c + (i - (N+1)/2) l0 (cos theta, sin theta), i = 1..N."""
    i = np.arange(1, n + 1, dtype=np.float64)
    s = (i - (n + 1) / 2.0) * l0
    return np.stack([cx + s * math.cos(theta), cy + s * math.sin(theta)], axis=1)


def stretch_constant(radius: float, l0: float) -> float:
    """k_s with k_s / l0^2 = 0.1 * pi * a^2 (stable explicit coupling)."""
    return 0.1 * math.pi * radius * radius * l0 * l0


def physical_to_lattice(*, nx: int, ny: int, n_beads: int, radius: float, l0: float,
                        u_wall: float, re_ps: float, kappa: float) -> dict:
    """nu_f and k_b from Re_ps and K of Eq. (18) (rho = 1, l_c = N l0)."""
    lc = n_beads * l0
    gamma = 2.0 * u_wall / ny
    nu_f = gamma * lc * lc / (4.0 * re_ps)
    k_b = kappa * nu_f * gamma * lc * lc / 2.0
    return {"nu_f": nu_f, "k_b": k_b, "k_s": stretch_constant(radius, l0),
            "confinement": lc / ny}


def _make(name, *, nx, ny, n_beads, radius, l0, u_wall, re_ps, kappa, theta0, steps,
          storage, eta_ratio=50.0, xi=1.0, init_flow=1) -> Workload:
    m = physical_to_lattice(nx=nx, ny=ny, n_beads=n_beads, radius=radius, l0=l0,
                            u_wall=u_wall, re_ps=re_ps, kappa=kappa)
    return Workload(name=name, nx=nx, ny=ny, u_wall=u_wall, nu_f=m["nu_f"],
                    eta_ratio=eta_ratio, xi=xi, n_beads=n_beads, radius=radius, l0=l0,
                    k_s=m["k_s"], k_b=m["k_b"], theta0=theta0, cx=nx / 2.0, cy=ny / 2.0,
                    steps=steps, storage=storage, init_flow=init_flow, kappa=kappa,
                    re_ps=re_ps, confinement=m["confinement"])


def c1_small_fp64() -> Workload:
    """64x32 channel, U = 0.01, 5 beads of radius 2 at spacing 2 tilted 45 deg,
    r_eta = 50, xi = 1, Re_ps = 1, K = 0.33 (the paper's S-turn stiffness), 1000 steps."""
    return _make("c1_64x32_fp64", nx=64, ny=32, n_beads=5, radius=2.0, l0=2.0, u_wall=0.01,
                 re_ps=1.0, kappa=0.33, theta0=math.pi / 4, steps=1000, storage="f64")


def c2_medium_fp32(seed: int = 2212) -> Workload:
    """1024x256, 20 beads of radius 3, l_c / H = 0.5, Re_ps = 10, K log-uniform in
    [1e-3, 1e1] drawn from the seed, flat start (theta = 0), 50k steps."""
    rng = np.random.default_rng(seed)
    kappa = float(10.0 ** rng.uniform(-3.0, 1.0))
    lc = 0.5 * 256
    return _make("c2_1024x256_fp32", nx=1024, ny=256, n_beads=20, radius=3.0, l0=lc / 20,
                 u_wall=0.01, re_ps=10.0, kappa=kappa, theta0=0.0, steps=50000,
                 storage="f32")


def c3_large(storage: str = "f32") -> Workload:
    """8192x2048 (16.8M sites), 40 beads of radius 4 at spacing 8, Re_ps = 5, K = 3.3,
    theta = 45 deg, 2000 steps: the bandwidth-roofline run."""
    return _make(f"c3_8192x2048_{storage}", nx=8192, ny=2048, n_beads=40, radius=4.0,
                 l0=8.0, u_wall=0.01, re_ps=5.0, kappa=3.3, theta0=math.pi / 4,
                 steps=2000, storage=storage)


def sweep_sims(count: int = 256, seed: int = 14153, steps: int = 20000,
               storage: str = "f32") -> list:
    """Parameter-sweep simulations: N_y ~ U{64..512}, N_x = 2 N_y, N ~ U{5..30},
    C ~ U[0.2, 0.8], l0 = C N_y / N, a = l0 / 2 (tuples with a < 2 are drawn again),
    Re_ps ~ U[1, 10], U = Re_ps / (15 C^2 H) clamped to [1e-3, 0.05] (targets nu = 1/30),
    K ~ log-uniform [1e-3, 1e1], xi = 1, r_eta = 50, theta = 45 deg."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        ny = int(rng.integers(64, 513))
        n = int(rng.integers(5, 31))
        conf = float(rng.uniform(0.2, 0.8))
        re = float(rng.uniform(1.0, 10.0))
        kappa = float(10.0 ** rng.uniform(-3.0, 1.0))
        lc = conf * ny
        l0 = lc / n
        a = l0 / 2.0
        if a < 2.0:
            continue
        u = min(max(re / (15.0 * conf * conf * ny), 1e-3), 0.05)
        out.append(_make(f"sweep{len(out):03d}", nx=2 * ny, ny=ny, n_beads=n, radius=a,
                         l0=l0, u_wall=u, re_ps=re, kappa=kappa, theta0=math.pi / 4,
                         steps=steps, storage=storage))
    return out


def sweep_sim_at_height(ny: int, seed: int, steps: int = 20000,
                        storage: str = "f32") -> Workload:
    """One simulation of the parameter sweep (sweep_sims) at a given channel height: N, C,
    Re_ps and K drawn from the sweep's distributions (tuples with a < 2 drawn again),
    N_x = 2 N_y, the same mapping to lattice units."""
    rng = np.random.default_rng(seed)
    while True:
        n = int(rng.integers(5, 31))
        conf = float(rng.uniform(0.2, 0.8))
        re = float(rng.uniform(1.0, 10.0))
        kappa = float(10.0 ** rng.uniform(-3.0, 1.0))
        l0 = conf * ny / n
        if l0 / 2.0 >= 2.0:
            break
    u = min(max(re / (15.0 * conf * conf * ny), 1e-3), 0.05)
    return _make(f"sweep_{2 * ny}x{ny}_s{seed}", nx=2 * ny, ny=ny, n_beads=n, radius=l0 / 2.0,
                 l0=l0, u_wall=u, re_ps=re, kappa=kappa, theta0=math.pi / 4, steps=steps,
                 storage=storage)


def flexible_fiber(kappa: float, confinement: float, re_ps: float, n_beads: int = 10,
                   diameter: float = 8.0, gamma: float = 1.5e-4, eta_ratio: float = 100.0,
                   xi: float = 1.0, theta0: float = 0.0, storage: str = "f32",
                   steps: int = 400000) -> Workload:
    """One point of the shape diagrams of Sec. IV.C: a fiber of N touching beads
    (l_0 = d, r_c = d / l_c = 1 / N) lying flat (theta = 0) at the centre of a channel of
    height H = N d / C (rounded to whole nodes) and length L_x = 25 d, r_eta = 100 and
    xi / d = 0.125 as in the paper's fiber runs.  The shear rate is the same for every
    point (so all runs cover the same strain per step); Re_ps sets nu_f and K sets k_b
    through Eq. (18)."""
    lc = n_beads * diameter
    ny = int(round(lc / confinement))
    nx = int(round(25 * diameter))
    u = 0.5 * gamma * ny
    name = f"shape_K{kappa:.3g}_C{lc / ny:.3f}_Re{re_ps:g}"
    return _make(name, nx=nx, ny=ny, n_beads=n_beads, radius=diameter / 2.0, l0=diameter,
                 u_wall=u, re_ps=re_ps, kappa=kappa, theta0=theta0, steps=steps,
                 storage=storage, eta_ratio=eta_ratio, xi=xi)


def poisson_arrivals(count: int, rate: float = 50.0, seed: int = 50) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


def driven_particle(n: int = 48, radius: float = 3.0, xi: float = 1.0, force: float = 1e-4,
                    eta_ratio: float = 50.0, nu_f: float = 1.0 / 6.0, storage: str = "f64",
                    steps: int = 4000, offset=(0.3, 0.1)) -> Workload:
    """The single-particle benchmark of Sec. III.B: one bead (a disk of radius a) in an
    n x n periodic box (no walls), pushed along x by a constant force F0; the uniform body
    force -F0 / n^2 on every node keeps the total momentum at zero, so the fluid far from
    the particle stays at rest on average.  The paper's box is H = 10 d; the bead starts
    slightly off the node lattice (offset) so that no symmetry is special."""
    return Workload(
        name=f"particle_{n}x{n}_a{radius:g}_{storage}", nx=n, ny=n, u_wall=0.0, nu_f=nu_f,
        eta_ratio=eta_ratio, xi=xi, n_beads=1, radius=radius, l0=2.0 * radius, k_s=0.0,
        k_b=0.0, theta0=0.0, cx=n / 2 + offset[0], cy=n / 2 + offset[1], steps=steps,
        storage=storage, init_flow=0, boundary=1, f_ext=(force, 0.0),
        g_body=(-force / (n * n), 0.0))


def fiber_suspension(n_fibers: int = 8, beads: int = 10, nx: int = 1024, ny: int = 256,
                     radius: float = 3.0, re_ps: float = 5.0, kappa: float = 1.0,
                     u_wall: float = 0.01, storage: str = "f32", seed: int = 4447,
                     steps: int = 5000) -> Workload:
    """Several straight fibers (touching beads, l0 = 2a) at seeded random positions and
    angles in the +-U Couette channel, kept apart by at least one contour length and away
    from the walls; the groups of Eq. (18) are those of one fiber."""
    l0 = 2.0 * radius
    lc = beads * l0
    gamma = 2.0 * u_wall / ny
    nu = gamma * lc * lc / (4.0 * re_ps)
    rng = np.random.default_rng(seed)
    centres = []
    reach = 0.5 * lc + radius + 2.0
    while len(centres) < n_fibers:
        th = float(rng.uniform(0, math.pi))
        x = float(rng.uniform(0, nx))
        y = float(rng.uniform(reach, ny - reach))
        if all(min(abs(x - cx), nx - abs(x - cx)) ** 2 + (y - cy) ** 2 > (1.2 * lc) ** 2
               for cx, cy, _ in centres):
            centres.append((x, y, th))
    return Workload(
        name=f"suspension_{n_fibers}x{beads}_{nx}x{ny}_{storage}", nx=nx, ny=ny,
        u_wall=u_wall, nu_f=nu, eta_ratio=50.0, xi=1.0, n_beads=n_fibers * beads,
        radius=radius, l0=l0, k_s=0.1 * math.pi * radius ** 2 * l0 ** 2,
        k_b=kappa * nu * gamma * lc * lc / 2.0, theta0=0.0, cx=0.0, cy=0.0, steps=steps,
        storage=storage, kappa=kappa, re_ps=re_ps, confinement=lc / ny, n_chains=n_fibers,
        centres=tuple(centres))


def sandwich_phi_at(y, H: float, xi: float) -> np.ndarray:
    """Eq. (14) at heights y: the solid | fluid | solid sandwich of Sec. III.A with the
    interfaces at z_L = H/3 and z_R = 2H/3."""
    y = np.asarray(y, dtype=np.float64)
    zl, zr = H / 3.0, 2.0 * H / 3.0
    return np.where(y <= H / 2.0, 0.5 * (np.tanh((zl - y) / xi) + 1.0),
                    0.5 * (np.tanh((y - zr) / xi) + 1.0))


def sandwich_phi(ny: int, xi: float) -> np.ndarray:
    """Eq. (14) at the row centres y = j + 1/2 of a channel of height H = ny."""
    return sandwich_phi_at(np.arange(ny, dtype=np.float64) + 0.5, float(ny), xi)


def sandwich(ny: int = 200, nx: int = 200, r_eta: float = 50.0, r_xi: float = 0.01,
             re: float = 0.1, u_wall: float = 0.005, storage: str = "f64",
             steps: int = 6000) -> Workload:
    """The Couette benchmark of Sec. III.A: walls at y = 0 and y = H moving at -U and +U
    (the paper's 0 and V0 = 2U, shifted by V0/2), Re = V0 H / nu_f, solid slabs of
    viscosity r_eta eta_f given by sandwich_phi(H, r_xi H); the paper's grid has
    dx / H = 0.005, i.e. H = 200.  No beads."""
    nu_f = 2.0 * u_wall * ny / re
    return Workload(
        name=f"sandwich_{ny}_r{r_eta:g}_x{r_xi:g}_{storage}", nx=nx, ny=ny, u_wall=u_wall,
        nu_f=nu_f, eta_ratio=r_eta, xi=r_xi * ny, n_beads=0, radius=1.0, l0=2.0, k_s=0.0,
        k_b=0.0, theta0=0.0, cx=0.0, cy=0.0, steps=steps, storage=storage, init_flow=1)


def perturbation(shape, amplitude: float, seed: int) -> np.ndarray:
    """Seeded uniform noise in [-amplitude, amplitude] (float64)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=shape)


def random_beads(n: int, nx: int, ny: int, margin: float, seed: int) -> np.ndarray:
    """n bead centres drawn uniformly in [0, nx) x [margin, ny - margin]."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.uniform(0.0, nx, n), rng.uniform(margin, ny - margin, n)], axis=1)
