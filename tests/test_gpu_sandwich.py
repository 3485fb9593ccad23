"""The sandwich benchmark of Sec. III.A on the GPU: a fixed interface profile phi_s(y)
(Eq. 14) in Eq. (1) between the moving walls, through the C ABI.

  * parity with the oracle on the same profile (FP64 1e-12 relative, FP32 1e-5, FP16 within
    its rounding), odd widths included;
  * the steady profile against the exact solution of the smooth problem: the shear stress
    is uniform, so v(y) follows int_0^y 1/eta; within 0.3 % of V0 = 2U at the paper's
    grid (dx / H = 0.005), and within 4 % of the sharp-interface Eq. (13) at r_eta = 50,
    r_xi = 0.01 (the paper's accuracy threshold);
  * a batch holding profiled and plain simulations equals each alone, bitwise.
"""
import numpy as np
import pytest

import oracle
import workloads
from paper_2212_14153_amd import _lib

pytestmark = pytest.mark.gpu


def rel_err(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def orc_params(w, phi):
    p = oracle.OracleParams.from_mapping(w.params())
    p.phi_static = phi
    return p


@pytest.mark.parametrize("nx", [8, 5])
@pytest.mark.parametrize("storage,steps", [("f64", 300), ("f32", 300), ("f16dev", 3)])
def test_sandwich_matches_oracle(nx, storage, steps):
    w = workloads.sandwich(ny=48, nx=nx, r_eta=20.0, r_xi=0.02, re=1.0, u_wall=0.01,
                           storage=storage)
    phi = workloads.sandwich_phi(48, w.xi)
    print(f"[case] sandwich {nx}x48 {storage}", flush=True)
    st = oracle.make_state(orc_params(w, phi), 1)
    oracle.run(st, steps)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.set_static_phi(phi)
        sim.step(steps)
        sim.sync()
        f = sim.populations()
        rho, ux, uy, eta = sim.fields()
    if storage == "f64":
        assert rel_err(f, st.f) <= 1e-12
    elif storage == "f32":
        assert rel_err(f, st.f) <= 1e-5
    else:
        assert np.max(np.abs(f - st.f)) <= 2.0 * (steps + 1) * 0.02 * 2.0 ** -11
    eta_o = w.nu_f * (1 + (w.eta_ratio - 1) * phi)
    assert np.abs(eta[:, 0] - eta_o).max() <= 1e-12 * eta_o.max()


def steady_profile_errors(u, w):
    H, U = w.ny, w.u_wall
    y = np.arange(H) + 0.5
    yy = np.linspace(0, H, 400001)
    inv = 1 / (w.nu_f * (1 + (w.eta_ratio - 1) * workloads.sandwich_phi_at(yy, H, w.xi)))
    cum = np.concatenate([[0], np.cumsum(0.5 * (inv[1:] + inv[:-1]) * np.diff(yy))])
    smooth = -U + 2 * U * np.interp(y, yy, cum) / cum[-1]
    sharp = np.clip(-U + 2 * U * (y - H / 3) / (H / 3), -U, U)      # Eq. (13), shifted
    return np.abs(u - smooth).max() / (2 * U), np.abs(u - sharp).max() / (2 * U)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_sandwich_steady_profile(storage):
    w = workloads.sandwich(ny=200, nx=64, r_eta=50.0, r_xi=0.01, storage=storage)
    print(f"[case] sandwich steady {storage}", flush=True)
    with _lib.simulation_from_workload(w, storage=storage) as sim:
        sim.set_static_phi(workloads.sandwich_phi(200, w.xi))
        sim.step(3000)
        rho, ux, uy, eta = sim.fields()
    assert np.abs(ux - ux[:, :1]).max() < 1e-12          # no x dependence
    e_smooth, e_sharp = steady_profile_errors(ux[:, 0], w)
    assert e_smooth < 3e-3
    assert e_sharp < 4e-2


def test_removing_the_profile_gives_plain_couette():
    w = workloads.sandwich(ny=32, nx=8, r_eta=50.0, r_xi=0.02, re=1.0, u_wall=0.01)
    with _lib.simulation_from_workload(w, storage="f64") as a, \
            _lib.simulation_from_workload(w, storage="f64") as b:
        a.set_static_phi(workloads.sandwich_phi(32, w.xi))
        a.set_static_phi(None)
        a.step(50)
        b.step(50)
        assert np.array_equal(a.populations(), b.populations())
        with pytest.raises(_lib.FpdError):
            a.set_static_phi(np.full(32, -1.0))


def test_sandwich_batch_equals_alone():
    ws = [workloads.sandwich(ny=40 + 8 * i, nx=24, r_eta=10.0 * (i + 1), r_xi=0.02, re=1.0,
                             u_wall=0.01, storage="f32") for i in range(3)]
    ws.append(workloads.c1_small_fp64().with_(storage="f32"))
    phis = [workloads.sandwich_phi(w.ny, w.xi) if i < 3 else None for i, w in enumerate(ws)]
    print("[case] sandwich batch", flush=True)
    alone = []
    for w, phi in zip(ws, phis):
        with _lib.simulation_from_workload(w, storage="f32") as sim:
            if phi is not None:
                sim.set_static_phi(phi)
            sim.step(70)
            alone.append(sim.populations())
    params = [_lib.params_from_mapping(w.params(), storage="f32") for w in ws]
    budget = sum(_lib.fpd_sim_footprint(p) for p in params) * 2
    with _lib.Batch(budget, len(ws), storage="f32") as b:
        ids = [b.add(p, w.beads(), 70) for p, w in zip(params, ws)]
        for sid, phi in zip(ids, phis):
            if phi is not None:
                b.set_static_phi(sid, phi)
        while b.run(32):
            pass
        for sid, f in zip(ids, alone):
            assert np.array_equal(b.populations(sid), f)
