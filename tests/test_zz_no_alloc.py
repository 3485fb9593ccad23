"""fpd_run_static, the entry point that allocates no device memory, against the entry points
it stands in for (fpd_create_with_buffers + fpd_init_fiber + fpd_step): bitwise the same
populations and bead positions, on two calls in a row, the second on a smaller input."""
import math

import numpy as np
import pytest

from paper_2212_14153_amd import _lib
import workloads

ELEM = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}


def case(big: bool, storage: str):
    """The larger case: the 64 x 32 channel with a 5-bead fiber; the smaller one a 40 x 24
    channel with 3 beads."""
    if big:
        w = workloads.c1_small_fp64()
        n_steps = 131          # two replayed graphs of 64 steps and three direct steps
    else:
        w = workloads._make("small_40x24", nx=40, ny=24, n_beads=3, radius=2.0, l0=3.0,
                            u_wall=0.02, re_ps=0.5, kappa=1.0, theta0=math.radians(30),
                            steps=20, storage=storage)
        n_steps = 20
    p = _lib.params_from_mapping(w.params(), storage=storage)
    return p, w.beads(), n_steps


def valid_words(buf, p, storage):
    """The populations of a raw buffer as integers (bitwise), padding columns dropped."""
    import torch
    dt = {8: torch.int64, 4: torch.int32, 2: torch.int16}[ELEM[storage]]
    plane = (p.nx + 63) // 64 * 64
    v = buf.view(dt)[: p.ny * 9 * plane].reshape(p.ny, 9, plane)
    return v[:, :, : p.nx].cpu()


def run_pair(storage, big, stream):
    import torch
    p, R, n_steps = case(big, storage)
    nbytes = _lib.fpd_population_bytes(p)
    # the existing entry points on buffers (a1, b1)
    a1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    sim = _lib.Simulation(p, stream=stream.cuda_stream, buffers=(a1, b1))
    initial = valid_words(a1, p, storage)
    sim.init_fiber(R)
    sim.step(n_steps)
    sim.sync()
    R_ref = sim.beads()[0]
    ref = valid_words(a1 if n_steps % 2 == 0 else b1, p, storage)
    sim.close()
    # the allocation-free entry point on buffers (a2, b2) filled with other bytes
    a2 = torch.full((nbytes,), 0x5A, dtype=torch.uint8, device="cuda")
    b2 = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    R_in = torch.tensor(R, dtype=torch.float64, device="cuda")
    R_out = torch.full_like(R_in, float("nan"))
    health = torch.full((1,), 0xFFFFFFF, dtype=torch.int32, device="cuda")
    if big:   # one call: initial state, fiber and steps
        _lib.fpd_run_static(p, stream.cuda_stream, a2, b2, nbytes, True, R_in, R_out, health,
                            n_steps)
    else:     # the initial state first (no steps), then the steps from it
        _lib.fpd_run_static(p, stream.cuda_stream, a2, b2, nbytes, True, R_in, R_out, health,
                            0)
        stream.synchronize()
        assert torch.equal(valid_words(a2, p, storage), initial)
        assert torch.equal(R_out.cpu(), R_in.cpu())
        _lib.fpd_run_static(p, stream.cuda_stream, a2, b2, nbytes, False, R_in, R_out, health,
                            n_steps)
    stream.synchronize()
    got = valid_words(a2 if n_steps % 2 == 0 else b2, p, storage)
    assert torch.equal(got, ref), f"{storage} big={big}: populations differ"
    assert np.array_equal(R_out.cpu().numpy(), R_ref), f"{storage} big={big}: beads differ"
    assert int(health.item()) == 0


@pytest.mark.gpu
@pytest.mark.parametrize("storage", ["f64", "f32", "f16dev", "bf16dev"])
def test_static_entry_matches_the_allocating_path(storage):
    import torch
    stream = torch.cuda.Stream()
    run_pair(storage, True, stream)
    run_pair(storage, False, stream)     # second call, smaller input, same scratch array


@pytest.mark.gpu
def test_static_entry_without_beads():
    """No fiber: populations only; the health word is cleared."""
    import torch
    p = _lib.params_from_mapping(workloads.c1_small_fp64().params(), storage="f32",
                                 n_beads=0)
    nbytes = _lib.fpd_population_bytes(p)
    a1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b1 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    sim = _lib.Simulation(p, stream=stream.cuda_stream, buffers=(a1, b1))
    sim.step(10)
    sim.sync()
    ref = valid_words(a1, p, "f32")
    sim.close()
    a2 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    b2 = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    health = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    _lib.fpd_run_static(p, stream.cuda_stream, a2, b2, nbytes, True, None, None, health, 10)
    stream.synchronize()
    assert torch.equal(valid_words(a2, p, "f32"), ref)
    assert int(health.item()) == 0


def test_static_entry_rejects_what_does_not_fit():
    """Checked on the host before any device work: a several-fiber lattice whose force
    window (the whole lattice) exceeds the static array, a small buffer, missing beads."""
    L = _lib.lib()
    w = workloads.fiber_suspension(n_fibers=4, beads=5, nx=2048, ny=1024, storage="f32")
    p = _lib.params_from_mapping(w.params(), storage="f32")
    need = _lib.fpd_static_scratch_need(p)
    assert need > _lib.FPD_STATIC_SCRATCH_BYTES
    nbytes = _lib.fpd_population_bytes(p)
    with pytest.raises(_lib.FpdError) as e:
        _lib.fpd_run_static(p, None, 1 << 20, 2 << 20, nbytes, True, 4096, 4096, None, 1)
    assert e.value.code == _lib.FPD_EINVAL
    assert b"FPD_STATIC_SCRATCH_BYTES" in L.fpd_last_error()
    q, R, _ = case(True, "f32")
    assert 0 < _lib.fpd_static_scratch_need(q) <= _lib.FPD_STATIC_SCRATCH_BYTES
    nb = _lib.fpd_population_bytes(q)
    with pytest.raises(_lib.FpdError) as e:
        _lib.fpd_run_static(q, None, 1 << 20, 2 << 20, nb - 16, True, 4096, 4096, None, 1)
    assert e.value.code == _lib.FPD_EINVAL
    with pytest.raises(_lib.FpdError) as e:
        _lib.fpd_run_static(q, None, 1 << 20, 2 << 20, nb, True, None, None, None, 1)
    assert e.value.code == _lib.FPD_EINVAL
