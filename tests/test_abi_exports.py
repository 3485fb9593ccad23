"""The C-ABI library loads on a machine without a GPU and exports every symbol that
include/fpdlbm.h declares; host-only entry points behave (no device work here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpdlbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2212_14153_amd import _lib
    return _lib.lib()


def test_header_declares_the_expected_entry_points():
    names = declared_functions()
    for must in ("fpd_create", "fpd_step", "fpd_read_fields", "fpd_read_beads",
                 "fpd_init_fiber", "fpd_read_populations", "fpd_destroy", "fpd_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2212_14153_amd import _lib
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert set(declared_functions()) == bound


def test_params_struct_layout_matches_header():
    """The ctypes mirror has the field order of the C struct (checked by name)."""
    from paper_2212_14153_amd import _lib
    text = open(HEADER).read()
    body = text[text.index("typedef struct fpd_params {"):text.index("} fpd_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b([a-z_0-9]+)(?:\[\d+\])?\s*[,;]", body)
    assert fields == [n for n, _ in _lib.fpd_params._fields_]


def test_params_default_and_physical_mapping(L):
    from paper_2212_14153_amd import _lib
    import workloads
    p = _lib.fpd_params_default()
    assert p.s_e == 1.64 and p.s_eps == 1.54 and p.storage == _lib.FPD_F32
    q = _lib.fpd_params_from_physical(5.0, 320 / 2048, 3.3, 40, 4.0, 50.0, 1.0, 0.01, 4)
    assert (q.nx, q.ny) == (8192, 2048)
    w = workloads.c3_large("f32")
    assert q.nu_f == pytest.approx(w.nu_f, rel=1e-12)
    assert q.k_b == pytest.approx(w.k_b, rel=1e-12)
    assert q.k_s == pytest.approx(w.k_s, rel=1e-12)


def test_invalid_parameters_are_rejected_without_a_device(L):
    from paper_2212_14153_amd import _lib
    with pytest.raises(_lib.FpdError) as e:
        _lib.fpd_params_from_physical(-1.0, 0.2, 1.0, 5, 2.0, 50, 1, 0.01, 2)
    assert e.value.code == _lib.FPD_EINVAL
    p = _lib.fpd_params_default()
    p.nu_f = 0.0
    h = ctypes.c_void_p()
    assert L.fpd_create(ctypes.byref(p), None, ctypes.byref(h)) == _lib.FPD_EINVAL
    assert b"tau_f" in L.fpd_last_error()


def test_population_bytes(L):
    from paper_2212_14153_amd import _lib
    p = _lib.fpd_params_default()
    p.nx, p.ny, p.storage = 100, 7, _lib.FPD_F16DEV
    assert _lib.fpd_population_bytes(p) == 9 * 7 * 128 * 2


def test_caller_buffer_arguments():
    """The binding's reading of caller-owned buffers (fpd_create_with_buffers): objects with
    data_ptr() give address and size (the smaller of the two), integers need a size."""
    from paper_2212_14153_amd import _lib

    class Tensor:  # the few attributes of a torch tensor the binding reads
        def __init__(self, ptr, numel, esize):
            self.ptr, self.n, self.e = ptr, numel, esize

        def data_ptr(self):
            return self.ptr

        def numel(self):
            return self.n

        def element_size(self):
            return self.e

    assert _lib.buffer_args((Tensor(4096, 100, 4), Tensor(8192, 96, 4))) == (4096, 8192, 384)
    assert _lib.buffer_args((Tensor(4096, 100, 4), Tensor(8192, 96, 4), 200)) == (4096, 8192, 200)
    assert _lib.buffer_args((4096, 8192, 123)) == (4096, 8192, 123)
    with pytest.raises(ValueError):
        _lib.buffer_args((4096, 8192))


def test_lattice_size_limits(L):
    """The row pitch (nine padded direction rows) must fit 32 bits and ny one grid row per
    lattice row; the buffer itself may exceed 2^31 values."""
    from paper_2212_14153_amd import _lib
    h = ctypes.c_void_p()
    p = _lib.fpd_params_default()
    p.nx, p.ny = 16384, 16384                       # 2.4e9 values per buffer: accepted
    assert _lib.fpd_sim_footprint(p) == 2 * 9 * 16384 * 16384 * 4 + _lib.fpd_sim_footprint(
        _lib.fpd_params_default()) - 2 * 9 * 32 * 64 * 4
    p.ny = 65536
    assert L.fpd_create(ctypes.byref(p), None, ctypes.byref(h)) == _lib.FPD_EINVAL
    assert b"ny" in L.fpd_last_error()
    p.ny, p.nx = 8, (1 << 31) // 9
    assert L.fpd_create(ctypes.byref(p), None, ctypes.byref(h)) == _lib.FPD_EINVAL
    assert b"nx" in L.fpd_last_error()
