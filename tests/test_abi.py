"""The C-ABI library loads and exports every entry point include/utrast.h declares; host-only
calls (tiling, sizes, argument validation) behave.  No GPU compute here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "utrast.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ut_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2510_12901_amd import _abi
    return _abi.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 18
    from paper_2510_12901_amd import _abi
    bound = {n for n, _, _ in _abi.SIGNATURES}
    for n in names:
        assert hasattr(L, n), n
        assert n in bound, f"{n} has no Python binding"


def test_record_size_and_status(L):
    assert L.ut_record_bytes() == 128
    assert L.ut_status_str(0) == b"ok"
    assert b"argument" in L.ut_status_str(-1)


def test_library_tiling_matches_oracle_alg1(L):
    from paper_2510_12901_amd import lidar_tiling
    for seed in range(4):
        be = synth.beams_uniform(np.random.default_rng(seed), 128)
        for n_phi, M in [(16, 32), (8, 64), (32, 32), (4, 256)]:
            a = lidar_tiling(be, 2048, n_phi, M)
            b = oracle.lidar_tiling(be, 2048, n_phi, M)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_argument_errors_return_before_launch(L):
    from paper_2510_12901_amd import _abi as A
    assert L.ut_project(None, None, None, None, None) == A.UT_ERR_ARG
    g = A.UtGaussians(None, None, None, None, None, 10, 5, 0)       # sh_degree 5 invalid
    assert L.ut_project(A.ref(g), None, None, None, None) == A.UT_ERR_ARG
    s = A.UtSensor()
    s.kind = 7
    assert L.ut_sensor_build(A.ref(s), None) == A.UT_ERR_ARG
    # unsorted beams are rejected by the tiling
    be = np.array([0.1, 0.0], np.float32)
    out = np.zeros(3)
    bs = np.zeros(3, np.int32)
    nt = C.c_int32()
    assert L.ut_lidar_tiling(be.ctypes.data, 2, 8, 2, 4, out.ctypes.data, bs.ctypes.data, C.byref(nt)) == A.UT_ERR_ARG
    # camera composite on a LiDAR sensor is an argument error
    s.kind = A.LIDAR
    assert L.ut_composite_camera(None, None, A.ref(s), None, None, None) == A.UT_ERR_ARG


def test_workspace_sizes_monotone(L):
    a = L.ut_workspace_bytes(0, 100, 1000)
    b = L.ut_workspace_bytes(10 ** 6, 100, 1000)
    assert b > a > 0
    assert L.ut_backward_workspace_bytes(1000) == 13 * 8 * 1000
    assert L.ut_batch_workspace_bytes(7) > 256


def test_argument_errors_of_the_later_entry_points(L):
    """Host-side checks of the device-count sort, the adjoint, the batch and the actor
    transforms return before anything is enqueued (no GPU needed)."""
    from paper_2510_12901_amd import _abi as A
    assert L.ut_bin_sort_device(None, 0, None, None, 0, None, 0, 0, None, None, None) == A.UT_ERR_ARG
    assert L.ut_composite_backward(None, None, None, None, None, None, None, None, 0, None, None) == A.UT_ERR_ARG
    assert L.ut_composite_batch(None, 0, None, None, 0, 1, None) == A.UT_ERR_ARG
    arr = (A.UtBatchItem * 1)()
    prm = A.UtRenderParams(1 / 255, 0.99, 1e-4)
    assert L.ut_composite_batch(C.cast(arr, C.c_void_p), 1, A.ref(prm), C.c_void_p(8), 1 << 20, -1, None) == A.UT_ERR_ARG
    g = A.UtGaussians(None, None, None, None, None, 0, 0, 0)
    assert L.ut_actor_transform(None, None, None, 0, None, None, None) == A.UT_ERR_ARG
    assert L.ut_actor_transform(A.ref(g), None, None, -1, None, None, None) == A.UT_ERR_ARG
    assert L.ut_actor_transform(A.ref(g), None, None, 2, None, None, None) == A.UT_ERR_ARG   # poses missing
    g.n = 5
    assert L.ut_actor_transform(A.ref(g), None, None, 0, None, None, None) == A.UT_ERR_ARG   # arrays missing
    assert L.ut_actor_transform_backward(A.ref(g), None, None, 0, None, None, None, None, None, None) == A.UT_ERR_ARG
    # an empty set with no actors is a valid no-op that touches no device memory
    g.n = 0
    assert L.ut_actor_transform(A.ref(g), None, None, 0, None, None, None) == A.UT_OK
