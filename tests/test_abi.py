"""The C ABI library loads, exports every declared symbol and validates input
on the host (no device needed)."""

import ctypes
import math

import pytest

from paper_1004_1122_amd import lshom


@pytest.fixture(scope="module")
def lib():
    return lshom.load()


def test_every_header_symbol_is_exported(lib):
    import glob
    import os
    names = []
    inc = os.path.join(os.path.dirname(lshom.HEADER_PATH), "*.h")
    for path in sorted(glob.glob(inc)):
        names += lshom.header_symbols(path)
    assert "lshom_solve" in names and "lshom_set_microstructure" in names
    assert "lshom_cnn_forward" in names and "lshom_cnn_train_step" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    for s in range(-7, 1):
        assert lshom.lshom_status_string(s)
    assert lshom.lshom_status_string(0) == "ok"


def test_default_opts():
    o = lshom.lshom_default_opts()
    assert o.max_iter == 10000 and o.precision == 0 and o.graph_block == 16
    assert o.refresh_every == 50 and abs(o.refresh_drop - 0.01) < 1e-15 and o.true_residual == 1


@pytest.mark.parametrize("d,N,cond,l0,E,tol,expect", [
    (2, (63, 63), [1.0, 10.0], 5.5, [1.0, 0.0], 1e-8, 0),
    (3, (15, 9, 7), [1.0, 2.0, 3.0], 0.0, [1, 2, 3], 1e-6, 0),
    (2, (4, 6), [1.0], 1.0, None, 0.0, 0),                    # even sizes
    (1, (63,), [1.0], 1.0, None, 1e-6, -1),                   # d not in {2,3}
    (4, (3, 3, 3, 3), [1.0], 1.0, None, 1e-6, -1),
    (2, (2, 63), [1.0], 1.0, None, 1e-6, -1),                 # N < 3
    (2, (19, 63), [1.0], 1.0, None, 1e-6, -7),                # prime factor 19
    (2, (255, 39), [1.0], 1.0, None, 1e-6, 0),                # prime factors 17 and 13
    (2, (8192, 3), [1.0], 1.0, None, 1e-6, -7),               # too long
    # the LDS footprint of the default pass shapes (both precisions, 160 KiB
    # per workgroup less the static reserve) and the threads of one block
    # bound the axis lengths below 4096: 1800 in 2-D, 1224 for cubes
    (2, (729, 729), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (2, (1331, 1331), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (2, (1600, 1600), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (2, (1800, 1800), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (2, (1728, 1728), [1.0, 10.0], 0.0, None, 1e-6, -7),
    (2, (2187, 2187), [1.0, 10.0], 0.0, None, 1e-6, -7),
    (3, (1224, 1224, 1224), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (2, (4096, 9), [1.0, 10.0], 0.0, None, 1e-6, -7),
    (3, (243, 243, 243), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (3, (975, 975, 975), [1.0, 10.0], 0.0, None, 1e-6, 0),
    (3, (1024, 1024, 1024), [1.0, 10.0], 0.0, None, 1e-6, -7),
    (3, (1331, 1331, 1331), [1.0, 10.0], 0.0, None, 1e-6, -7),  # 2^31 or more nodes
    (2, (9, 9), [1.0, 0.0], 1.0, None, 1e-6, -1),             # cond <= 0
    (2, (9, 9), [1.0, math.inf], 1.0, None, 1e-6, -1),        # cond not finite
    (2, (9, 9), [1.0, math.nan], 1.0, None, 1e-6, -1),
    (2, (9, 9), [1.0], -1.0, None, 1e-6, -1),                 # l0 < 0
    (2, (9, 9), [1.0], math.inf, None, 1e-6, -1),
    (2, (9, 9), [1.0], 1.0, [math.nan, 0.0], 1e-6, -1),       # E not finite
    (2, (9, 9), [1.0], 1.0, None, math.nan, -1),              # tol NaN
    (2, (9, 9), [1.0], 1.0, None, math.inf, -1),
])
def test_check_problem(d, N, cond, l0, E, tol, expect):
    assert lshom.lshom_check_problem(d, N, cond, l0, E, tol) == expect


def test_phase_count_limits():
    assert lshom.lshom_check_problem(2, (9, 9), [1.0] * 256) == 0
    assert lshom.lshom_check_problem(2, (9, 9), [1.0] * 257) == -1
    assert lshom.lshom_check_problem(2, (9, 9), []) == -1


def test_null_context_is_rejected(lib):
    assert lib.lshom_solve(None, None, 1e-6, None, None, None, None, None) == -1
    assert lib.lshom_set_reference(None, 1.0) == -1
    assert lib.lshom_apply(None, None, None) == -1
    size = ctypes.c_size_t()
    assert lib.lshom_workspace_size(None, 0, ctypes.byref(size)) == -1
    assert lshom.load().lshom_last_error(None) == b""
    # the entry points of tensor phases, cells, general references and sizing by options
    eye = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 1.0)
    assert lib.lshom_set_reference_tensor(None, eye) == -1
    assert lib.lshom_set_cell(None, eye) == -1
    N = (ctypes.c_int64 * 2)(9, 9)
    assert lib.lshom_set_microstructure_tensor(None, 2, N, None, 1, eye) == -1
    o = lshom.lshom_default_opts()
    assert lib.lshom_workspace_size_for(None, ctypes.byref(o), ctypes.byref(size)) == -1
    E = (ctypes.c_double * 2)(1.0, 0.0)
    assert lib.lshom_solve_static(None, E, 1e-6, None, None, None, None) == -1


def test_static_workspace_size_matches_header():
    import re
    text = open(lshom.HEADER_PATH).read()
    m = re.search(r"#define LSHOM_STATIC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", text)
    assert m, "LSHOM_STATIC_WORKSPACE_BYTES not found in the header"
    assert int(m.group(1)) << int(m.group(2)) == lshom.LSHOM_STATIC_WORKSPACE_BYTES


def test_method_constants_match_header():
    import re
    text = open(lshom.HEADER_PATH).read()
    for name in ("METHOD_CG", "METHOD_FFTH", "METHOD_BICG", "METHOD_PIPECG", "NORM_RESIDUAL",
                 "NORM_EQUILIBRIUM", "PRECISION_FP64", "PRECISION_MIXED"):
        m = re.search(r"#define LSHOM_%s (-?\d+)" % name, text)
        assert m and int(m.group(1)) == getattr(lshom, name), name


def test_create_without_gpu_fails_cleanly(lib):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert lib.lshom_create(ctypes.byref(h), 0, None) == lshom.LSHOM_ERR_HIP
    assert not h.value


def test_cnn_create_without_gpu_fails_cleanly(lib):
    import ctypes
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1004_1122_amd import cnn
    lib = cnn._lib()
    h = ctypes.c_void_p()
    assert lib.lshom_cnn_create(ctypes.byref(h), 0, None, 32) == lshom.LSHOM_ERR_HIP
    assert lib.lshom_cnn_create(ctypes.byref(h), 0, None, 12) == lshom.LSHOM_ERR_INVALID_ARG
    assert not h.value
