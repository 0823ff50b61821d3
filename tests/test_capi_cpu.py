"""C ABI checks that need no GPU: the library loads, exports every function
the header declares, and its host-only entry points behave."""
import ctypes as C

from paper_1502_03543_amd import capi


def test_exports_every_declared_symbol():
    lib = capi.load()
    declared = capi.declared_functions()
    assert "lp_setup" in declared and "lp_iterate" in declared and "lp_solve" in declared
    missing = [f for f in declared if not hasattr(lib, f)]
    assert not missing, missing


def test_status_strings():
    for code, name in [(0, "LP_OK"), (1, "LP_CONVERGED"), (2, "LP_OPTIMAL_PSI1"),
                       (-4, "LP_ERR_BREAKDOWN"), (-9, "LP_ERR_DEVICE"), (99, "LP_UNKNOWN_STATUS")]:
        assert capi.status_string(code) == name


def test_workspace_size_and_validation():
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    assert o.alpha == 0.95 and o.precision == capi.LP_PREC_FP64
    sz = C.c_size_t(0)
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_OK
    small = sz.value
    assert small > 0 and small % 256 == 0
    assert capi.lp_workspace_size(2048, 8192, C.byref(o), C.byref(sz)) == capi.LP_OK
    # M alone is m^2 doubles
    assert sz.value >= 2048 * 2048 * 8
    assert capi.lp_workspace_size(10, 10, C.byref(o), C.byref(sz)) == capi.LP_ERR_SHAPE
    assert capi.lp_workspace_size(0, 10, C.byref(o), C.byref(sz)) == capi.LP_ERR_SHAPE
    o.alpha = 1.0
    assert capi.lp_workspace_size(8, 16, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
    o.alpha = 0.9
    o.tape_capacity = 30
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_OK
    assert sz.value >= small + 31 * (2 * 256 + 64) * 8


def test_setup_rejects_bad_workspace_without_touching_device():
    h = C.c_void_p()
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    dummy = C.c_void_p(256)
    st = capi.lp_setup(C.byref(h), 8, 16, dummy, dummy, dummy, dummy, dummy, dummy,
                       C.byref(o), None, 0, None)
    assert st == capi.LP_ERR_WORKSPACE and not h.value
    st = capi.lp_setup(C.byref(h), 16, 8, dummy, dummy, dummy, dummy, dummy, dummy,
                       C.byref(o), dummy, 1 << 30, None)
    assert st == capi.LP_ERR_SHAPE


def test_method_validation():
    """LP_METHOD_PC runs in FP64 without a tape and not in batches; an unknown
    method is rejected."""
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    assert o.method == capi.LP_METHOD_AFFINE
    sz = C.c_size_t(0)
    o.method = capi.LP_METHOD_PC
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_OK
    o.precision = capi.LP_PREC_MIXED
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
    o.precision = capi.LP_PREC_FP64
    o.tape_capacity = 4
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
    o.tape_capacity = 0
    o.method = 2
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
    o.method = capi.LP_METHOD_PC
    m = (C.c_int64 * 2)(16, 20)
    n = (C.c_int64 * 2)(40, 60)
    assert capi.lp_batch_workspace_size(2, m, n, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG


def test_solver_validation():
    """LP_SOLVER_WOODBURY: FP64, Section 3 method, no tape, and a problem whose
    recurrence fits one workgroup's LDS."""
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    assert o.solver == capi.LP_SOLVER_CHOLESKY and o.reserved == 0
    sz = C.c_size_t(0)
    o.solver = capi.LP_SOLVER_WOODBURY
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_OK
    assert capi.lp_workspace_size(128, 1024, C.byref(o), C.byref(sz)) == capi.LP_ERR_SHAPE
    for field, value in (("precision", capi.LP_PREC_MIXED), ("method", capi.LP_METHOD_PC),
                         ("tape_capacity", 2), ("reserved", 1)):
        old = getattr(o, field)
        setattr(o, field, value)
        assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
        setattr(o, field, old)
    o.solver = 2
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG


def test_csr_validation():
    """lp_setup_csr's workspace rules: FP64 Cholesky without a tape (either
    method), m <= LP_CSR_MAX_M, 0 <= nnz <= INT32_MAX; the sparse workspace
    holds the CSC (index, value and map arrays) but no split-K scratch."""
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    sz = C.c_size_t(0)
    dense = C.c_size_t(0)
    assert capi.lp_workspace_size_csr(2048, 8192, 170000, C.byref(o), C.byref(sz)) == capi.LP_OK
    assert capi.lp_workspace_size(2048, 8192, C.byref(o), C.byref(dense)) == capi.LP_OK
    assert sz.value % 256 == 0 and sz.value >= 2048 * 2048 * 8 + 170000 * 20
    assert capi.lp_workspace_size_csr(64, 256, 0, C.byref(o), C.byref(sz)) == capi.LP_OK
    assert capi.lp_workspace_size_csr(16384, 20000, 10, C.byref(o), C.byref(sz)) == capi.LP_OK
    assert capi.lp_workspace_size_csr(16385, 20000, 10, C.byref(o),
                                      C.byref(sz)) == capi.LP_ERR_SHAPE
    assert capi.lp_workspace_size_csr(64, 256, -1, C.byref(o), C.byref(sz)) == capi.LP_ERR_SHAPE
    assert capi.lp_workspace_size_csr(64, 256, 2 ** 31, C.byref(o),
                                      C.byref(sz)) == capi.LP_ERR_SHAPE
    assert capi.lp_workspace_size_csr(64, 64, 10, C.byref(o), C.byref(sz)) == capi.LP_ERR_SHAPE
    o.method = capi.LP_METHOD_PC
    assert capi.lp_workspace_size_csr(64, 256, 100, C.byref(o), C.byref(sz)) == capi.LP_OK
    o.method = capi.LP_METHOD_AFFINE
    for field, value in (("precision", capi.LP_PREC_MIXED), ("solver", capi.LP_SOLVER_WOODBURY),
                         ("tape_capacity", 2)):
        old = getattr(o, field)
        setattr(o, field, value)
        assert capi.lp_workspace_size_csr(64, 256, 100, C.byref(o),
                                          C.byref(sz)) == capi.LP_ERR_INVALID_ARG
        setattr(o, field, old)
    assert capi.lp_csr_workspace_size(64, 256, 100, C.byref(sz)) == capi.LP_OK
    assert capi.lp_csr_workspace_size(16385, 256, 100, C.byref(sz)) == capi.LP_ERR_SHAPE
    h = C.c_void_p()
    dummy = C.c_void_p(256)
    st = capi.lp_setup_csr(C.byref(h), 8, 16, 10, dummy, dummy, dummy, dummy, dummy, dummy,
                           dummy, dummy, C.byref(o), None, 0, None)
    assert st == capi.LP_ERR_WORKSPACE and not h.value


def test_batch_launch_options():
    """lp_options.batch_tile (0, 32, 64, 128) and batch_graph_iters (0..16) are
    validated by the single-LP and the batched workspace calls alike."""
    o = capi.lp_options()
    capi.lp_options_default(C.byref(o))
    assert o.batch_tile == 0 and o.batch_graph_iters == 0 and o.reserved2 == 0
    sz = C.c_size_t(0)
    m = (C.c_int64 * 2)(16, 20)
    n = (C.c_int64 * 2)(40, 60)
    for tile, g, ok in ((32, 1, True), (64, 16, True), (0, 0, True), (16, 0, False),
                        (128, 4, True), (256, 0, False), (96, 0, False), (32, 17, False),
                        (32, -1, False)):
        o.batch_tile, o.batch_graph_iters = tile, g
        want = capi.LP_OK if ok else capi.LP_ERR_INVALID_ARG
        assert capi.lp_batch_workspace_size(2, m, n, C.byref(o), C.byref(sz)) == want, (tile, g)
        assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == want, (tile, g)
    o.batch_tile, o.batch_graph_iters = 0, 0
    o.reserved2 = 1
    assert capi.lp_workspace_size(64, 256, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
    o.reserved2 = 0
    o.solver = capi.LP_SOLVER_WOODBURY
    assert capi.lp_batch_workspace_size(2, m, n, C.byref(o), C.byref(sz)) == capi.LP_ERR_INVALID_ARG
