"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and rejects invalid arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "genios.h")


@pytest.fixture(scope="module")
def abi():
    from paper_2310_08333_amd import _abi
    _abi.load()
    return _abi


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(genios_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(abi):
    lib = abi.load()
    names = _declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(abi.EXPORTED)


def test_struct_layouts_match(abi):
    sizes = [C.c_size_t(), C.c_size_t(), C.c_size_t()]
    abi.load().genios_abi_struct_sizes(*[C.byref(s) for s in sizes])
    assert tuple(s.value for s in sizes) == (C.sizeof(abi.Matrix), C.sizeof(abi.Opts),
                                             C.sizeof(abi.Info))


def test_default_opts_are_the_papers(abi):
    o = abi.default_opts()
    assert o.struct_size == C.sizeof(abi.Opts)
    assert o.sigma == 1e-6 and o.gamma == 1.2 and o.alpha == 1.6
    assert o.eps_abs == 1e-4 and o.eps_rel == 1e-4 and o.tau == 2.0 and o.mu == 10.0
    assert o.resketch_every == 20 and o.sketch_rank == 0 and o.rho_update_every == 25
    # Sec. 2.1's relative CG tolerance is taken against the warm-started initial residual
    assert o.rhs_relative == 0
    # a batch sharing one matrix uses the matrix-core products from 5 problems on
    assert o.batch_mfma == 1


def _mat(abi, m=100, n=200, lda=None, batch=1, dt=None):
    M = abi.Matrix()
    M.m, M.n, M.lda, M.batch = m, n, lda or n, batch
    M.stride_A = 0
    M.hi_dtype = abi.DT_F32 if dt is None else dt
    M.A_hi = 0x10000000  # never dereferenced: validation fails first
    return M


def test_workspace_sizes(abi):
    lib = abi.load()
    M = _mat(abi)
    o = abi.default_opts()
    for op in (abi.OP_LASSO, abi.OP_LOGREG, abi.OP_NYSTROM, abi.OP_BACKWARD, abi.OP_MATVEC,
               abi.OP_HUBER):
        assert lib.genios_workspace_size(op, C.byref(M), C.byref(o)) > 0
    assert lib.genios_workspace_size(99, C.byref(M), C.byref(o)) == 0
    # the BF16 copy lives in the workspace when the caller gives none
    o2 = abi.default_opts()
    o2.precision = abi.PREC_F32
    a = lib.genios_workspace_size(abi.OP_LASSO, C.byref(M), C.byref(o))
    b = lib.genios_workspace_size(abi.OP_LASSO, C.byref(M), C.byref(o2))
    assert a - b >= 100 * 200 * 2


def _solve(abi, M, o, lam=0.1, rho=1.0, ptrs=True):
    lib = abi.load()
    lam_a = (C.c_double * max(1, M.batch))(*([lam] * max(1, M.batch)))
    info = (abi.Info * max(1, M.batch))()
    p = 0x20000000 if ptrs else None
    return lib.genios_lasso_solve(C.byref(M), p, lam_a, rho, C.byref(o), p, p, p, info)


@pytest.mark.parametrize("field,value,code", [
    ("lda", 50, -2), ("m", 0, -2), ("batch", 0, -2), ("hi_dtype", 7, -1)])
def test_matrix_validation(abi, field, value, code):
    M = _mat(abi)
    setattr(M, field, value)
    o = abi.default_opts()
    assert _solve(abi, M, o) == code
    assert abi.last_error()


@pytest.mark.parametrize("field,value", [
    ("alpha", 2.5), ("alpha", 0.0), ("sigma", -1.0), ("gamma", 0.0), ("tau", 1.0), ("mu", 0.5),
    ("max_iter", 0), ("max_cg_iter", 0), ("cg_tol_floor", 0.0), ("sketch_rank", 129),
    ("resketch_every", 0), ("precision", 9), ("struct_size", 8), ("batch_mfma", 3),
    ("batch_mfma", -1)])
def test_option_validation(abi, field, value):
    o = abi.default_opts()
    setattr(o, field, value)
    assert _solve(abi, _mat(abi), o) == abi.ERR_ARG


def test_scalar_validation(abi):
    o = abi.default_opts()
    assert _solve(abi, _mat(abi), o, lam=-1.0) == abi.ERR_ARG
    assert _solve(abi, _mat(abi), o, lam=float("nan")) == abi.ERR_ARG
    assert _solve(abi, _mat(abi), o, rho=0.0) == abi.ERR_ARG
    assert _solve(abi, _mat(abi), o, ptrs=False) == abi.ERR_ARG


def test_precision_dtype_and_workspace(abi):
    o = abi.default_opts()
    o.precision = abi.PREC_F64
    assert _solve(abi, _mat(abi), o) == abi.ERR_ARG
    o = abi.default_opts()
    assert _solve(abi, _mat(abi, dt=abi.DT_F64), o) == abi.ERR_UNSUPPORTED
    o = abi.default_opts()  # no workspace
    assert _solve(abi, _mat(abi), o) == abi.ERR_WORKSPACE
    o.workspace, o.workspace_bytes = 0x30000000, 1024  # too small
    assert _solve(abi, _mat(abi), o) == abi.ERR_WORKSPACE
    o.workspace, o.workspace_bytes = 0x30000001, 1 << 40  # misaligned
    assert _solve(abi, _mat(abi), o) == abi.ERR_WORKSPACE


def test_nystrom_and_apply_validation(abi):
    lib = abi.load()
    M = _mat(abi, 30, 40)
    o = abi.default_opts()
    info = (abi.Info * 1)()
    p = 0x20000000
    assert lib.genios_nystrom_build(C.byref(M), None, 0, None, C.byref(o), p, p, info) == abi.ERR_ARG
    assert lib.genios_nystrom_build(C.byref(M), None, 41, None, C.byref(o), p, p, info) == abi.ERR_ARG
    assert lib.genios_nystrom_apply(10, 20, 1, abi.DT_F32, p, p, 1.0, p, p, C.byref(o)) == abi.ERR_SHAPE
    assert lib.genios_nystrom_apply(100, 20, 1, abi.DT_F32, p, p, 0.0, p, p, C.byref(o)) == abi.ERR_ARG
    assert lib.genios_nystrom_apply(100, 20, 1, abi.DT_F32, p, p, 1.0, p, p, C.byref(o)) == abi.ERR_WORKSPACE
    assert lib.genios_admm_update(0, abi.DT_F32, 1.6, 0.1, p, p, p, None, C.byref(o)) == abi.ERR_SHAPE
    assert lib.genios_matvec(C.byref(M), 2, 0, p, p, C.byref(o)) == abi.ERR_ARG
    assert lib.genios_matvec(C.byref(M), 0, 1, p, p, C.byref(o)) == abi.ERR_ARG  # no BF16 copy


def test_status_strings(abi):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7):
        assert abi.status_string(code) != "unknown status"


def test_stream_read_rejects_bad_arguments_before_any_device_call(abi):
    lib = abi.load()
    o = abi.default_opts()
    sec = C.c_double(0.0)
    dummy = C.c_void_p(16)  # never dereferenced: the checks come first
    assert lib.genios_stream_read(dummy, 15, 1, dummy, C.byref(sec), C.byref(o)) == abi.ERR_SHAPE
    assert lib.genios_stream_read(C.c_void_p(8), 32, 1, dummy, C.byref(sec), C.byref(o)) == abi.ERR_SHAPE
    assert lib.genios_stream_read(dummy, 32, 0, dummy, C.byref(sec), C.byref(o)) == abi.ERR_ARG
    assert lib.genios_stream_read(None, 32, 1, dummy, C.byref(sec), C.byref(o)) == abi.ERR_ARG


def test_termination_options_defaults_and_checks(abi):
    o = abi.default_opts()
    assert o.termination == 0 and o.gap_every == 1 and o.eps_gap == 1e-4
    lib = abi.load()
    M = abi.Matrix()
    M.m, M.n, M.lda, M.batch = 4, 8, 8, 1
    M.hi_dtype = abi.DT_F32
    M.A_hi = C.c_void_p(16)  # never dereferenced: the option checks come first
    lam = (C.c_double * 1)(0.1)
    info = (abi.Info * 1)()
    for field, bad in (("termination", 3), ("termination", -1), ("gap_every", 0), ("eps_gap", 0.0)):
        q = abi.default_opts()
        setattr(q, field, bad)
        rc = lib.genios_lasso_solve(C.byref(M), C.c_void_p(16), lam, 1.0, C.byref(q),
                                    C.c_void_p(16), C.c_void_p(16), C.c_void_p(16), info)
        assert rc == abi.ERR_ARG, (field, rc)


def test_huber_entry_point_checks_its_arguments(abi):
    o = abi.default_opts()
    assert o.huber_delta == 1.0  # the loss of Sec. 4.3
    lib = abi.load()
    M = _mat(abi)
    lam = (C.c_double * 1)(0.1)
    info = (abi.Info * 1)()
    p = C.c_void_p(0x20000000)  # never dereferenced: the argument checks come first
    for bad in (0.0, -1.0, float("inf"), float("nan")):
        q = abi.default_opts()
        q.huber_delta = bad
        assert lib.genios_huber_solve(C.byref(M), p, lam, 1.0, C.byref(q), p, p, p, info) == abi.ERR_ARG
    q = abi.default_opts()
    assert lib.genios_huber_solve(C.byref(M), None, lam, 1.0, C.byref(q), p, p, p, info) == abi.ERR_ARG
    assert lib.genios_huber_solve(C.byref(M), p, lam, 1.0, C.byref(q), p, p, p, info) == abi.ERR_WORKSPACE
    # the Huber path carries the curvature vector and two right-hand columns like the logistic one
    a = lib.genios_workspace_size(abi.OP_HUBER, C.byref(M), C.byref(q))
    b = lib.genios_workspace_size(abi.OP_LOGREG, C.byref(M), C.byref(q))
    assert a == b > 0


def test_adaptive_sketch_options_defaults_and_checks(abi):
    o = abi.default_opts()
    assert o.adaptive_sketch == 0 and o.sketch_rank_init == 8 and o.sketch_kappa == 10.0
    assert o.power_iters == 10
    M = _mat(abi)
    for field, bad in (("adaptive_sketch", 2), ("sketch_rank_init", 0), ("sketch_kappa", 1.0),
                       ("sketch_kappa", float("nan")), ("power_iters", 0), ("power_iters", 1001)):
        q = abi.default_opts()
        setattr(q, field, bad)
        assert _solve(abi, M, q) == abi.ERR_ARG, field


def test_boxls_entry_point_checks_its_arguments(abi):
    lib = abi.load()
    M = _mat(abi)
    info = (abi.Info * 1)()
    p = C.c_void_p(0x20000000)  # never dereferenced: the argument checks come first
    q = abi.default_opts()
    assert lib.genios_boxls_solve(C.byref(M), None, None, None, 1.0, C.byref(q), p, p, p, info) == abi.ERR_ARG
    assert lib.genios_boxls_solve(C.byref(M), p, None, None, 0.0, C.byref(q), p, p, p, info) == abi.ERR_ARG
    q.lambda2 = 0.5
    assert lib.genios_boxls_solve(C.byref(M), p, None, None, 1.0, C.byref(q), p, p, p, info) == abi.ERR_UNSUPPORTED
    q = abi.default_opts()
    assert lib.genios_boxls_solve(C.byref(M), p, p, p, 1.0, C.byref(q), p, p, p, info) == abi.ERR_WORKSPACE
    a = lib.genios_workspace_size(abi.OP_BOXLS, C.byref(M), C.byref(q))
    assert a == lib.genios_workspace_size(abi.OP_LASSO, C.byref(M), C.byref(q)) > 0


def test_hvp_noalloc_rejects_a_product_beyond_its_scratch(abi):
    # 20000 x 200000: the fused product's partial slots alone exceed the static
    # scratch; the call must fail on the host, before any HIP call
    lib = abi.load()
    M = _mat(abi, m=20000, n=200000)
    o = abi.default_opts()
    o.precision = abi.PREC_F32
    need = lib.genios_workspace_size(abi.OP_HVP, C.byref(M), C.byref(o))
    assert need > (128 << 20)
    rc = lib.genios_hvp_noalloc(C.byref(M), 0, None, C.c_void_p(0x20000000),
                                C.c_void_p(0x30000000), C.byref(o))
    assert rc == abi.ERR_WORKSPACE
    assert b"scratch" in lib.genios_last_error()
    # and a size within the buffer passes the same check (not called: no device here)
    M2 = _mat(abi, m=20000, n=40000)
    assert lib.genios_workspace_size(abi.OP_HVP, C.byref(M2), C.byref(o)) <= (128 << 20)


def test_refine_cg_option_is_validated(abi):
    lib = abi.load()
    o = abi.default_opts()
    assert o.refine_cg_bf16 == -1  # automatic: BF16 CG products for large master copies
    o.refine_cg_bf16 = 2
    M = _mat(abi)
    rc = lib.genios_lasso_solve(C.byref(M), C.c_void_p(0x1000), (C.c_double * 1)(0.1), 1.0,
                                C.byref(o), C.c_void_p(0x2000), C.c_void_p(0x3000),
                                C.c_void_p(0x4000), (abi.Info * 1)())
    assert rc == abi.ERR_ARG
