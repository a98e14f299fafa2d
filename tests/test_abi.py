"""The C-ABI library loads without a GPU and exports every function that
include/mgwd.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mgwd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_boundary():
    names = declared_functions()
    for n in ("wilson_apply", "mg_setup", "mg_restrict", "mg_prolong", "coarse_apply", "mg_solve",
              "mg_destroy", "mg_last_error"):
        assert n in names


def test_library_exports_all_symbols():
    import paper_1005_3043_amd as mgwd
    lib = ctypes.CDLL(mgwd.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(mgwd.EXPORTED) == sorted(declared_functions())


def test_argument_errors_without_gpu():
    """Host-side argument validation returns error codes, never aborts."""
    import paper_1005_3043_amd as mgwd
    lib = mgwd.lib()
    lat = mgwd.lattice((4, 4, 4, 0))
    rc = lib.wilson_apply(ctypes.byref(lat), None, 0.0, None, None, 1, 0, None)
    assert rc == -1
    assert b"positive" in lib.mg_last_error()
    lat = mgwd.lattice((4, 4, 4, 4))
    rc = lib.wilson_apply(ctypes.byref(lat), None, 0.0, None, None, 1, 0, None)
    assert rc == -1


def test_setup_parameter_errors_without_gpu():
    """mg_setup rejects bad setup-refinement parameters on the host, before
    any device work (the dummy pointers are never dereferenced)."""
    import paper_1005_3043_amd as mgwd
    lib = mgwd.lib()
    lat = mgwd.lattice((8, 8, 8, 8))

    def params(group, iters):
        p = mgwd.Params()
        p.n_levels = 2
        for mu in range(4):
            p.block[0][mu] = 4
        p.nv[0] = 4
        p.setup_rounds, p.setup_mr_steps, p.omega, p.pre, p.post = 5, 4, 0.9, 4, 4
        p.coarse_tol, p.coarse_maxiter, p.gcr_restart, p.max_iter = 1e-3, 1000, 8, 100
        p.precond_prec, p.max_rhs, p.use_graph = 0, 1, 1
        p.init_vectors[0] = 1
        p.refine_group, p.refine_iters = group, iters
        return p
    h = ctypes.c_void_p()
    for group, iters, msg in ((4, 5, b"refine_group"), (-1, 5, b"refine_group"), (17, 5, b"refine_group"),
                              (2, 9, b"refine_iters"), (2, -1, b"refine_iters")):
        p = params(group, iters)
        rc = lib.mg_setup(ctypes.byref(lat), ctypes.c_void_p(1), -0.3, ctypes.byref(p), ctypes.byref(h), None)
        assert rc == -1 and msg in lib.mg_last_error(), (group, iters, lib.mg_last_error())
    # a transfer storage outside MG_F64..MG_F16 is refused the same way
    p = params(0, 5)
    p.transfer_prec = 7
    rc = lib.mg_setup(ctypes.byref(lat), ctypes.c_void_p(1), -0.3, ctypes.byref(p), ctypes.byref(h), None)
    assert rc == -6 and b"transfer_prec" in lib.mg_last_error(), lib.mg_last_error()  # MG_ENOTSUP
