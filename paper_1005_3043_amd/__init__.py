"""Python binding of libmgwd: the MI355X adaptive multigrid Wilson-Dirac solver.

Argument marshalling only: every step of the computation runs in the HIP
library behind the C ABI declared in include/mgwd.h.  PyTorch supplies device
memory (complex128 CUDA/HIP tensors) and the current stream.  If the shared
library is missing or cannot be loaded the functions raise; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import sys
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgwd.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
MAX_LEVELS = 3
MAX_RHS = 16

EXPORTED = ["wilson_apply", "wilson_apply_noalloc", "mg_setup", "mg_set_precond_prec", "mg_set_mass", "mg_set_timing", "mg_restrict",
            "mg_prolong", "coarse_apply", "mg_apply_op", "mg_vcycle", "mg_transfer", "mg_set_transfer_variant", "mg_transfer_variant", "mg_set_coarse_variant", "mg_coarse_variant", "mg_set_cgnr_persistent", "mg_set_gcr_fusion", "mg_coarse_solve", "mg_solve", "mg_time_dslash", "mg_time_dslash_mrq", "mg_time_coarse",
            "mg_destroy", "mg_release_cached_memory", "mg_last_error", "mg_export_maps", "mg_export_P",
            "mg_export_coarse_op", "mg_export_nullvecs", "mg_level_info",
            "ptc_create", "ptc_set_links", "ptc_set_targets", "ptc_forward", "ptc_loss_grad", "ptc_adam",
            "ptc_destroy"]


class MGError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__(f"mgwd error {rc}: {msg}")
        self.rc = rc


class Lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("t_antiperiodic", ctypes.c_int)]


class Params(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int),
                ("block", (ctypes.c_int * 4) * (MAX_LEVELS - 1)),
                ("nv", ctypes.c_int * (MAX_LEVELS - 1)),
                ("setup_rounds", ctypes.c_int),
                ("setup_mr_steps", ctypes.c_int),
                ("omega", ctypes.c_double),
                ("pre", ctypes.c_int), ("post", ctypes.c_int),
                ("coarse_tol", ctypes.c_double),
                ("coarse_maxiter", ctypes.c_int),
                ("gcr_restart", ctypes.c_int),
                ("max_iter", ctypes.c_int),
                ("precond_prec", ctypes.c_int),
                ("max_rhs", ctypes.c_int),
                ("use_graph", ctypes.c_int),
                ("init_vectors", ctypes.c_void_p * (MAX_LEVELS - 1)),
                ("refine_group", ctypes.c_int), ("refine_iters", ctypes.c_int),
                ("smoother", ctypes.c_int), ("cycles", ctypes.c_int),
                ("setup_prec", ctypes.c_int),
                ("learned_setup", ctypes.c_int), ("ptc_hidden", ctypes.c_int),
                ("ptc_weights", ctypes.c_void_p * 2),
                ("transfer_prec", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int * MAX_RHS),
                ("rel_resid", ctypes.c_double * MAX_RHS),
                ("n_fine_dslash", ctypes.c_int),
                ("n_coarse_apply", ctypes.c_int),
                ("n_coarse_dispatch", ctypes.c_int),
                ("n_cgnr_iters", ctypes.c_int),
                ("n_vcycles", ctypes.c_int),
                ("t_setup_s", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * 10),
                ("kernel_launches", ctypes.c_int * 10),
                ("kernel_sites", ctypes.c_double * 10),
                ("n_cgnr_fallbacks", ctypes.c_int)]

    KERNELS = ("dslash_f64", "coarse_f64", "dslash_f32", "coarse_f32", "dslash_f16", "coarse_f16", "cgnr_f32",
               "cgnr_f16", "dslash_mrq_f32", "dslash_mrq_f16")

    def as_dict(self, nrhs=1):
        return dict(iters=list(self.iters[:nrhs]), rel_resid=list(self.rel_resid[:nrhs]),
                    n_fine_dslash=self.n_fine_dslash, n_coarse_apply=self.n_coarse_apply,
                    n_coarse_dispatch=self.n_coarse_dispatch,
                    n_cgnr_iters=self.n_cgnr_iters, n_vcycles=self.n_vcycles,
                    n_cgnr_fallbacks=self.n_cgnr_fallbacks,
                    t_setup_s=self.t_setup_s, t_solve_s=self.t_solve_s,
                    kernels={k: dict(ms=self.kernel_ms[i], launches=self.kernel_launches[i],
                                     sites=self.kernel_sites[i]) for i, k in enumerate(self.KERNELS)})


_lib = None


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1005_3043_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sig = {
            "wilson_apply": [ctypes.POINTER(Lattice), vp, cd, vp, vp, ci, ci, vp],
            "wilson_apply_noalloc": [ctypes.POINTER(Lattice), vp, cd, vp, vp, ci, ci, vp],
            "mg_setup": [ctypes.POINTER(Lattice), vp, cd, ctypes.POINTER(Params), ctypes.POINTER(vp), vp],
            "mg_set_precond_prec": [vp, ci],
            "mg_set_mass": [vp, cd],
            "mg_set_timing": [vp, ci],
            "mg_restrict": [vp, ci, vp, vp, ci, vp],
            "mg_prolong": [vp, ci, vp, vp, ci, vp],
            "coarse_apply": [vp, ci, vp, vp, ci, ci, vp],
            "mg_apply_op": [vp, ci, ci, vp, vp, ci, vp],
            "mg_vcycle": [vp, ci, vp, vp, ci, ctypes.POINTER(ci), vp],
            "mg_transfer": [vp, ci, ci, ci, vp, vp, ci, vp],
            "mg_set_transfer_variant": [vp, ci],
            "mg_transfer_variant": [vp, ci, ci, ctypes.POINTER(ci), ctypes.POINTER(ci), ctypes.POINTER(cd)],
            "mg_set_coarse_variant": [vp, ci],
            "mg_set_cgnr_persistent": [vp, ci],
            "mg_set_gcr_fusion": [vp, ci],
            "mg_coarse_variant": [vp, ci, ci, ci, ctypes.POINTER(ci), ctypes.POINTER(cd)],
            "mg_coarse_solve": [vp, ci, vp, vp, ci, ctypes.POINTER(ci), vp],
            "mg_solve": [vp, vp, vp, ci, cd, ctypes.POINTER(Info), vp],
            "mg_time_dslash": [vp, ci, ci, ci, ctypes.POINTER(cd), vp],
            "mg_time_dslash_mrq": [vp, ci, ci, ci, ctypes.POINTER(cd), vp],
            "mg_time_coarse": [vp, ci, ci, ci, ci, ctypes.POINTER(cd), vp],
            "mg_destroy": [vp],
            "mg_release_cached_memory": [ctypes.POINTER(ctypes.c_size_t)],
            "mg_last_error": [],
            "mg_export_maps": [vp, ci, vp, vp, vp, vp],
            "mg_export_P": [vp, ci, vp],
            "mg_export_coarse_op": [vp, ci, vp, vp],
            "mg_export_nullvecs": [vp, ci, vp],
            "mg_level_info": [vp, ci, vp, vp],
            "ptc_create": [ctypes.POINTER(Lattice), ctypes.POINTER(ci), ci, ci, ctypes.POINTER(vp)],
            "ptc_set_links": [vp, vp, vp],
            "ptc_set_targets": [vp, vp, ci, vp],
            "ptc_forward": [vp, vp, vp, vp, vp, vp],
            "ptc_loss_grad": [vp, vp, vp, vp, ctypes.POINTER(cd), vp, vp, vp],
            "ptc_adam": [vp, vp, vp, vp, ctypes.c_size_t, ci, cd, cd, cd, cd, vp],
            "ptc_destroy": [vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_char_p if name == "mg_last_error" else ctypes.c_int
        _lib = L
    return _lib


def _check(rc, allow_not_converged=False):
    if rc == MG_OK or (allow_not_converged and rc == MG_NOT_CONVERGED):
        return rc
    raise MGError(rc, lib().mg_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex128 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def lattice(L, t_antiperiodic=True) -> Lattice:
    return Lattice((ctypes.c_int * 4)(*[int(v) for v in L]), int(bool(t_antiperiodic)))


def dims_of_spinor(psi: torch.Tensor):
    Lt, Lz, Ly, Lx = psi.shape[-6:-2]
    return (Lx, Ly, Lz, Lt)


def release_cached_memory() -> int:
    """Frees the library's cache of device allocations on the current device
    (buffers of destroyed contexts kept for reuse); returns the bytes freed."""
    n = ctypes.c_size_t(0)
    _check(lib().mg_release_cached_memory(ctypes.byref(n)))
    return int(n.value)


def wilson_apply(U: torch.Tensor, psi: torch.Tensor, mass: float, prec: str = "f64",
                 t_antiperiodic: bool = True, out: torch.Tensor | None = None) -> torch.Tensor:
    """out = D(U) psi (Eq. 2) for psi[..., t, z, y, x, 4, 3] (leading axes = RHS)."""
    L = dims_of_spinor(psi)
    nrhs = int(psi.numel() // (12 * L[0] * L[1] * L[2] * L[3]))
    if out is None:
        out = torch.empty_like(psi)
    lat = lattice(L, t_antiperiodic)
    _check(lib().wilson_apply(ctypes.byref(lat), _dev(U, "U"), float(mass), _dev(psi, "psi"),
                              _dev(out, "out"), nrhs, PREC[prec], _stream()))
    return out


def wilson_apply_noalloc(U: torch.Tensor, psi: torch.Tensor, mass: float, out: torch.Tensor, prec: str = "f64",
                         t_antiperiodic: bool = True) -> torch.Tensor:
    """wilson_apply through the entry point that allocates nothing (the
    caller passes out; the library's fixed scratch holds the internal
    layouts)."""
    L = dims_of_spinor(psi)
    nrhs = int(psi.numel() // (12 * L[0] * L[1] * L[2] * L[3]))
    lat = lattice(L, t_antiperiodic)
    _check(lib().wilson_apply_noalloc(ctypes.byref(lat), _dev(U, "U"), float(mass), _dev(psi, "psi"),
                                      _dev(out, "out"), nrhs, PREC[prec], _stream()))
    return out


class MG:
    """Owning handle of an mg_ctx_t (setup done on construction)."""

    def __init__(self, U: torch.Tensor, mass: float, blocks, nv, init_vectors, *,
                 t_antiperiodic=True, setup_rounds=5, setup_mr_steps=4, omega=0.9, pre=4,
                 post=4, coarse_tol=1e-3, coarse_maxiter=1000, gcr_restart=8, max_iter=10000,
                 precond_prec="f64", max_rhs=1, use_graph=True, refine_group=0, refine_iters=5,
                 smoother="mr", cycles=1, setup_prec="f64", learned=None, transfer_prec="f64"):
        """learned = (W1, W2, n_hidden): the level-0 start vectors are the
        network's output for the noise field init_vectors[0] (one field),
        computed inside mg_setup."""
        Lt, Lz, Ly, Lx = U.shape[1:5]
        self.L = (Lx, Ly, Lz, Lt)
        self.nv = list(nv)
        self.blocks = [tuple(b) for b in blocks]
        p = Params()
        p.n_levels = len(blocks) + 1
        for i, b in enumerate(blocks):
            for mu in range(4):
                p.block[i][mu] = int(b[mu])
            p.nv[i] = int(nv[i])
        p.setup_rounds, p.setup_mr_steps, p.omega = setup_rounds, setup_mr_steps, omega
        p.pre, p.post, p.coarse_tol, p.coarse_maxiter = pre, post, coarse_tol, coarse_maxiter
        p.gcr_restart, p.max_iter = gcr_restart, max_iter
        p.precond_prec, p.max_rhs, p.use_graph = PREC[precond_prec], max_rhs, int(bool(use_graph))
        p.refine_group, p.refine_iters = int(refine_group), int(refine_iters)
        p.smoother, p.cycles = {"mr": 0, "gmres": 1}[smoother], int(cycles)
        p.setup_prec = PREC[setup_prec]
        p.transfer_prec = transfer_prec if isinstance(transfer_prec, int) else PREC[transfer_prec]
        self._keep = list(init_vectors)
        if learned is not None:
            W1, W2, n_hidden = learned
            p.learned_setup, p.ptc_hidden = 1, int(n_hidden)
            p.ptc_weights[0] = _dev64(W1, "W1").value
            p.ptc_weights[1] = _dev64(W2, "W2").value
            self._keep += [W1, W2]
        for i, v in enumerate(init_vectors):
            p.init_vectors[i] = _dev(v, f"init_vectors[{i}]").value
        self.params = p
        lat = lattice(self.L, t_antiperiodic)
        h = ctypes.c_void_p()
        _check(lib().mg_setup(ctypes.byref(lat), _dev(U, "U"), float(mass), ctypes.byref(p),
                              ctypes.byref(h), _stream()))
        self.ctx = h
        self._keep = None

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime (and a profiler's hooks) may
        # already be torn down: a handle still open then is left to process
        # exit, which frees device memory anyway.  close() is the teardown.
        # (The check is bound at definition: module globals such as sys may
        # already be cleared when this runs.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def level_info(self, level):
        L = (ctypes.c_int * 4)()
        n = ctypes.c_int()
        _check(lib().mg_level_info(self.ctx, level, L, ctypes.byref(n)))
        return tuple(L), n.value

    def set_precond_prec(self, prec: str):
        _check(lib().mg_set_precond_prec(self.ctx, PREC[prec]))

    def set_mass(self, mass: float):
        """Shift the setup to another mass (exact: X += (m' - m) I on every level)."""
        _check(lib().mg_set_mass(self.ctx, float(mass)))
        self.mass = float(mass)

    def set_timing(self, on: bool):
        _check(lib().mg_set_timing(self.ctx, int(bool(on))))

    def restrict(self, level, fine, nrhs=None):
        Lc, n = self.level_info(level + 1)
        if nrhs is None:
            nrhs = self._nvec(level, fine)
        out = torch.empty((nrhs, Lc[3], Lc[2], Lc[1], Lc[0], n), dtype=torch.complex128, device=fine.device)
        _check(lib().mg_restrict(self.ctx, level, _dev(fine, "fine"), _dev(out, "coarse"), nrhs, _stream()))
        return out

    def prolong(self, level, coarse, nrhs=None):
        Lf, n = self.level_info(level)
        if nrhs is None:
            nrhs = self._nvec(level + 1, coarse)
        shape = (nrhs, Lf[3], Lf[2], Lf[1], Lf[0]) + ((4, 3) if level == 0 else (n,))
        out = torch.empty(shape, dtype=torch.complex128, device=coarse.device)
        _check(lib().mg_prolong(self.ctx, level, _dev(coarse, "coarse"), _dev(out, "fine"), nrhs, _stream()))
        return out

    def coarse_apply(self, level, v, dagger=False, nrhs=None):
        if nrhs is None:
            nrhs = self._nvec(level, v)
        out = torch.empty_like(v)
        _check(lib().coarse_apply(self.ctx, level, _dev(v, "in"), _dev(out, "out"), nrhs, int(bool(dagger)),
                                  _stream()))
        return out

    def apply_op(self, level, v, prec="f64", nrhs=None):
        """Level operator (fine Wilson D at level 0, D_c above) with the stored
        copies of precision `prec`; canonical complex128 in and out."""
        if nrhs is None:
            nrhs = self._nvec(level, v)
        out = torch.empty_like(v)
        _check(lib().mg_apply_op(self.ctx, level, PREC[prec], _dev(v, "in"), _dev(out, "out"), nrhs, _stream()))
        return out

    def vcycle(self, r, prec="f64"):
        """One preconditioner application z = K(r) on canonical fine spinors
        (complex128, [nrhs] + lattice shape or one spinor); returns (z, summed
        coarsest-level CGNR iterations)."""
        nrhs = self._nvec(0, r)
        out = torch.empty_like(r)
        it = ctypes.c_int(0)
        _check(lib().mg_vcycle(self.ctx, PREC[prec], _dev(r, "in"), _dev(out, "out"), nrhs, ctypes.byref(it),
                               _stream()))
        return out, it.value

    def transfer(self, level, v, direction, prec="f64", nrhs=None):
        """Restriction (direction 0, level -> level+1) or prolongation
        (direction 1, level+1 -> level) with the stored P of precision
        `prec`; canonical complex128 in and out."""
        lin, lout = (level, level + 1) if direction == 0 else (level + 1, level)
        if nrhs is None:
            nrhs = self._nvec(lin, v)
        Lo, no = self.level_info(lout)
        shape = (nrhs, Lo[3], Lo[2], Lo[1], Lo[0]) + ((4, 3) if lout == 0 else (no,))
        out = torch.empty(shape, dtype=torch.complex128, device=v.device)
        _check(lib().mg_transfer(self.ctx, level, PREC[prec], direction, _dev(v, "in"), _dev(out, "out"), nrhs,
                                 _stream()))
        return out

    def set_transfer_variant(self, variant):
        """Force the fine-level transfer kernels (0 vector, 1 matrix-core GEMM)
        or restore tuning (-1)."""
        _check(lib().mg_set_transfer_variant(self.ctx, int(variant)))

    def transfer_variant(self, prec, nrhs):
        """(restriction, prolongation) kernel choices for `prec` and nrhs and
        the tuning times {(direction, variant): us}."""
        r, p = ctypes.c_int(0), ctypes.c_int(0)
        us = (ctypes.c_double * 4)()
        _check(lib().mg_transfer_variant(self.ctx, PREC[prec], int(nrhs), ctypes.byref(r), ctypes.byref(p), us))
        return r.value, p.value, {("restrict", 0): us[0], ("restrict", 1): us[1], ("prolong", 0): us[2],
                                  ("prolong", 1): us[3]}

    def set_coarse_variant(self, variant):
        """Force the coarse-stencil kernel (0 per-RHS, 1/2/4 matrix-core GEMM
        with that K split) or restore autotuning (-1)."""
        _check(lib().mg_set_coarse_variant(self.ctx, int(variant)))

    def set_gcr_fusion(self, mode: int):
        """Outer FGCR step: 1 (default) orthogonalisation and residual update
        in one pass, 0 two passes, 2 the fused pass with every step taking
        the second pass (the fallback where the norm estimate cancels)."""
        _check(lib().mg_set_gcr_fusion(self.ctx, int(mode)))

    def set_cgnr_persistent(self, on, polls=None):
        """Single-RHS coarsest CGNR as one cooperative launch (True, default)
        or as chunks of per-iteration launches (False); same arithmetic.
        polls (>= 2): barrier polls before a wait gives up (default 2^20)."""
        _check(lib().mg_set_cgnr_persistent(self.ctx, (int(polls) if polls else 1) if on else 0))

    def coarse_variant(self, level=1, prec="f32", nrhs=1):
        v, us = ctypes.c_int(), ctypes.c_double()
        _check(lib().mg_coarse_variant(self.ctx, level, PREC[prec], nrhs, ctypes.byref(v), ctypes.byref(us)))
        return v.value, us.value

    def coarse_solve(self, b, prec="f64", nrhs=None):
        """The cycle's coarsest-level CGNR on canonical coarsest-level vectors
        (complex128); returns (x, CGNR iterations per right-hand side)."""
        lc = len(self.nv)
        if nrhs is None:
            nrhs = self._nvec(lc, b)
        x = torch.empty_like(b)
        it = (ctypes.c_int * nrhs)()
        _check(lib().mg_coarse_solve(self.ctx, PREC[prec], _dev(b, "b"), _dev(x, "x"), nrhs, it, _stream()))
        return x, list(it)

    def solve(self, b, tol=1e-10, nrhs=None, x=None):
        if nrhs is None:
            nrhs = self._nvec(0, b)
        if x is None:
            x = torch.empty_like(b)
        info = Info()
        rc = _check(lib().mg_solve(self.ctx, _dev(b, "b"), _dev(x, "x"), nrhs, float(tol), ctypes.byref(info),
                                   _stream()), allow_not_converged=True)
        return x, info.as_dict(nrhs), rc

    def time_dslash(self, prec="f64", nrhs=1, reps=20):
        ms = ctypes.c_double()
        _check(lib().mg_time_dslash(self.ctx, PREC[prec], nrhs, reps, ctypes.byref(ms), _stream()))
        return ms.value

    def time_dslash_mrq(self, prec="f32", nrhs=12, reps=20):
        """Mean device time (ms) of the fine stencil in the form the MR steps
        of the FP32 / FP16-class V-cycle launch (q recursion)."""
        ms = ctypes.c_double()
        _check(lib().mg_time_dslash_mrq(self.ctx, PREC[prec], nrhs, reps, ctypes.byref(ms), _stream()))
        return ms.value

    def time_coarse(self, level=1, prec="f64", nrhs=1, reps=20):
        ms = ctypes.c_double()
        _check(lib().mg_time_coarse(self.ctx, level, PREC[prec], nrhs, reps, ctypes.byref(ms), _stream()))
        return ms.value

    def _nvec(self, level, t):
        L, n = self.level_info(level)
        per = L[0] * L[1] * L[2] * L[3] * n
        return int(t.numel() // per)

    # parity exports --------------------------------------------------------
    def export_maps(self, level):
        import numpy as np
        L, _ = self.level_info(level)
        Lc, _ = self.level_info(level + 1)
        V = L[0] * L[1] * L[2] * L[3]
        Vc = Lc[0] * Lc[1] * Lc[2] * Lc[3]
        f2c = np.zeros(V, np.int32)
        f2l = np.zeros(V, np.int32)
        nbr = np.zeros((Vc, 8), np.int32)
        face = np.zeros(V, np.int32)
        p = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
        _check(lib().mg_export_maps(self.ctx, level, p(f2c), p(f2l), p(nbr), p(face)))
        return f2c, f2l, nbr, face

    def export_P(self, level):
        import numpy as np
        Lc, n_c = self.level_info(level + 1)
        L, n = self.level_info(level)
        nv = n_c // 2
        vb = 1
        for mu in range(4):
            vb *= self.blocks[level][mu]
        Vc = Lc[0] * Lc[1] * Lc[2] * Lc[3]
        P = np.zeros((Vc, 2, vb * n // 2, nv), np.complex128)
        _check(lib().mg_export_P(self.ctx, level, ctypes.c_void_p(P.ctypes.data)))
        return P

    def export_coarse_op(self, level):
        import numpy as np
        Lc, n = self.level_info(level)
        X = np.zeros((Lc[3], Lc[2], Lc[1], Lc[0], n, n), np.complex128)
        Y = np.zeros((8, Lc[3], Lc[2], Lc[1], Lc[0], n, n), np.complex128)
        _check(lib().mg_export_coarse_op(self.ctx, level, ctypes.c_void_p(X.ctypes.data),
                                         ctypes.c_void_p(Y.ctypes.data)))
        return X, Y

    def export_nullvecs(self, level):
        import numpy as np
        L, n = self.level_info(level)
        nv = self.nv[level]
        shape = (nv, L[3], L[2], L[1], L[0]) + ((4, 3) if level == 0 else (n,))
        V = np.zeros(shape, np.complex128)
        _check(lib().mg_export_nullvecs(self.ctx, level, ctypes.c_void_p(V.ctypes.data)))
        return V


def _dev64(t: torch.Tensor, name: str):
    if not (t.is_cuda and t.dtype == torch.complex64 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous complex64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


class PTC:
    """Owning handle of a ptc_ctx_t: the parallel-transport network that
    proposes near-null vectors (weights complex64 [c_out][c_in][9][4][4])."""

    def __init__(self, L, block, n_hidden=8, n_out=24, t_antiperiodic=True):
        self.L = tuple(int(v) for v in L)
        self.n_hidden, self.n_out = int(n_hidden), int(n_out)
        lat = lattice(self.L, t_antiperiodic)
        h = ctypes.c_void_p()
        _check(lib().ptc_create(ctypes.byref(lat), (ctypes.c_int * 4)(*[int(b) for b in block]), self.n_hidden,
                                self.n_out, ctypes.byref(h)))
        self.ctx = h

    def close(self):
        if getattr(self, "ctx", None):
            lib().ptc_destroy(self.ctx)
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # At interpreter shutdown the HIP runtime (and a profiler's hooks) may
        # already be torn down: a handle still open then is left to process
        # exit, which frees device memory anyway.  close() is the teardown.
        # (The check is bound at definition: module globals such as sys may
        # already be cleared when this runs.)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def set_links(self, U):
        _check(lib().ptc_set_links(self.ctx, _dev(U, "U"), _stream()))

    def set_targets(self, V):
        nv = int(V.shape[0])
        _check(lib().ptc_set_targets(self.ctx, _dev(V, "V"), nv, _stream()))

    def forward(self, W1, W2, eta):
        Lx, Ly, Lz, Lt = self.L
        Y = torch.empty((self.n_out, Lt, Lz, Ly, Lx, 4, 3), dtype=torch.complex128, device=eta.device)
        _check(lib().ptc_forward(self.ctx, _dev64(W1, "W1"), _dev64(W2, "W2"), _dev(eta, "eta"), _dev(Y, "Y"),
                                 _stream()))
        return Y

    def loss_grad(self, W1, W2, eta):
        g1, g2 = torch.empty_like(W1), torch.empty_like(W2)
        loss = ctypes.c_double()
        _check(lib().ptc_loss_grad(self.ctx, _dev64(W1, "W1"), _dev64(W2, "W2"), _dev(eta, "eta"),
                                   ctypes.byref(loss), _dev64(g1, "gW1"), _dev64(g2, "gW2"), _stream()))
        return loss.value, g1, g2


def ptc_adam(W, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam step on complex64 W with moments m (complex64) and v
    (float32, 2 entries per parameter)."""
    if not (v.is_cuda and v.dtype == torch.float32 and v.numel() == 2 * W.numel()):
        raise ValueError("v must be a float32 device tensor with 2 entries per parameter")
    _check(lib().ptc_adam(_dev64(W, "W"), _dev64(g, "g"), _dev64(m, "m"), ctypes.c_void_p(v.data_ptr()),
                          W.numel(), int(step), float(lr), float(b1), float(b2), float(eps), _stream()))
