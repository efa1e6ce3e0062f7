"""Python binding of the C-ABI in ``include/fe.h`` (argument marshalling only).

Arrays are torch tensors on the GPU; their device pointers and torch's current
HIP stream are handed to the library, which does all of the work in its own
kernels.  Nothing here computes any part of the method, and nothing falls back
to the CPU: if ``libfe_hip.so`` is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch  # loaded first: the library then shares torch's HIP runtime

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfe_hip.so")

FE_OK, FE_PENDING, FE_NOT_CONVERGED = 0, 1, 2
FE_EINVAL, FE_ENOMEM, FE_EHIP, FE_ENAN, FE_ESTATE = -1, -2, -3, -4, -5
FE_FP64, FE_FP32 = 0, 1
FE_PC_AUTO, FE_PC_BJACOBI, FE_PC_MULTIGRID = 0, 1, 2

EXPORTS = [
    "fe_problem_create", "fe_problem_destroy", "fe_problem_set_phys", "fe_problem_ndof",
    "fe_residual", "fe_jvp", "fe_adjoint_jtvp", "fe_dR_dgamma", "fe_compliance",
    "fe_solve_opts_default", "newton_solve", "fe_adjoint_solve", "fe_block_diagonal",
    "fe_line_search_lambda", "fe_solve_footprint_bytes", "serve_create", "serve_submit",
    "serve_poll", "serve_times", "serve_error", "serve_destroy", "fe_last_error", "fe_version",
    "serve_create_ex", "serve_engine_stats", "fe_jvp_batch_create", "fe_jvp_batch_run",
    "fe_jvp_batch_destroy", "fe_block_diagonal_fp32",
]
FE_SERVE_BATCHED = 1


class FeGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("h", ctypes.c_double)]


class FePhys(ctypes.Structure):
    _fields_ = [("Pr", ctypes.c_double), ("Gr", ctypes.c_double), ("Ck", ctypes.c_double),
                ("qf", ctypes.c_double), ("alpha_max", ctypes.c_double),
                ("q_alpha", ctypes.c_double), ("eg", ctypes.c_double * 3)]


class FeSolveOpts(ctypes.Structure):
    _fields_ = [("rtol_newton", ctypes.c_double), ("rtol_lin", ctypes.c_double),
                ("max_newton", ctypes.c_int), ("restart", ctypes.c_int),
                ("max_lin", ctypes.c_int), ("n_refine", ctypes.c_int),
                ("krylov_op_prec", ctypes.c_int), ("ls_lambda_min", ctypes.c_double),
                ("verbose", ctypes.c_int), ("precond", ctypes.c_int), ("mg_nu", ctypes.c_int),
                ("mg_omega", ctypes.c_double), ("atol_newton", ctypes.c_double),
                ("ramp_steps", ctypes.c_int),
                ("mg_assembled_nodes", ctypes.c_int), ("mg_nu_post", ctypes.c_int),
                ("pc_prec", ctypes.c_int), ("mg_coarse_reuse", ctypes.c_int)]


class FeSolveReport(ctypes.Structure):
    _fields_ = [("newton_its", ctypes.c_int), ("lin_its_total", ctypes.c_int),
                ("status", ctypes.c_int), ("res0", ctypes.c_double),
                ("res_final", ctypes.c_double), ("lambda_last", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("t_jv_s", ctypes.c_double),
                ("t_prec_s", ctypes.c_double), ("t_orth_s", ctypes.c_double),
                ("t_res_s", ctypes.c_double), ("t_setup_s", ctypes.c_double),
                ("lin_its", ctypes.c_int * 64), ("res_hist", ctypes.c_double * 65),
                ("precond", ctypes.c_int), ("mg_levels", ctypes.c_int),
                ("ramp_stages", ctypes.c_int)]

    def as_dict(self) -> dict:
        n = min(self.newton_its, 64)
        return {"newton_its": self.newton_its, "lin_its_total": self.lin_its_total,
                "status": self.status, "res0": self.res0, "res_final": self.res_final,
                "lambda_last": self.lambda_last, "t_total_s": self.t_total_s,
                "t_jv_s": self.t_jv_s, "t_prec_s": self.t_prec_s, "t_orth_s": self.t_orth_s,
                "t_res_s": self.t_res_s, "t_setup_s": self.t_setup_s,
                "lin_its": list(self.lin_its[:n]), "res_hist": list(self.res_hist[:n + 1]),
                "precond": {1: "bjacobi", 2: "multigrid"}.get(self.precond, "none"),
                "mg_levels": self.mg_levels, "ramp_stages": self.ramp_stages}


class FeTopoptOpts(ctypes.Structure):
    _fields_ = [("n_steps", ctypes.c_int), ("iters_per_step", ctypes.c_int * 5),
                ("q_f", ctypes.c_double * 5), ("q_alpha", ctypes.c_double * 5),
                ("alpha_max", ctypes.c_double * 5), ("vf", ctypes.c_double),
                ("filter_radius", ctypes.c_double), ("move", ctypes.c_double),
                ("state", FeSolveOpts), ("adjoint", FeSolveOpts)]


class FeTopoptRecord(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int), ("step", ctypes.c_int), ("f", ctypes.c_double),
                ("f_scaled", ctypes.c_double), ("g", ctypes.c_double),
                ("change", ctypes.c_double), ("lambda_mma", ctypes.c_double),
                ("newton_its", ctypes.c_int), ("lin_its", ctypes.c_int),
                ("adj_its", ctypes.c_int), ("ramp_stages", ctypes.c_int),
                ("t_state_s", ctypes.c_double), ("t_adjoint_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class FeError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed with code {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load ``libfe_hip.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with "
                              "`python -m paper_1508_04596_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        P = ctypes.POINTER
        L.fe_problem_create.argtypes = [P(FeGrid), P(FePhys), vp, P(vp)]
        L.fe_problem_destroy.argtypes = [vp]
        L.fe_problem_set_phys.argtypes = [vp, P(FePhys)]
        L.fe_problem_ndof.argtypes = [vp]
        L.fe_problem_ndof.restype = i64
        L.fe_residual.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fe_jvp.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.fe_adjoint_jtvp.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.fe_jacobian_dense.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fe_filter_create.argtypes = [P(FeGrid), dbl, P(vp)]
        L.fe_filter_apply.argtypes = [vp, vp, vp, vp]
        L.fe_filter_apply_transpose.argtypes = [vp, vp, vp, vp]
        L.fe_filter_iterations.argtypes = [vp]
        L.fe_filter_destroy.argtypes = [vp]
        L.fe_mma_create.argtypes = [ctypes.c_int64, dbl, dbl, dbl, P(vp)]
        L.fe_mma_update.argtypes = [vp, vp, vp, dbl, vp, P(dbl), vp]
        L.fe_mma_destroy.argtypes = [vp]
        L.fe_topopt_opts_default.argtypes = [P(FeTopoptOpts)]
        L.fe_topopt_opts_default.restype = None
        L.fe_topopt_create.argtypes = [vp, vp, vp, vp, P(FeTopoptOpts), P(vp)]
        L.fe_topopt_evaluate.argtypes = [vp, vp, vp, P(dbl), P(dbl), vp, vp, P(FeTopoptRecord), vp]
        L.fe_topopt_step.argtypes = [vp, vp, vp, P(FeTopoptRecord), vp]
        L.fe_topopt_run.argtypes = [vp, vp, vp, P(FeTopoptRecord), i32, P(i32), vp]
        L.fe_topopt_destroy.argtypes = [vp]
        L.fe_kernel_timer.argtypes = [vp, i32]
        L.fe_kernel_timer_read.argtypes = [vp, P(dbl), P(ctypes.c_int64)]
        L.fe_dR_dgamma.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.fe_jvp_noalloc.argtypes = [P(FeGrid), P(FePhys), i32, vp, vp, vp, vp, vp, vp, vp]
        L.fe_jvp_noalloc_scratch_bytes.argtypes = [P(FeGrid), i32]
        L.fe_jvp_noalloc_scratch_bytes.restype = i64
        L.fe_compliance.argtypes = [vp, vp, vp, P(dbl), vp, vp]
        L.fe_block_diagonal.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fe_block_diagonal_fp32.argtypes = [vp, vp, vp, vp, vp, vp]
        L.fe_solve_opts_default.argtypes = [P(FeSolveOpts)]
        L.fe_solve_opts_default.restype = None
        L.newton_solve.argtypes = [vp, vp, vp, vp, P(FeSolveOpts), P(FeSolveReport), vp]
        L.fe_adjoint_solve.argtypes = [vp, vp, vp, vp, vp, vp, P(FeSolveOpts), P(FeSolveReport), vp]
        L.fe_line_search_lambda.argtypes = [dbl, dbl, dbl, dbl]
        L.fe_line_search_lambda.restype = dbl
        L.fe_solve_footprint_bytes.argtypes = [P(FeGrid), P(FeSolveOpts)]
        L.fe_solve_footprint_bytes.restype = i64
        L.serve_create.argtypes = [ctypes.c_size_t, i32, P(vp)]
        L.serve_create_ex.argtypes = [ctypes.c_size_t, i32, i32, P(vp)]
        L.serve_engine_stats.argtypes = [vp, P(ctypes.c_uint64), P(ctypes.c_uint64)]
        L.fe_jvp_batch_create.argtypes = [i32, P(vp), i32, P(vp), P(vp), P(vp), P(vp), P(vp), P(vp)]
        L.fe_jvp_batch_run.argtypes = [vp, vp]
        L.fe_jvp_batch_destroy.argtypes = [vp]
        L.serve_submit.argtypes = [vp, P(FeGrid), P(FePhys), vp, vp, P(FeSolveOpts),
                                   P(ctypes.c_uint64)]
        L.serve_submit_x0.argtypes = [vp, P(FeGrid), P(FePhys), vp, vp, vp, P(FeSolveOpts),
                                      P(ctypes.c_uint64)]
        L.serve_poll.argtypes = [vp, ctypes.c_uint64, vp, P(FeSolveReport)]
        L.serve_times.argtypes = [vp, ctypes.c_uint64, P(dbl), P(dbl), P(dbl)]
        L.serve_destroy.argtypes = [vp]
        L.serve_error.argtypes = [vp, ctypes.c_uint64]
        L.serve_error.restype = ctypes.c_char_p
        L.fe_last_error.restype = ctypes.c_char_p
        L.fe_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str, ok=(FE_OK,)) -> int:
    if rc not in ok:
        raise FeError(rc, what, lib().fe_last_error().decode())
    return rc


def _ptr(t: Optional[torch.Tensor], dtype=None, n: Optional[int] = None, what: str = "array"):
    """Device pointer of ``t`` after checking device, layout, dtype and (if ``n``
    is given) the number of entries: the kernels index up to the grid's sizes,
    so a short tensor is rejected here, before any launch."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what}: expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what}: expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what}: expected {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: expected {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def make_phys(Pr=1.0, Gr=1e3, Ck=0.1, qf=0.881, alpha_max=1e4, q_alpha=1.0, eg=(0.0, 0.0, -1.0)):
    ph = FePhys()
    ph.Pr, ph.Gr, ph.Ck, ph.qf, ph.alpha_max, ph.q_alpha = Pr, Gr, Ck, qf, alpha_max, q_alpha
    for d in range(3):
        ph.eg[d] = eg[d]
    return ph


def solve_opts(**kw) -> FeSolveOpts:
    o = FeSolveOpts()
    lib().fe_solve_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "krylov_op_prec" and isinstance(v, str):
            v = FE_FP32 if v in ("fp32", "mixed") else FE_FP64
        if k == "pc_prec" and isinstance(v, str):
            v = {"fp64": FE_FP64, "fp32": FE_FP32}[v]
        if k == "precond" and isinstance(v, str):
            v = {"auto": FE_PC_AUTO, "bjacobi": FE_PC_BJACOBI, "multigrid": FE_PC_MULTIGRID,
                 "mg": FE_PC_MULTIGRID}[v]
        setattr(o, k, v)
    return o


class Problem:
    """Owns an ``fe_problem`` handle (grid, parameters, Dirichlet mask, workspace)."""

    def __init__(self, nx, ny, nz, h, phys: FePhys, mask: Optional[torch.Tensor] = None):
        self.nx, self.ny, self.nz, self.h = nx, ny, nz, h
        self.n_nodes = (nx + 1) * (ny + 1) * (nz + 1)
        self.n_dof = 5 * self.n_nodes
        self.n_el = nx * ny * nz
        g = FeGrid(nx, ny, nz, h)
        self._grid = g
        self.phys = phys
        handle = ctypes.c_void_p()
        _check(lib().fe_problem_create(ctypes.byref(g), ctypes.byref(phys),
                                       _ptr(mask, torch.uint8, self.n_dof, "mask"),
                                       ctypes.byref(handle)),
               "fe_problem_create")
        self.handle = handle

    @classmethod
    def from_inputs(cls, p, mask="solve", device="cuda"):
        """Problem for an ``inputs.Problem`` (``mask`` = 'solve', 'walls' or None)."""
        lib()  # a missing library is the error to report, before any device work
        m = None
        if mask is not None:
            arr = p.mask_solve if mask == "solve" else p.mask_walls
            m = torch.from_numpy(arr).to(device)
        ph = make_phys(p.Pr, p.Gr, p.Ck, p.qf, p.alpha_max, p.q_alpha, p.eg)
        return cls(p.nx, p.ny, p.nz, p.h, ph, m)

    def set_phys(self, phys: FePhys):
        _check(lib().fe_problem_set_phys(self.handle, ctypes.byref(phys)), "fe_problem_set_phys")
        self.phys = phys

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().fe_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _prec_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return FE_FP64
    if t.dtype == torch.float32:
        return FE_FP32
    raise ValueError("x/v must be float64 or float32")


def fe_residual(prob: Problem, x, gamma, s, out=None, stream=None):
    out = torch.empty_like(x) if out is None else out
    nd, ne = prob.n_dof, prob.n_el
    _check(lib().fe_residual(prob.handle, _ptr(x, torch.float64, nd, "x"),
                             _ptr(gamma, torch.float64, ne, "gamma"), _ptr(s, torch.float64, ne, "s"),
                             _ptr(out, torch.float64, nd, "out"), _stream(stream)),
           "fe_residual")
    return out


def fe_jvp(prob: Problem, x, gamma, s, v, out=None, stream=None):
    prec = _prec_of(x)
    out = torch.empty_like(v) if out is None else out
    nd, ne = prob.n_dof, prob.n_el
    _check(lib().fe_jvp(prob.handle, prec, _ptr(x, x.dtype, nd, "x"),
                        _ptr(gamma, torch.float64, ne, "gamma"), _ptr(s, torch.float64, ne, "s"),
                        _ptr(v, x.dtype, nd, "v"), _ptr(out, x.dtype, nd, "out"),
                        _stream(stream)), "fe_jvp")
    return out


FE_NOALLOC_SCRATCH_BYTES = 64 << 20


def fe_jvp_noalloc_scratch_bytes(nx, ny, nz, prec=FE_FP64) -> int:
    return int(lib().fe_jvp_noalloc_scratch_bytes(ctypes.byref(FeGrid(nx, ny, nz, 1.0)), prec))


def fe_jvp_noalloc(nx, ny, nz, h, phys: FePhys, mask, x, gamma, s, v, out=None, stream=None):
    """J v through the allocation-free entry point (no problem handle); ``mask``
    is a device uint8 tensor of n_dof entries or None."""
    prec = _prec_of(x)
    nd = 5 * (nx + 1) * (ny + 1) * (nz + 1)
    ne = nx * ny * nz
    out = torch.empty_like(v) if out is None else out
    _check(lib().fe_jvp_noalloc(ctypes.byref(FeGrid(nx, ny, nz, h)), ctypes.byref(phys), prec,
                                _ptr(mask, torch.uint8, nd, "mask"), _ptr(x, x.dtype, nd, "x"),
                                _ptr(gamma, torch.float64, ne, "gamma"),
                                _ptr(s, torch.float64, ne, "s"), _ptr(v, x.dtype, nd, "v"),
                                _ptr(out, x.dtype, nd, "out"), _stream(stream)), "fe_jvp_noalloc")
    return out


def fe_jacobian_dense(prob: Problem, x, gamma, s, stream=None):
    """Assembled J(x) of a small problem as a dense row-major numpy array."""
    import numpy as np
    n = int(lib().fe_problem_ndof(prob.handle))
    J = np.empty((n, n), dtype=np.float64)
    _check(lib().fe_jacobian_dense(prob.handle, _ptr(x, torch.float64, n, "x"),
                                   _ptr(gamma, torch.float64, prob.n_el, "gamma"),
                                   _ptr(s, torch.float64, prob.n_el, "s"),
                                   J.ctypes.data_as(ctypes.c_void_p),
                                   _stream(stream)), "fe_jacobian_dense")
    return J


def fe_kernel_timer(prob: Problem, enable: bool = True):
    """Start (clearing the record) or stop timing fe_jvp's element-pass kernel."""
    _check(lib().fe_kernel_timer(prob.handle, 1 if enable else 0), "fe_kernel_timer")


def fe_kernel_timer_read(prob: Problem):
    """(summed element-pass milliseconds, launches) since the last read; clears the record."""
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib().fe_kernel_timer_read(prob.handle, ctypes.byref(ms), ctypes.byref(n)),
           "fe_kernel_timer_read")
    return ms.value, n.value


def fe_adjoint_jtvp(prob: Problem, x, gamma, s, w, out=None, stream=None):
    prec = _prec_of(x)
    out = torch.empty_like(w) if out is None else out
    nd, ne = prob.n_dof, prob.n_el
    _check(lib().fe_adjoint_jtvp(prob.handle, prec, _ptr(x, x.dtype, nd, "x"),
                                 _ptr(gamma, torch.float64, ne, "gamma"),
                                 _ptr(s, torch.float64, ne, "s"), _ptr(w, x.dtype, nd, "w"),
                                 _ptr(out, x.dtype, nd, "out"), _stream(stream)), "fe_adjoint_jtvp")
    return out


def fe_dR_dgamma(prob: Problem, x, gamma, s, lam, out=None, stream=None):
    out = torch.empty_like(gamma) if out is None else out
    nd, ne = prob.n_dof, prob.n_el
    _check(lib().fe_dR_dgamma(prob.handle, _ptr(x, torch.float64, nd, "x"),
                              _ptr(gamma, torch.float64, ne, "gamma"), _ptr(s, torch.float64, ne, "s"),
                              _ptr(lam, torch.float64, nd, "lambda"),
                              _ptr(out, torch.float64, ne, "out"), _stream(stream)), "fe_dR_dgamma")
    return out


def fe_compliance(prob: Problem, x, s, dfdx=None, stream=None):
    f = ctypes.c_double()
    _check(lib().fe_compliance(prob.handle, _ptr(x, torch.float64, prob.n_dof, "x"),
                               _ptr(s, torch.float64, prob.n_el, "s"), ctypes.byref(f),
                               _ptr(dfdx, torch.float64, prob.n_dof, "dfdx"), _stream(stream)),
           "fe_compliance")
    return f.value


def fe_block_diagonal_fp32(prob: Problem, x32, gamma, s, out=None, stream=None):
    """Nodal 5x5 blocks in FP32 arithmetic from an FP32 state (mixed-precision set-up)."""
    out = torch.empty(25 * prob.n_nodes, dtype=torch.float32, device=x32.device) if out is None else out
    ne = prob.n_el
    _check(lib().fe_block_diagonal_fp32(prob.handle, _ptr(x32, torch.float32, prob.n_dof, "x"),
                                        _ptr(gamma, torch.float64, ne, "gamma"),
                                        _ptr(s, torch.float64, ne, "s"),
                                        _ptr(out, torch.float32, 25 * prob.n_nodes, "out"),
                                        _stream(stream)), "fe_block_diagonal_fp32")
    return out


def fe_block_diagonal(prob: Problem, x, gamma, s, out=None, stream=None):
    out = torch.empty(25 * prob.n_nodes, dtype=torch.float64, device=x.device) if out is None else out
    ne = prob.n_el
    _check(lib().fe_block_diagonal(prob.handle, _ptr(x, torch.float64, prob.n_dof, "x"),
                                   _ptr(gamma, torch.float64, ne, "gamma"),
                                   _ptr(s, torch.float64, ne, "s"),
                                   _ptr(out, torch.float64, 25 * prob.n_nodes, "out"),
                                   _stream(stream)), "fe_block_diagonal")
    return out


def newton_solve(prob: Problem, gamma, s, x, opts: Optional[FeSolveOpts] = None, stream=None,
                 allow_not_converged=False) -> dict:
    rep = FeSolveReport()
    o = solve_opts() if opts is None else opts
    rc = lib().newton_solve(prob.handle, _ptr(gamma, torch.float64, prob.n_el, "gamma"),
                            _ptr(s, torch.float64, prob.n_el, "s"),
                            _ptr(x, torch.float64, prob.n_dof, "x"), ctypes.byref(o),
                            ctypes.byref(rep), _stream(stream))
    _check(rc, "newton_solve", ok=(FE_OK, FE_NOT_CONVERGED) if allow_not_converged else (FE_OK,))
    return rep.as_dict()


def fe_adjoint_solve(prob: Problem, x, gamma, s, rhs, lam=None, opts: Optional[FeSolveOpts] = None,
                     stream=None, allow_not_converged=False):
    lam = torch.empty_like(rhs) if lam is None else lam
    rep = FeSolveReport()
    o = solve_opts() if opts is None else opts
    nd, ne = prob.n_dof, prob.n_el
    rc = lib().fe_adjoint_solve(prob.handle, _ptr(x, torch.float64, nd, "x"),
                                _ptr(gamma, torch.float64, ne, "gamma"),
                                _ptr(s, torch.float64, ne, "s"), _ptr(rhs, torch.float64, nd, "rhs"),
                                _ptr(lam, torch.float64, nd, "lambda"), ctypes.byref(o),
                                ctypes.byref(rep), _stream(stream))
    _check(rc, "fe_adjoint_solve", ok=(FE_OK, FE_NOT_CONVERGED) if allow_not_converged else (FE_OK,))
    return lam, rep.as_dict()


def fe_line_search_lambda(phi0, phi_half, phi1, lambda_min=0.05) -> float:
    return float(lib().fe_line_search_lambda(phi0, phi_half, phi1, lambda_min))


def fe_solve_footprint_bytes(nx, ny, nz, h=1.0, opts: Optional[FeSolveOpts] = None) -> int:
    g = FeGrid(nx, ny, nz, h)
    return int(lib().fe_solve_footprint_bytes(ctypes.byref(g), ctypes.byref(opts) if opts else None))


class JvpBatch:
    """J v of several problems in one batched launch (``fe_jvp_batch_*``).

    ``probs``: distinct :class:`Problem` objects; ``x``, ``v``, ``out``: lists
    of device tensors of one precision (float64 or float32); ``gamma``, ``s``:
    lists of float64 device tensors.  The table holds the tensors' addresses:
    keep them alive (and in place) while the batch is used."""

    def __init__(self, probs, x, gamma, s, v, out):
        n = len(probs)
        if not (len(x) == len(gamma) == len(s) == len(v) == len(out) == n) or n < 1:
            raise ValueError("JvpBatch: lists of equal length >= 1 expected")
        self.handle = None
        prec = _prec_of(x[0])
        dt = x[0].dtype
        arr = ctypes.c_void_p * n
        ptrs = {}
        for name, lst, dty, size in (("x", x, dt, "n_dof"), ("v", v, dt, "n_dof"),
                                     ("out", out, dt, "n_dof"),
                                     ("gamma", gamma, torch.float64, "n_el"),
                                     ("s", s, torch.float64, "n_el")):
            ptrs[name] = arr(*[_ptr(t, dty, getattr(pr, size), f"{name}[{i}]").value
                               for i, (t, pr) in enumerate(zip(lst, probs))])
        ph = arr(*[pr.handle.value for pr in probs])
        h = ctypes.c_void_p()
        _check(lib().fe_jvp_batch_create(n, ph, prec, ptrs["x"], ptrs["gamma"], ptrs["s"],
                                         ptrs["v"], ptrs["out"], ctypes.byref(h)),
               "fe_jvp_batch_create")
        self.handle = h
        self._keep = (list(x), list(gamma), list(s), list(v), list(out))

    def run(self, stream=None):
        _check(lib().fe_jvp_batch_run(self.handle, _stream(stream)), "fe_jvp_batch_run")

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().fe_jvp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fe_version() -> str:
    return lib().fe_version().decode()


class Server:
    """Continuous-batching solve server (``serve_*`` entry points).

    Requests carry their own grid, parameters, design and source (host numpy
    arrays, copied at submit); walls and the pressure pin are applied by the
    library and every solve starts from x = 0."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 4, batched: bool = False):
        """``batched``: run the requests' linear solves in lockstep, one launch
        per kernel over all running requests (``FE_SERVE_BATCHED``)."""
        self.handle = None
        h = ctypes.c_void_p()
        _check(lib().serve_create_ex(ctypes.c_size_t(int(hbm_budget_bytes)), int(max_active),
                                     FE_SERVE_BATCHED if batched else 0, ctypes.byref(h)),
               "serve_create_ex")
        self.handle = h
        self.batched = batched
        self.n_dof = {}

    def engine_stats(self):
        """(lockstep steps, batched launches) of the batched engine so far."""
        a, b = ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().serve_engine_stats(self.handle, ctypes.byref(a), ctypes.byref(b)),
               "serve_engine_stats")
        return a.value, b.value

    def submit(self, nx, ny, nz, h, phys: FePhys, gamma, s, opts: Optional[FeSolveOpts] = None,
               allow_enomem=False, x0=None) -> int:
        """Queue a state solve; ``x0`` (host, n_dof) warm-starts Newton (default zero)."""
        import numpy as np
        g = np.ascontiguousarray(gamma, dtype=np.float64)
        ss = np.ascontiguousarray(s, dtype=np.float64)
        assert g.size == nx * ny * nz and ss.size == nx * ny * nz
        t = ctypes.c_uint64()
        grid = FeGrid(nx, ny, nz, h)
        if x0 is None:
            rc = lib().serve_submit(self.handle, ctypes.byref(grid), ctypes.byref(phys),
                                    g.ctypes.data_as(ctypes.c_void_p),
                                    ss.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(opts) if opts is not None else None, ctypes.byref(t))
        else:
            xx = np.ascontiguousarray(x0, dtype=np.float64)
            assert xx.size == 5 * (nx + 1) * (ny + 1) * (nz + 1)
            rc = lib().serve_submit_x0(self.handle, ctypes.byref(grid), ctypes.byref(phys),
                                       g.ctypes.data_as(ctypes.c_void_p),
                                       ss.ctypes.data_as(ctypes.c_void_p),
                                       xx.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(t))
        _check(rc, "serve_submit", ok=(FE_OK, FE_ENOMEM) if allow_enomem else (FE_OK,))
        self.n_dof[t.value] = 5 * (nx + 1) * (ny + 1) * (nz + 1)
        return t.value

    def poll(self, ticket: int, want_x=True):
        """(status, x or None, report dict); status FE_PENDING while not finished."""
        import numpy as np
        x = np.empty(self.n_dof[ticket]) if want_x else None
        rep = FeSolveReport()
        rc = lib().serve_poll(self.handle, ctypes.c_uint64(ticket),
                              x.ctypes.data_as(ctypes.c_void_p) if want_x else None,
                              ctypes.byref(rep))
        if rc == FE_PENDING:
            return rc, None, None
        return rc, x, rep.as_dict()

    def error(self, ticket: int) -> str:
        return lib().serve_error(self.handle, ctypes.c_uint64(ticket)).decode()

    def times(self, ticket: int):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        lib().serve_times(self.handle, ctypes.c_uint64(ticket), ctypes.byref(a), ctypes.byref(b),
                          ctypes.byref(c))
        return a.value, b.value, c.value

    def wait(self, ticket: int, poll_s=0.0005, timeout_s=600.0):
        import time
        t0 = time.time()
        while True:
            rc, x, rep = self.poll(ticket)
            if rc != FE_PENDING:
                return rc, x, rep
            if time.time() - t0 > timeout_s:
                raise TimeoutError(f"request {ticket} not finished after {timeout_s} s")
            time.sleep(poll_s)

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---- optimisation loop ----------------------------------------------------------------

class Filter:
    """PDE density filter on an element grid (radius R in length units)."""

    def __init__(self, nx, ny, nz, h, radius):
        self.handle = None
        self.n_el = nx * ny * nz
        h_ = ctypes.c_void_p()
        _check(lib().fe_filter_create(ctypes.byref(FeGrid(nx, ny, nz, h)), radius, ctypes.byref(h_)),
               "fe_filter_create")
        self.handle = h_

    def apply(self, x, out=None, stream=None):
        out = torch.empty_like(x) if out is None else out
        _check(lib().fe_filter_apply(self.handle, _ptr(x, torch.float64, self.n_el, "in"),
                                     _ptr(out, torch.float64, self.n_el, "out"), _stream(stream)),
               "fe_filter_apply")
        return out

    def apply_transpose(self, x, out=None, stream=None):
        out = torch.empty_like(x) if out is None else out
        _check(lib().fe_filter_apply_transpose(self.handle, _ptr(x, torch.float64, self.n_el, "in"),
                                               _ptr(out, torch.float64, self.n_el, "out"),
                                               _stream(stream)),
               "fe_filter_apply_transpose")
        return out

    @property
    def iterations(self) -> int:
        return int(lib().fe_filter_iterations(self.handle))

    def close(self):
        if self.handle:
            lib().fe_filter_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MMA:
    """Method of moving asymptotes, one constraint, on the device."""

    def __init__(self, n, xmin=0.0, xmax=1.0, move=0.2):
        self.handle = None
        self.n = int(n)
        h_ = ctypes.c_void_p()
        _check(lib().fe_mma_create(n, xmin, xmax, move, ctypes.byref(h_)), "fe_mma_create")
        self.handle = h_

    def update(self, x, df0, f1, df1, stream=None) -> float:
        lam = ctypes.c_double()
        n = self.n
        _check(lib().fe_mma_update(self.handle, _ptr(x, torch.float64, n, "x"),
                                   _ptr(df0, torch.float64, n, "df0"), float(f1),
                                   _ptr(df1, torch.float64, n, "df1"), ctypes.byref(lam),
                                   _stream(stream)), "fe_mma_update")
        return lam.value

    def close(self):
        if self.handle:
            lib().fe_mma_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def topopt_opts(**kw) -> FeTopoptOpts:
    o = FeTopoptOpts()
    lib().fe_topopt_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k in ("state", "adjoint") and isinstance(v, dict):
            sub = getattr(o, k)
            for kk, vv in v.items():
                if kk == "krylov_op_prec" and isinstance(vv, str):
                    vv = FE_FP32 if vv in ("fp32", "mixed") else FE_FP64
                if kk == "pc_prec" and isinstance(vv, str):
                    vv = {"fp64": FE_FP64, "fp32": FE_FP32}[vv]
                setattr(sub, kk, vv)
        elif k in ("iters_per_step", "q_f", "q_alpha", "alpha_max"):
            arr = getattr(o, k)
            for i, vv in enumerate(v):
                arr[i] = vv
        else:
            setattr(o, k, v)
    return o


class TopOpt:
    """Design loop on a state problem; design_mask (uint8), gamma_fixed, s: device tensors
    of length n_el, kept alive by this object."""

    def __init__(self, prob: Problem, design_mask, gamma_fixed, s, opts: Optional[FeTopoptOpts] = None):
        self.handle = None
        self.prob = prob
        self._keep = (design_mask, gamma_fixed, s)
        h_ = ctypes.c_void_p()
        ne = prob.n_el
        _check(lib().fe_topopt_create(prob.handle, _ptr(design_mask, torch.uint8, ne, "design_mask"),
                                      _ptr(gamma_fixed, torch.float64, ne, "gamma_fixed"),
                                      _ptr(s, torch.float64, ne, "s"),
                                      ctypes.byref(opts) if opts is not None else None,
                                      ctypes.byref(h_)), "fe_topopt_create")
        self.handle = h_

    def evaluate(self, rho, x, grads=True, stream=None):
        f, g = ctypes.c_double(), ctypes.c_double()
        df = torch.zeros_like(rho) if grads else None
        dg = torch.zeros_like(rho) if grads else None
        rec = FeTopoptRecord()
        nd, ne = self.prob.n_dof, self.prob.n_el
        _check(lib().fe_topopt_evaluate(self.handle, _ptr(rho, torch.float64, ne, "rho"),
                                        _ptr(x, torch.float64, nd, "x"), ctypes.byref(f),
                                        ctypes.byref(g), _ptr(df, torch.float64, ne, "dfdrho"),
                                        _ptr(dg, torch.float64, ne, "dgdrho"), ctypes.byref(rec),
                                        _stream(stream)),
               "fe_topopt_evaluate")
        return f.value, g.value, df, dg, rec.as_dict()

    def step(self, rho, x, stream=None) -> dict:
        rec = FeTopoptRecord()
        _check(lib().fe_topopt_step(self.handle, _ptr(rho, torch.float64, self.prob.n_el, "rho"),
                                    _ptr(x, torch.float64, self.prob.n_dof, "x"),
                                    ctypes.byref(rec), _stream(stream)), "fe_topopt_step")
        return rec.as_dict()

    def run(self, rho, x, cap=10000, stream=None):
        hist = (FeTopoptRecord * cap)()
        n = ctypes.c_int()
        _check(lib().fe_topopt_run(self.handle, _ptr(rho, torch.float64, self.prob.n_el, "rho"),
                                   _ptr(x, torch.float64, self.prob.n_dof, "x"),
                                   hist, cap, ctypes.byref(n), _stream(stream)), "fe_topopt_run")
        return [hist[i].as_dict() for i in range(min(n.value, cap))]

    def close(self):
        if self.handle:
            lib().fe_topopt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
