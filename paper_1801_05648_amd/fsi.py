"""Python binding of libfsi (argument marshalling only).

Every step of the solve runs in the HIP library behind the C ABI declared in
``include/fsi.h``; this module converts numpy / torch arguments to plain
pointers and sizes and turns status codes into exceptions.  PyTorch provides
device memory and the HIP stream.  There is no fallback: if ``libfsi.so`` is
missing the import fails.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfsi.so")

BLOCKS = ("M", "C_ms", "C_sm", "S", "C_sf", "C_fm", "C_fs", "F")
HIERARCHIES = {"H_M": 0, "H_SIG": 1, "H_MS": 2, "H_A": 3, "H_P": 4}
PRECISION = {"f64": 0, "f32": 1, "f32-bf16diag": 2}
SCHUR = {"simple": 0, "simplec": 1}

STATUS = {0: "FSI_OK", 1: "FSI_NOT_CONVERGED", -1: "FSI_ERR_ARG", -2: "FSI_ERR_CSR",
          -3: "FSI_ERR_STRUCT", -4: "FSI_ERR_HIP", -5: "FSI_ERR_OOM", -6: "FSI_ERR_NUMERIC",
          -7: "FSI_ERR_STATE"}


NEWTON_MAX = 64
NEWTON_PC = {"rebuild": 0, "reuse": 1, "keep": 2}


class CFeMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("cells", ctypes.c_int32 * 3), ("extent", ctypes.c_double * 3),
                ("solid_lo", ctypes.c_int32 * 3), ("solid_hi", ctypes.c_int32 * 3),
                ("rho_f", ctypes.c_double), ("nu_f", ctypes.c_double), ("rho_s", ctypes.c_double),
                ("mu_s", ctypes.c_double), ("lambda_s", ctypes.c_double), ("dt", ctypes.c_double),
                ("theta", ctypes.c_double), ("newton_mesh", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n_nodes", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                                ("vdof", "udof", "pdof", "v", "u", "p", "v_old", "u_old", "w",
                                                 "u_fz")]


class CNewtonOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("reassemble_ratio", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("lin_tol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("maxit", ctypes.c_int32)]


class CNewtonInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int32), ("steps", ctypes.c_int32), ("reassemblies", ctypes.c_int32),
                ("lin_iters_total", ctypes.c_int32), ("resid", ctypes.c_double * (NEWTON_MAX + 1)),
                ("reassembled", ctypes.c_int32 * NEWTON_MAX), ("lin_iters", ctypes.c_int32 * NEWTON_MAX),
                ("t_assemble_ms", ctypes.c_double), ("t_precond_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


@dataclasses.dataclass
class NewtonInfo:
    status: str
    converged: bool
    steps: int
    reassemblies: int
    residuals: list      # ||r_k||_inf, k = 0 .. steps
    reassembled: list    # per step
    lin_iters: list      # per step
    t_assemble_ms: float
    t_precond_ms: float
    t_solve_ms: float
    t_total_ms: float


class FsiError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.name = STATUS.get(code, str(code))


class CCsr(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class CLayout(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n_m", ctypes.c_int64), ("n_s", ctypes.c_int64), ("n_f", ctypes.c_int64),
                ("n_vs", ctypes.c_int64), ("n_vf", ctypes.c_int64), ("dt_theta", ctypes.c_double),
                ("n_nodes", ctypes.c_int64), ("coords", ctypes.c_void_p), ("dof_node", ctypes.c_void_p),
                ("node_ijk", ctypes.c_void_p)]


class CPrecondOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_coarse", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("cheb_degree", ctypes.c_int32), ("strength0", ctypes.c_double),
                ("cheb_mask", ctypes.c_int32), ("poly_mask", ctypes.c_int32), ("poly_degree", ctypes.c_int32),
                ("schur", ctypes.c_int32), ("poly_ratio", ctypes.c_double), ("fluid_inner", ctypes.c_int32),
                ("fluid_inner_pc", ctypes.c_int32), ("reuse", ctypes.c_int32), ("x_approx", ctypes.c_int32),
                ("uzawa_inner", ctypes.c_int32), ("order", ctypes.c_int32)]


class CSolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("pad", ctypes.c_int32)]


class CSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("true_rel_resid", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("t_precond_ms", ctypes.c_double), ("t_spmv_ms", ctypes.c_double), ("t_gs_ms", ctypes.c_double),
                ("n_timed", ctypes.c_int32), ("mlp_fallbacks", ctypes.c_int32),
                ("resid_block", ctypes.c_double * 3), ("bytes_spmv", ctypes.c_double),
                ("bytes_precond", ctypes.c_double), ("bytes_gs", ctypes.c_double)]


class CMlpTrainOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("exact_tol", ctypes.c_double), ("exact_maxit", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("loss", ctypes.c_int32), ("coarse_cycles", ctypes.c_int32)]


MLP_LOSS = {"l2": 0, "energy": 1}
INNER_PC = {"uzawa": 0, "triangular": 1}
X_APPROX = {"F": 0, "blockdiag": 1}
ORDER = {"msf": 0, "fsm": 1, "mfs": 2, "smf": 3, "sfm": 4, "fms": 5}


class CMlpTrainInfo(ctypes.Structure):
    _fields_ = [("vectors", ctypes.c_int32 * 2), ("samples", ctypes.c_int64 * 2),
                ("loss_first", ctypes.c_double * 2), ("loss_last", ctypes.c_double * 2)]


@dataclasses.dataclass
class SolveInfo:
    status: str
    iters: int
    restarts: int
    converged: bool
    true_rel_resid: float
    t_total_ms: float
    t_precond_ms: float = 0.0
    t_spmv_ms: float = 0.0
    t_gs_ms: float = 0.0
    n_timed: int = 0
    mlp_fallbacks: int = 0
    resid_block: tuple = (0.0, 0.0, 0.0)
    bytes_spmv: float = 0.0
    bytes_precond: float = 0.0
    bytes_gs: float = 0.0


def _declare(lib):
    P = ctypes.c_void_p
    i32, i64 = ctypes.c_int, ctypes.c_int64
    sig = {
        "fsi_create": ([ctypes.POINTER(P), i32, P], i32),
        "fsi_destroy": ([P], i32),
        "fsi_last_error": ([P], ctypes.c_char_p),
        "fsi_setup_blocks": ([P, ctypes.POINTER(CLayout), ctypes.POINTER(CCsr), i32], i32),
        "fsi_update_values": ([P, ctypes.POINTER(CCsr)], i32),
        "fsi_build_precond": ([P, ctypes.POINTER(CPrecondOpts)], i32),
        "fsi_solve": ([P, P, P, ctypes.POINTER(CSolveOpts), ctypes.POINTER(CSolveInfo)], i32),
        "fsi_spmv": ([P, P, P], i32),
        "fsi_apply_precond": ([P, P, P], i32),
        "fsi_vcycle": ([P, i32, P, P], i32),
        "fsi_set_hierarchy": ([P, i32, i32, ctypes.POINTER(CCsr), ctypes.POINTER(CCsr), ctypes.POINTER(CCsr), P], i32),
        "fsi_hierarchy_info": ([P, i32, P, P, P, P], i32),
        "fsi_get_level": ([P, i32, i32, i32, P, P, P, P, P, P], i32),
        "fsi_get_aggregates": ([P, i32, i32, P, P], i32),
        "fsi_vcycle_bytes": ([P, i32, P], i32),
        "fsi_spmv_bytes": ([P, P], i32),
        "fsi_precond_bytes": ([P, P], i32),
        "fsi_default_mlp_train_opts": ([ctypes.POINTER(CMlpTrainOpts)], None),
        "fsi_mlp_set_weights": ([P, i32, P, P, P], i32),
        "fsi_mlp_get_weights": ([P, i32, P, P, P], i32),
        "fsi_mlp_enable": ([P, i32, i32], i32),
        "fsi_mlp_forward": ([P, i32, P, P], i32),
        "fsi_mlp_forward_noalloc": ([P, i32, P, P], i32),
        "fsi_mlp_loss_grad": ([P, i32, i64, P, P, P, P, P, P, P], i32),
        "fsi_mlp_energy_grad": ([P, i32, P, i32, P, P, P, P], i32),
        "fsi_mlp_collect": ([P, i32, i32], i32),
        "fsi_mlp_train": ([P, ctypes.POINTER(CMlpTrainOpts), ctypes.POINTER(CMlpTrainInfo)], i32),
        "fsi_fe_setup": ([P, ctypes.POINTER(CFeMesh)], i32),
        "fsi_fe_residual": ([P, P, P], i32),
        "fsi_fe_jacobian": ([P, P, i32], i32),
        "fsi_newton": ([P, ctypes.POINTER(CNewtonOpts), P, ctypes.POINTER(CNewtonInfo)], i32),
        "fsi_default_newton_opts": ([ctypes.POINTER(CNewtonOpts)], None),
        "fsi_fe_advance": ([P, P], i32),
        "fsi_time_step": ([P, ctypes.POINTER(CNewtonOpts), ctypes.POINTER(CNewtonInfo)], i32),
        "fsi_fe_get_fields": ([P, P, P, P], i32),
        "fsi_default_precond_opts": ([ctypes.POINTER(CPrecondOpts)], None),
        "fsi_default_solve_opts": ([ctypes.POINTER(CSolveOpts)], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = None


def load():
    """Load libfsi.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def exported_symbols():
    """Names of the C ABI entry points this binding declares."""
    return ["fsi_create", "fsi_destroy", "fsi_last_error", "fsi_setup_blocks", "fsi_update_values",
            "fsi_build_precond",
            "fsi_solve", "fsi_spmv", "fsi_apply_precond", "fsi_vcycle", "fsi_set_hierarchy",
            "fsi_hierarchy_info", "fsi_vcycle_bytes", "fsi_spmv_bytes", "fsi_precond_bytes", "fsi_get_level", "fsi_get_aggregates",
            "fsi_default_precond_opts", "fsi_default_solve_opts", "fsi_default_mlp_train_opts",
            "fsi_mlp_set_weights", "fsi_mlp_get_weights", "fsi_mlp_enable", "fsi_mlp_forward",
            "fsi_mlp_forward_noalloc",
            "fsi_mlp_loss_grad", "fsi_mlp_energy_grad", "fsi_mlp_collect", "fsi_mlp_train",
            "fsi_fe_setup", "fsi_fe_residual", "fsi_fe_jacobian", "fsi_newton", "fsi_default_newton_opts",
            "fsi_fe_advance", "fsi_time_step", "fsi_fe_get_fields"]


def _csr_struct(nrows, ncols, rowptr, col, val, keep):
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(col, dtype=np.int32)
    vv = np.ascontiguousarray(val, dtype=np.float64)
    keep.extend([rp, ci, vv])
    return CCsr(int(nrows), int(ncols), int(ci.shape[0]), rp.ctypes.data, ci.ctypes.data, vv.ctypes.data)


def _dptr(t, n, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} entries")
    return ctypes.c_void_p(t.data_ptr())


class FsiSolver:
    """One linearised FSI system on one GPU.

    ``blocks``: mapping of the eight block names to (nrows, ncols, rowptr, col,
    val) host arrays or objects with those attributes; ``layout``: mapping with
    dim, n_m, n_s, n_f, n_vs, n_vf, dt_theta, coords (n_nodes x dim) and
    dof_node (N).
    """

    def __init__(self, blocks, layout, device: int = 0, stream=None):
        import torch
        self.lib = load()
        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        ctx = ctypes.c_void_p()
        rc = self.lib.fsi_create(ctypes.byref(ctx), device, ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise FsiError(rc, self.lib.fsi_last_error(None).decode())
        self.ctx = ctx
        self.set_system(blocks, layout)

    def set_system(self, blocks, layout):
        """Replace the linear system (fsi_setup_blocks); invalidates the
        preconditioner, keeps a learned smoother's weights.  On failure the
        previous system stays in place."""
        keep = []
        arr = (CCsr * 8)()
        for i, name in enumerate(BLOCKS):
            b = blocks[name]
            if isinstance(b, tuple):
                nr, ncl, rp, ci, vv = b
            else:
                nr, ncl, rp, ci, vv = b.nrows, b.ncols, b.rowptr, b.col, b.val
            arr[i] = _csr_struct(nr, ncl, rp, ci, vv, keep)
        coords = np.ascontiguousarray(layout["coords"], dtype=np.float64)
        dof_node = np.ascontiguousarray(layout["dof_node"], dtype=np.int32)
        ijk = layout.get("node_ijk")
        ijk = None if ijk is None else np.ascontiguousarray(ijk, dtype=np.int32)
        lay = CLayout(int(layout["dim"]), 0, int(layout["n_m"]), int(layout["n_s"]), int(layout["n_f"]),
                      int(layout["n_vs"]), int(layout["n_vf"]), float(layout["dt_theta"]),
                      int(coords.shape[0]), coords.ctypes.data, dof_node.ctypes.data,
                      None if ijk is None else ijk.ctypes.data)
        self._check(self.lib.fsi_setup_blocks(self.ctx, ctypes.byref(lay), arr, 0))
        self.N = int(layout["n_m"] + layout["n_s"] + layout["n_f"])
        self.layout = dict(layout)

    def update_values(self, blocks):
        """fsi_update_values: new values of the same sparsity patterns; A_h is
        rewritten in place, the preconditioner kept.  On failure nothing
        changes."""
        keep = []
        arr = (CCsr * 8)()
        for i, name in enumerate(BLOCKS):
            b = blocks[name]
            if isinstance(b, tuple):
                nr, ncl, rp, ci, vv = b
            else:
                nr, ncl, rp, ci, vv = b.nrows, b.ncols, b.rowptr, b.col, b.val
            arr[i] = _csr_struct(nr, ncl, rp, ci, vv, keep)
        self._check(self.lib.fsi_update_values(self.ctx, arr))

    @staticmethod
    def layout_of(sysm):
        return dict(dim=sysm.dim, n_m=sysm.n_m, n_s=sysm.n_s, n_f=sysm.n_f, n_vs=sysm.n_vs,
                    n_vf=sysm.n_vf, dt_theta=sysm.dt_theta, coords=sysm.coords, dof_node=sysm.dof_node,
                    node_ijk=sysm.node_ijk)

    @classmethod
    def from_system(cls, sysm, **kw):
        """A context on the generated system; with its finite-element
        description (generate(..., fe=True)) the assembly is set up too."""
        s = cls(sysm.blocks, cls.layout_of(sysm), **kw)
        if getattr(sysm, "fe", None) is not None:
            s.fe_setup(sysm.cfg, sysm.fe)
        return s

    def set_from_system(self, sysm):
        self.set_system(sysm.blocks, self.layout_of(sysm))
        if getattr(sysm, "fe", None) is not None:
            self.fe_setup(sysm.cfg, sysm.fe)

    # -- plumbing ------------------------------------------------------------
    def _check(self, rc):
        if rc < 0:
            raise FsiError(rc, self.lib.fsi_last_error(self.ctx).decode())
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.fsi_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _hier_len(self, which: int) -> int:
        n, _, _ = self.hierarchy_info(which)
        return int(n[0]) * (self.layout["dim"] if which == 0 else 1)

    # -- calls -----------------------------------------------------------------
    def build_precond(self, precision: str = "f64", max_coarse: int = 500, max_levels: int = 10,
                      strength0: float = 0.08, cheb_degree: int = 0, cheb=("H_MS", "H_SIG", "H_P"),
                      poly=(), poly_degree: int = 3, poly_ratio: float = 8.0, schur: str = "simple",
                      fluid_inner: int = 0, fluid_inner_pc: str = "uzawa", reuse: bool = False,
                      x_approx: str = "F", uzawa_inner: int = 0, order: str = "msf"):
        """fsi_build_precond.  reuse=True keeps the context's SA hierarchies
        (same system, same AMG parameters, Schur and X options as the
        previous build) and rebuilds only what the other options change.
        x_approx: "F" or "blockdiag" (the fluid operator standing for the
        Schur complement X).  uzawa_inner: GMRES steps per inverse of the
        Uzawa-like fluid step (Section 4.4 as written; 0 = one V-cycle).
        order: the block order of the factorisation, "msf" (the paper's)
        or another permutation of m(esh), s(olid), f(luid)."""
        def mask_of(names):
            m = 0
            for name in names:
                m |= 1 << HIERARCHIES[name]
            return m
        o = CPrecondOpts(PRECISION[precision], max_coarse, max_levels, int(cheb_degree), strength0, mask_of(cheb),
                         mask_of(poly), int(poly_degree), SCHUR[schur], float(poly_ratio), int(fluid_inner),
                         INNER_PC[fluid_inner_pc], int(bool(reuse)), X_APPROX[x_approx], int(uzawa_inner),
                         ORDER[order])
        self._check(self.lib.fsi_build_precond(self.ctx, ctypes.byref(o)))

    def fe_setup(self, cfg, fe: dict):
        """fsi_fe_setup: the grid and material data of a workload config (dim,
        cells, extent, solid_lo, solid_hi, rho_f, nu_f, rho_s, mu_s, lambda_s,
        dt, theta, newton_mesh) and its node arrays (vdof, udof, pdof, v, u,
        p, v_old, u_old, w, u_fz)."""
        d = int(cfg.dim)
        m = CFeMesh()
        m.dim = d
        for a in range(3):
            m.cells[a] = int(cfg.cells[a]) if a < d else 1
            m.extent[a] = float(cfg.extent[a]) if a < d else 1.0
            m.solid_lo[a] = int(cfg.solid_lo[a]) if a < d else 0
            m.solid_hi[a] = int(cfg.solid_hi[a]) if a < d else 1
        for k in ("rho_f", "nu_f", "rho_s", "mu_s", "lambda_s", "dt", "theta"):
            setattr(m, k, float(getattr(cfg, k)))
        m.newton_mesh = int(cfg.newton_mesh)
        keep = []
        m.n_nodes = int(np.asarray(fe["vdof"]).shape[0])
        for k in ("vdof", "udof", "pdof"):
            a = np.ascontiguousarray(fe[k], dtype=np.int64)
            keep.append(a)
            setattr(m, k, a.ctypes.data)
        for k in ("v", "u", "p", "v_old", "u_old", "w", "u_fz"):
            a = np.ascontiguousarray(fe[k], dtype=np.float64)
            keep.append(a)
            setattr(m, k, a.ctypes.data)
        self._check(self.lib.fsi_fe_setup(self.ctx, ctypes.byref(m)))

    def fe_residual(self, dU=None, R=None):
        """fsi_fe_residual: R(U) at U = the given fields + dU (device FP64)."""
        torch = self.torch
        if R is None:
            R = torch.empty(self.N, dtype=torch.float64, device=f"cuda:{self.device}")
        du = None if dU is None else _dptr(dU, self.N, "dU")
        self._check(self.lib.fsi_fe_residual(self.ctx, du, _dptr(R, self.N, "R")))
        return R

    def fe_jacobian(self, dU=None, host_blocks: bool = True):
        """fsi_fe_jacobian: A'(U) into the context's A_h (and the host blocks)."""
        du = None if dU is None else _dptr(dU, self.N, "dU")
        self._check(self.lib.fsi_fe_jacobian(self.ctx, du, int(bool(host_blocks))))

    def newton(self, dU=None, rtol: float = 1e-6, reassemble_ratio: float = 0.1, max_steps: int = 25,
               precond: str = "rebuild", lin_tol: float = 1e-3, restart: int = 50, maxit: int = 2000):
        """fsi_newton: the quasi-Newton loop of Section 6 from U = fields + dU."""
        torch = self.torch
        if dU is None:
            dU = torch.zeros(self.N, dtype=torch.float64, device=f"cuda:{self.device}")
        o = CNewtonOpts(float(rtol), float(reassemble_ratio), int(max_steps), NEWTON_PC[precond], float(lin_tol),
                        int(restart), int(maxit))
        info = CNewtonInfo()
        rc = self._check(self.lib.fsi_newton(self.ctx, ctypes.byref(o), _dptr(dU, self.N, "dU"),
                                             ctypes.byref(info)))
        return dU, self._newton_info(rc, info)

    def _newton_info(self, rc, info):
        n = info.steps
        return NewtonInfo(STATUS[rc], bool(info.converged), n, info.reassemblies,
                          list(info.resid[:n + 1]), [bool(x) for x in info.reassembled[:n]],
                          list(info.lin_iters[:n]), info.t_assemble_ms, info.t_precond_ms, info.t_solve_ms,
                          info.t_total_ms)

    def fe_advance(self, dU):
        """fsi_fe_advance: U = fields + dU becomes the next step's fields."""
        self._check(self.lib.fsi_fe_advance(self.ctx, _dptr(dU, self.N, "dU")))

    def time_step(self, rtol: float = 1e-6, reassemble_ratio: float = 0.1, max_steps: int = 25,
                  precond: str = "rebuild", lin_tol: float = 1e-3, restart: int = 50, maxit: int = 2000):
        """fsi_time_step: the quasi-Newton loop from the current fields, then the advance."""
        o = CNewtonOpts(float(rtol), float(reassemble_ratio), int(max_steps), NEWTON_PC[precond], float(lin_tol),
                        int(restart), int(maxit))
        info = CNewtonInfo()
        rc = self._check(self.lib.fsi_time_step(self.ctx, ctypes.byref(o), ctypes.byref(info)))
        return self._newton_info(rc, info)

    def fe_fields(self, n_nodes: int, dim: int):
        """fsi_fe_get_fields: the current state fields (host copies)."""
        v = np.empty((n_nodes, dim))
        u = np.empty((n_nodes, dim))
        p = np.empty(n_nodes)
        self._check(self.lib.fsi_fe_get_fields(self.ctx, v.ctypes.data, u.ctypes.data, p.ctypes.data))
        return v, u, p

    def solve(self, b, x=None, tol: float = 1e-8, restart: int = 50, maxit: int = 2000,
              timing: bool = False):
        torch = self.torch
        if x is None:
            x = torch.zeros(self.N, dtype=torch.float64, device=b.device)
        o = CSolveOpts(tol, restart, maxit, int(timing), 0)
        info = CSolveInfo()
        rc = self._check(self.lib.fsi_solve(self.ctx, _dptr(b, self.N, "b"), _dptr(x, self.N, "x"),
                                            ctypes.byref(o), ctypes.byref(info)))
        return x, SolveInfo(STATUS[rc], info.iters, info.restarts, bool(info.converged),
                            info.true_rel_resid, info.t_total_ms, info.t_precond_ms, info.t_spmv_ms,
                            info.t_gs_ms, info.n_timed, info.mlp_fallbacks, tuple(info.resid_block),
                            info.bytes_spmv, info.bytes_precond, info.bytes_gs)

    def spmv(self, x, y=None):
        if y is None:
            y = self.torch.empty_like(x)
        self._check(self.lib.fsi_spmv(self.ctx, _dptr(x, self.N, "x"), _dptr(y, self.N, "y")))
        return y

    def apply_precond(self, r, z=None):
        if z is None:
            z = self.torch.empty_like(r)
        self._check(self.lib.fsi_apply_precond(self.ctx, _dptr(r, self.N, "r"), _dptr(z, self.N, "z")))
        return z

    def vcycle(self, which, b, x=None):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        n = self._hier_len(w)
        if x is None:
            x = self.torch.empty_like(b)
        self._check(self.lib.fsi_vcycle(self.ctx, w, _dptr(b, n, "b"), _dptr(x, n, "x")))
        return x

    def set_hierarchy(self, which, A, P, R, omega):
        """A, P, R: lists of (nrows, ncols, rowptr, col, val); omega: list of floats."""
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        keep = []
        nl = len(A)
        Aa = (CCsr * nl)(*[_csr_struct(*a, keep) for a in A])
        Pa = (CCsr * max(nl - 1, 1))(*[_csr_struct(*p, keep) for p in P])
        Ra = (CCsr * max(nl - 1, 1))(*[_csr_struct(*r, keep) for r in R])
        om = np.ascontiguousarray(list(omega) + [0.0], dtype=np.float64)
        self._check(self.lib.fsi_set_hierarchy(self.ctx, w, nl, Aa, Pa, Ra, om.ctypes.data))

    def hierarchy_info(self, which):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        nl = ctypes.c_int32()
        n = np.zeros(16, np.int64)
        nnz = np.zeros(16, np.int64)
        om = np.zeros(16, np.float64)
        self._check(self.lib.fsi_hierarchy_info(self.ctx, w, ctypes.byref(nl), n.ctypes.data,
                                                nnz.ctypes.data, om.ctypes.data))
        k = nl.value
        return n[:k].copy(), nnz[:k].copy(), om[:k].copy()

    def spmv_bytes(self) -> float:
        b = ctypes.c_double()
        self._check(self.lib.fsi_spmv_bytes(self.ctx, ctypes.byref(b)))
        return b.value

    def precond_bytes(self) -> float:
        b = ctypes.c_double()
        self._check(self.lib.fsi_precond_bytes(self.ctx, ctypes.byref(b)))
        return b.value

    def vcycle_bytes(self, which) -> float:
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        b = ctypes.c_double()
        self._check(self.lib.fsi_vcycle_bytes(self.ctx, w, ctypes.byref(b)))
        return b.value

    def get_level(self, which, level: int, what: str = "A"):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        wt = {"A": 0, "P": 1}[what]
        nr, nc, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._check(self.lib.fsi_get_level(self.ctx, w, level, wt, ctypes.byref(nr), ctypes.byref(nc),
                                           ctypes.byref(nz), None, None, None))
        rp = np.empty(nr.value + 1, np.int64)
        ci = np.empty(nz.value, np.int32)
        vv = np.empty(nz.value, np.float64)
        self._check(self.lib.fsi_get_level(self.ctx, w, level, wt, None, None, None, rp.ctypes.data,
                                           ci.ctypes.data, vv.ctypes.data))
        return nr.value, nc.value, rp, ci, vv

    def get_aggregates(self, which, level: int):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        cnt = ctypes.c_int64()
        self._check(self.lib.fsi_get_aggregates(self.ctx, w, level, None, ctypes.byref(cnt)))
        a = np.empty(cnt.value, np.int32)
        self._check(self.lib.fsi_get_aggregates(self.ctx, w, level, a.ctypes.data, None))
        return a

    # -- learned smoother ---------------------------------------------------------
    def mlp_set_weights(self, which, W1, W2, W3):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        a = [np.ascontiguousarray(x, dtype=np.float32) for x in (W1, W2, W3)]
        self._check(self.lib.fsi_mlp_set_weights(self.ctx, w, *[x.ctypes.data for x in a]))

    def mlp_get_weights(self, which, k_in: int, d: int):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        a = [np.empty((k_in, 64), np.float32), np.empty((64, 64), np.float32), np.empty((64, d), np.float32)]
        self._check(self.lib.fsi_mlp_get_weights(self.ctx, w, *[x.ctypes.data for x in a]))
        return a

    def mlp_enable(self, which, enable: bool = True):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        self._check(self.lib.fsi_mlp_enable(self.ctx, w, int(enable)))

    def mlp_forward(self, which, b, x=None):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        n = self._hier_len(w)
        if x is None:
            x = self.torch.empty_like(b)
        self._check(self.lib.fsi_mlp_forward(self.ctx, w, _dptr(b, n, "b"), _dptr(x, n, "x")))
        return x

    def mlp_forward_noalloc(self, which, b, x):
        """fsi_mlp_forward_noalloc: the caller provides x; nothing is allocated."""
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        n = self._hier_len(w)
        self._check(self.lib.fsi_mlp_forward_noalloc(self.ctx, w, _dptr(b, n, "b"), _dptr(x, n, "x")))
        return x

    def mlp_loss_grad(self, which, Z, E, wgt, d: int):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        Z = np.ascontiguousarray(Z, dtype=np.float32)
        E = np.ascontiguousarray(E, dtype=np.float32)
        wgt = np.ascontiguousarray(wgt, dtype=np.float32)
        m, k_in = Z.shape
        G = [np.empty((k_in, 64), np.float32), np.empty((64, 64), np.float32), np.empty((64, d), np.float32)]
        loss = ctypes.c_double()
        self._check(self.lib.fsi_mlp_loss_grad(self.ctx, w, m, Z.ctypes.data, E.ctypes.data, wgt.ctypes.data,
                                               *[g.ctypes.data for g in G], ctypes.byref(loss)))
        return loss.value, G

    def mlp_energy_grad(self, which, b, d: int, coarse_cycles: int = 4):
        w = HIERARCHIES[which] if isinstance(which, str) else int(which)
        n = self._hier_len(w)
        k_in = 3 ** d * d
        G = [np.empty((k_in, 64), np.float32), np.empty((64, 64), np.float32), np.empty((64, d), np.float32)]
        loss = ctypes.c_double()
        self._check(self.lib.fsi_mlp_energy_grad(self.ctx, w, _dptr(b, n, "b"), int(coarse_cycles),
                                                 *[g.ctypes.data for g in G], ctypes.byref(loss)))
        return loss.value, G

    def mlp_collect(self, max_vectors: int, every: int = 1):
        self._check(self.lib.fsi_mlp_collect(self.ctx, int(max_vectors), int(every)))

    def mlp_train(self, steps=400, batch=16384, lr=1e-3, exact_tol=1e-10, exact_maxit=300, seed=0,
                  loss="energy", coarse_cycles=4):
        o = CMlpTrainOpts(int(steps), int(batch), float(lr), float(exact_tol), int(exact_maxit), int(seed),
                          MLP_LOSS[loss], int(coarse_cycles))
        info = CMlpTrainInfo()
        self._check(self.lib.fsi_mlp_train(self.ctx, ctypes.byref(o), ctypes.byref(info)))
        return dict(vectors=list(info.vectors), samples=list(info.samples),
                    loss_first=list(info.loss_first), loss_last=list(info.loss_last))
