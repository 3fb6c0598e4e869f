"""Seeded synthetic inputs: linearised monolithic ALE-FSI Jacobians.

This module is the only code shared by the CPU oracle and the GPU library's
tests and benchmark.  It holds no part of the linear solver: it assembles, on
structured channels, the 3x3 block matrix A_h of the paper's Section 3.4
(blocks M, C_ms, C_sm, S, C_sf, C_fm, C_fs, F; unknowns ordered mesh, solid,
fluid) and the Newton right-hand side, from the variational ALE-FSI equations
of Section 3 (Q2 velocity and displacement, Q1 pressure, Backward Euler).

The native assembler lives in ``csrc/fsigen.cpp`` and is built by
:func:`build` into ``libfsigen.so`` next to this file.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libfsigen.so")
_SRC = os.path.join(_HERE, "csrc", "fsigen.cpp")

BLOCK_NAMES = ("M", "C_ms", "C_sm", "S", "C_sf", "C_fm", "C_fs", "F")


def build(force: bool = True) -> str:
    """Compile the assembler with g++ (host code only, portable x86-64)."""
    if force or not os.path.exists(_SO):
        cmd = ["g++", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", _SO + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32),
        ("nc", ctypes.c_int32 * 3),
        ("L", ctypes.c_double * 3),
        ("solid_lo", ctypes.c_int32 * 3),
        ("solid_hi", ctypes.c_int32 * 3),
        ("rho_f", ctypes.c_double),
        ("nu_f", ctypes.c_double),
        ("rho_s", ctypes.c_double),
        ("mu_s", ctypes.c_double),
        ("lambda_s", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("v_peak", ctypes.c_double),
        ("u_peak", ctypes.c_double),
        ("p_amp", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("t_phase", ctypes.c_double),
        ("newton_mesh", ctypes.c_int32),
        ("pad", ctypes.c_int32),
    ]


@dataclasses.dataclass(frozen=True)
class Config:
    """Grid, solid placement and material data of one synthetic workload."""

    name: str
    dim: int
    cells: tuple
    extent: tuple
    solid_lo: tuple
    solid_hi: tuple
    rho_f: float = 1e3
    nu_f: float = 1e-3
    rho_s: float = 1e4
    mu_s: float = 5e5
    lambda_s: float = 2e6
    dt: float = 1e-2
    theta: float = 1.0
    v_peak: float = 1.0
    p_amp: float = 10.0
    u_frac: float = 0.05   # peak displacement as a fraction of the solid thickness
    newton_mesh: int = 0

    @property
    def solid_thickness(self) -> float:
        h = self.extent[1] / self.cells[1]
        return (self.solid_hi[1] - self.solid_lo[1]) * h

    def with_(self, **kw) -> "Config":
        return dataclasses.replace(self, **kw)


# Material values follow the paper's FSI-2 tables (fluid density 1e3,
# viscosity 1e-3, solid density 1e4, Lame mu 0.5e6, lambda 2e6); time step
# 1e-2 with theta = 1.
CONFIGS = {
    "tiny2d": Config("tiny2d", 2, (4, 2), (2.0, 0.5), (1, 0), (3, 1)),
    "tiny3d": Config("tiny3d", 3, (4, 2, 2), (2.5, 0.41, 0.41), (1, 0, 0), (3, 1, 1)),
    "c1": Config("c1", 2, (32, 8), (2.0, 0.5), (12, 0), (20, 2)),
    "c2": Config("c2", 2, (256, 64), (2.0, 0.5), (96, 0), (160, 16)),
    "m3": Config("m3", 3, (32, 8, 8), (2.5, 0.41, 0.41), (8, 0, 2), (16, 1, 6)),
    "c3": Config("c3", 3, (64, 16, 16), (2.5, 0.41, 0.41), (16, 0, 4), (32, 2, 12)),
    "c4": Config("c4", 3, (128, 32, 32), (2.5, 0.41, 0.41), (32, 0, 8), (64, 4, 24)),
}

# Unit-parameter variants keep the block scales comparable (small condition
# numbers), for brute-force comparisons at tight tolerances.
UNIT = dict(rho_f=1.0, nu_f=1.0, rho_s=1.0, mu_s=1.0, lambda_s=1.0, dt=1.0)


def config(name: str, **overrides) -> Config:
    base = name
    unit = False
    if name.endswith("_unit"):
        base, unit = name[: -len("_unit")], True
    cfg = CONFIGS[base]
    if unit:
        cfg = cfg.with_(name=name, **UNIT)
    if overrides:
        cfg = cfg.with_(**overrides)
    return cfg


def _ccfg(cfg: Config, seed: int, t_phase: float) -> _Cfg:
    c = _Cfg()
    c.dim = cfg.dim
    for a in range(3):
        c.nc[a] = cfg.cells[a] if a < cfg.dim else 1
        c.L[a] = cfg.extent[a] if a < cfg.dim else 1.0
        c.solid_lo[a] = cfg.solid_lo[a] if a < cfg.dim else 0
        c.solid_hi[a] = cfg.solid_hi[a] if a < cfg.dim else 1
    c.rho_f, c.nu_f, c.rho_s = cfg.rho_f, cfg.nu_f, cfg.rho_s
    c.mu_s, c.lambda_s, c.dt, c.theta = cfg.mu_s, cfg.lambda_s, cfg.dt, cfg.theta
    c.v_peak, c.p_amp = cfg.v_peak, cfg.p_amp
    c.u_peak = cfg.u_frac * cfg.solid_thickness
    c.seed = int(seed)
    c.t_phase = float(t_phase)
    c.newton_mesh = int(cfg.newton_mesh)
    return c


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        lib.fsigen_build.argtypes = [P(_Cfg), P(ctypes.c_void_p), ctypes.c_char_p, ctypes.c_int]
        lib.fsigen_build.restype = ctypes.c_int
        lib.fsigen_sizes.argtypes = [ctypes.c_void_p, P(ctypes.c_int64)]
        lib.fsigen_block_sizes.argtypes = [ctypes.c_void_p, ctypes.c_int, P(ctypes.c_int64)]
        lib.fsigen_block_copy.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.fsigen_rhs.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.fsigen_nodes.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 5
        lib.fsigen_jrange.argtypes = [ctypes.c_void_p, P(ctypes.c_double)]
        lib.fsigen_free.argtypes = [ctypes.c_void_p]
        lib.fsigen_fe_data.argtypes = [ctypes.c_void_p] * 11
        lib.fsigen_residual.argtypes = [P(_Cfg), ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_char_p, ctypes.c_int]
        lib.fsigen_residual.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclasses.dataclass
class Csr:
    """Plain CSR arrays: int64 row pointers, int32 columns, float64 values."""

    nrows: int
    ncols: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


@dataclasses.dataclass
class FsiSystem:
    """One linearised FSI system A_h x = b with its block layout."""

    cfg: Config
    seed: int
    t_phase: float
    dim: int
    n_m: int
    n_s: int
    n_f: int
    n_vs: int
    n_vf: int
    n_p: int
    blocks: dict            # name -> Csr, names as in BLOCK_NAMES
    b: np.ndarray           # Newton right-hand side -R(U_bar)
    coords: np.ndarray      # (nnodes, dim) node coordinates
    node_ijk: np.ndarray    # (nnodes, dim) lattice index (Q2 lattice)
    node_flags: np.ndarray  # bit0 solid, bit1 fluid, bit2 v-Dirichlet, bit3 u-Dirichlet
    dof_node: np.ndarray    # (N,) node id of every dof
    dof_comp: np.ndarray    # (N,) vector component of every dof (0 for p)
    j_range: tuple
    fe: dict = None         # finite-element description (generate(..., fe=True)), see FE_FIELDS

    @property
    def N(self) -> int:
        return self.n_m + self.n_s + self.n_f

    @property
    def dt_theta(self) -> float:
        return self.cfg.dt * self.cfg.theta

    @property
    def nnz(self) -> int:
        return sum(b.nnz for b in self.blocks.values())

    @property
    def offsets(self) -> tuple:
        return (0, self.n_m, self.n_m + self.n_s, self.N)


# Finite-element description of a workload (node arrays on the Q2 lattice,
# nodes numbered row-major with axis 0 slowest): first velocity dof, first
# displacement dof and pressure dof of every node (-1: none), the linearisation
# state v, u, p (also the Dirichlet data on constrained dofs), the previous time
# level v_old, u_old, the advecting velocity w of the convective term and the
# displacement u_fz whose Jacobian determinant scales the mesh stiffness.
FE_FIELDS = ("vdof", "udof", "pdof", "v", "u", "p", "v_old", "u_old", "w", "u_fz")


def generate(name_or_cfg, seed: int = 0, t_phase: float = 0.0, fe: bool = False) -> FsiSystem:
    """Assemble the seeded system for a configuration (name or Config).

    With ``fe`` the system also carries its finite-element description
    (``FsiSystem.fe``, keys FE_FIELDS), for assembling residual and Jacobian
    elsewhere."""
    cfg = config(name_or_cfg) if isinstance(name_or_cfg, str) else name_or_cfg
    lib = _load()
    c = _ccfg(cfg, seed, t_phase)
    h = ctypes.c_void_p()
    err = ctypes.create_string_buffer(512)
    rc = lib.fsigen_build(ctypes.byref(c), ctypes.byref(h), err, 512)
    if rc != 0:
        raise RuntimeError(f"fsigen: {err.value.decode()}")
    try:
        s = np.zeros(9, np.int64)
        lib.fsigen_sizes(h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        dim, nnodes, N, n_m, n_s, n_f, n_vs, n_vf, n_p = (int(x) for x in s)
        blocks = {}
        for i, name in enumerate(BLOCK_NAMES):
            bs = np.zeros(3, np.int64)
            lib.fsigen_block_sizes(h, i, bs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
            nr, ncl, nnz = (int(x) for x in bs)
            rp = np.empty(nr + 1, np.int64)
            cl = np.empty(nnz, np.int32)
            vl = np.empty(nnz, np.float64)
            lib.fsigen_block_copy(h, i, rp.ctypes.data, cl.ctypes.data, vl.ctypes.data)
            blocks[name] = Csr(nr, ncl, rp, cl, vl)
        b = np.empty(N, np.float64)
        lib.fsigen_rhs(h, b.ctypes.data)
        coords = np.empty((nnodes, dim), np.float64)
        ijk = np.empty((nnodes, dim), np.int32)
        flags = np.empty(nnodes, np.uint8)
        dof_node = np.empty(N, np.int32)
        dof_comp = np.empty(N, np.int8)
        lib.fsigen_nodes(h, coords.ctypes.data, ijk.ctypes.data, flags.ctypes.data,
                         dof_node.ctypes.data, dof_comp.ctypes.data)
        jr = (ctypes.c_double * 2)()
        lib.fsigen_jrange(h, jr)
        fed = None
        if fe:
            fed = {k: np.empty(nnodes, np.int64) for k in ("vdof", "udof", "pdof")}
            fed["p"] = np.empty(nnodes, np.float64)
            for k in ("v", "u", "v_old", "u_old", "w", "u_fz"):
                fed[k] = np.empty((nnodes, dim), np.float64)
            lib.fsigen_fe_data(h, *(fed[k].ctypes.data for k in FE_FIELDS))
    finally:
        lib.fsigen_free(h)
    return FsiSystem(cfg, seed, t_phase, dim, n_m, n_s, n_f, n_vs, n_vf, n_p, blocks, b,
                     coords, ijk, flags, dof_node, dof_comp, (jr[0], jr[1]), fed)


def residual(name_or_cfg, seed: int, direction: np.ndarray, eps: float, t_phase: float = 0.0) -> np.ndarray:
    """R(U_bar + eps * direction) on the free dofs, frozen fields held at U_bar."""
    cfg = config(name_or_cfg) if isinstance(name_or_cfg, str) else name_or_cfg
    lib = _load()
    c = _ccfg(cfg, seed, t_phase)
    d = np.ascontiguousarray(direction, np.float64)
    out = np.empty_like(d)
    err = ctypes.create_string_buffer(512)
    rc = lib.fsigen_residual(ctypes.byref(c), d.ctypes.data, float(eps), out.ctypes.data,
                             int(d.shape[0]), err, 512)
    if rc != 0:
        raise RuntimeError(f"fsigen: {err.value.decode()}")
    return out


def pseudo_time_phase(step: int, solve: int, dt: float = 1e-2, period: float = 0.5) -> float:
    """Phase angle of pseudo-time step `step`, Newton solve `solve` in {0,1,2}."""
    t = step * dt + solve * dt / 3.0
    return 2.0 * math.pi * t / period


def smooth_vector(sysm: FsiSystem, seed: int) -> np.ndarray:
    """A seeded smooth-ish test vector on the free dofs (for manufactured RHS)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(sysm.N)
    return x
