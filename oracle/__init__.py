"""FP64 CPU oracle for the two-species Shan-Chen lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package (that
leg times the oracle on the benchmark's workloads; the benchmark's precision
study compares the GPU fields with the fields of the leg's 1024^2 run).  It
is the reference the GPU library is checked against and shares no code with
it.

The arithmetic lives in ``lbref.c`` (plain C, FP64, no FMA contraction); this
module only marshals numpy arrays into it.  ``theory.py`` holds the paper's
closed-form results (Secs. III-V) used as pins.

Populations are numpy arrays of shape (2, 9, ny, nx): species (A, B),
D2Q9 direction (rest, +x, +y, -x, -y, (1,1), (-1,1), (-1,-1), (1,-1)), row, column.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbref.c")
_LIB_PATH = os.path.join(_HERE, "liblbref.so")

CFLAGS = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile lbref.c into liblbref.so next to it (gcc)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("walls", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("tau", ctypes.c_double * 2), ("rho0", ctypes.c_double),
                ("Ga", ctypes.c_double * 2), ("Gr", ctypes.c_double * 2), ("Gab", ctypes.c_double),
                ("u_wall", ctypes.c_double), ("g_body", ctypes.c_double),
                ("g_uniform", ctypes.c_double)]


@dataclass
class Params:
    """Model parameters (Sec. II, Eqs. (1), (2), (5)).

    Ga, Gr: intra-species couplings G^a_s (first belt, w-weights) and G^r_s
    (both belts, p-weights); Gab: cross coupling G_AB; rho0: pseudopotential
    scale.  walls: halfway bounce-back walls below row 0 (x-velocity -u_wall)
    and above row ny-1 (+u_wall); x stays periodic.  g_body: amplitude of the
    shear forcing of Sec. VIII, a force rho_s g_body sin(2 pi y / ny) along x
    on each species.  g_uniform: a uniform body force rho_s g_uniform along x
    on each species (between walls: plane Poiseuille flow).
    """
    nx: int
    ny: int
    tau: tuple = (1.0, 1.0)
    rho0: float = 0.83
    Ga: tuple = (-9.0, -9.0)
    Gr: tuple = (8.1, 8.1)
    Gab: float = 0.405
    walls: bool = False
    u_wall: float = 0.0
    g_body: float = 0.0
    g_uniform: float = 0.0

    def c(self) -> _CParams:
        cp = _CParams()
        cp.nx, cp.ny, cp.walls, cp.pad_ = int(self.nx), int(self.ny), int(bool(self.walls)), 0
        cp.tau[0], cp.tau[1] = float(self.tau[0]), float(self.tau[1])
        cp.rho0 = float(self.rho0)
        cp.Ga[0], cp.Ga[1] = float(self.Ga[0]), float(self.Ga[1])
        cp.Gr[0], cp.Gr[1] = float(self.Gr[0]), float(self.Gr[1])
        cp.Gab = float(self.Gab)
        cp.u_wall = float(self.u_wall)
        cp.g_body = float(self.g_body)
        cp.g_uniform = float(self.g_uniform)
        return cp


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_CParams)
        L.lbref_step.argtypes = [pp, dp, dp, dp, dp]
        L.lbref_run.argtypes = [pp, dp, ctypes.c_int64, ctypes.c_int64, dp]
        L.lbref_init_equilibrium.argtypes = [pp, dp, dp, dp, dp, dp]
        L.lbref_fields.argtypes = [pp, dp, dp, dp, dp, dp]
        L.lbref_totals.argtypes = [pp, dp, dp]
        L.lbref_density.argtypes = [pp, dp, dp]
        L.lbref_psi.argtypes = [pp, dp, dp]
        L.lbref_force.argtypes = [pp, dp, dp, dp]
        L.lbref_work_doubles.argtypes = [pp]
        L.lbref_work_doubles.restype = ctypes.c_size_t
        ip = ctypes.POINTER(ctypes.c_int)
        L.lbref_tables.argtypes = [ip, ip, dp, ip, ip, dp, dp]
        L.lbref_max_threads.argtypes = []
        L.lbref_max_threads.restype = ctypes.c_int
        L.lbref_set_threads.argtypes = [ctypes.c_int]
        L.lbref_set_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ctypes.c_double))
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def init_equilibrium(p: Params, rhoA, rhoB, ux=None, uy=None) -> np.ndarray:
    """f_is = f^eq_i(rho_s, u) (zero velocity unless given)."""
    rhoA, rhoB = _f64(rhoA), _f64(rhoB)
    assert rhoA.shape == (p.ny, p.nx) and rhoB.shape == (p.ny, p.nx)
    ux = None if ux is None else _f64(ux)
    uy = None if uy is None else _f64(uy)
    f = np.empty((2, 9, p.ny, p.nx), dtype=np.float64)
    cp = p.c()
    lib().lbref_init_equilibrium(ctypes.byref(cp), _ptr(rhoA), _ptr(rhoB), _ptr(ux), _ptr(uy), _ptr(f))
    return f


def step(p: Params, f: np.ndarray, wall_mom: np.ndarray | None = None) -> np.ndarray:
    """One time step; returns the new populations (f is not modified)."""
    f = _f64(f)
    assert f.shape == (2, 9, p.ny, p.nx)
    out = np.empty_like(f)
    cp = p.c()
    rc = lib().lbref_step(ctypes.byref(cp), _ptr(f), _ptr(out), _ptr(None), _ptr(wall_mom))
    if rc != 0:
        raise MemoryError("oracle step failed")
    return out


def run(p: Params, f: np.ndarray, nsteps: int, avg_from: int | None = None):
    """Advance nsteps steps.  Returns (f, wall_mom) where wall_mom[0:2] is the
    x-momentum handed to the (bottom, top) walls summed over steps
    k >= avg_from (k counted from 0 in this call)."""
    f = _f64(f).copy()
    assert f.shape == (2, 9, p.ny, p.nx)
    wm = np.zeros(2, dtype=np.float64)
    cp = p.c()
    rc = lib().lbref_run(ctypes.byref(cp), _ptr(f), int(nsteps),
                         int(nsteps if avg_from is None else avg_from), _ptr(wm))
    if rc != 0:
        raise MemoryError("oracle run failed")
    return f, wm


def fields(p: Params, f: np.ndarray) -> dict:
    """rho (2,ny,nx), u' (2,ny,nx), u_phys (2,ny,nx), F (2,2,ny,nx) at time t."""
    f = _f64(f)
    n = p.nx * p.ny
    rho = np.empty((2, p.ny, p.nx))
    u = np.empty((2, p.ny, p.nx))
    uphys = np.empty((2, p.ny, p.nx))
    F = np.empty((2, 2, p.ny, p.nx))
    cp = p.c()
    rc = lib().lbref_fields(ctypes.byref(cp), _ptr(f), _ptr(rho), _ptr(u), _ptr(uphys), _ptr(F))
    if rc != 0:
        raise MemoryError
    assert rho.size == 2 * n
    return {"rho": rho, "u": u, "uphys": uphys, "F": F}


def totals(p: Params, f: np.ndarray) -> dict:
    """Global sums of the state: mass[2], mom[2], mom_phys[2], pxy_kin, the
    first sine mode u_mode of the line-averaged x-velocity (R(t) times U0,
    Sec. VIII Eq. (66)) and the interface indicator i_ab (Eq. (67))."""
    f = _f64(f)
    out = np.zeros(9)
    cp = p.c()
    rc = lib().lbref_totals(ctypes.byref(cp), _ptr(f), _ptr(out))
    if rc != 0:
        raise MemoryError
    return {"mass": out[0:2].copy(), "mom": out[2:4].copy(), "mom_phys": out[4:6].copy(),
            "pxy_kin": float(out[6]), "u_mode": float(out[7]), "i_ab": float(out[8])}


def density(p: Params, f: np.ndarray) -> np.ndarray:
    f = _f64(f)
    rho = np.empty((2, p.ny, p.nx))
    cp = p.c()
    lib().lbref_density(ctypes.byref(cp), _ptr(f), _ptr(rho))
    return rho


def force(p: Params, rho: np.ndarray) -> np.ndarray:
    """Forces (2 species, 2 components, ny, nx) of a given density field."""
    rho = _f64(rho)
    assert rho.shape == (2, p.ny, p.nx)
    psi = np.empty_like(rho)
    F = np.empty((2, 2, p.ny, p.nx))
    cp = p.c()
    lib().lbref_psi(ctypes.byref(cp), _ptr(rho), _ptr(psi))
    lib().lbref_force(ctypes.byref(cp), _ptr(rho), _ptr(psi), _ptr(F))
    return F


def tables() -> dict:
    """The oracle's lattice tables: D2Q9 (cx, cy, w) and the 25-speed
    interaction set (ex, ey, p, w)."""
    ci = (ctypes.c_int * 9)()
    cyi = (ctypes.c_int * 9)()
    wq = (ctypes.c_double * 9)()
    ex = (ctypes.c_int * 25)()
    ey = (ctypes.c_int * 25)()
    pe = (ctypes.c_double * 25)()
    we = (ctypes.c_double * 25)()
    lib().lbref_tables(ci, cyi, wq, ex, ey, pe, we)
    return {"cx": list(ci), "cy": list(cyi), "wq": list(wq), "ex": list(ex), "ey": list(ey),
            "p": list(pe), "w": list(we)}


def max_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().lbref_max_threads())


def set_threads(n: int) -> None:
    """Set the oracle's OpenMP thread count (n > 0)."""
    lib().lbref_set_threads(int(n))
