"""ctypes wrapper of the plain FP64 CPU oracle (oracle/mrp_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py, never by the product package.  It shares no
code with the HIP library; both sides only receive the same seeded inputs.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB, build as build_library

M_FULL, M_AXISYM = 0, 1
BC_ABSORB, BC_SPECULAR, BC_DIFFUSE = 0, 1, 2


class _Params(C.Structure):
    _fields_ = [
        ("d", C.c_double), ("eps_r", C.c_double), ("r_out", C.c_double), ("dt", C.c_double),
        ("ntilde", C.c_double), ("ion_density", C.c_double),
        ("l_max", C.c_int32), ("m_mode", C.c_int32), ("probe_bc", C.c_int32),
        ("wall_bc", C.c_int32), ("seed", C.c_uint64),
        ("ion_prof", C.POINTER(C.c_double)), ("ion_prof_len", C.c_int64),
        ("ion_mass", C.c_double),
    ]


@dataclass
class Params:
    d: float = 0.25
    eps_r: float = 4.0
    r_out: float = 5.0
    dt: float = 0.05
    ntilde: float = 1.0
    ion_density: float = 1.0
    l_max: int = 8
    m_mode: int = M_FULL
    probe_bc: int = BC_ABSORB
    wall_bc: int = BC_SPECULAR
    seed: int = 0
    ion_profile: np.ndarray | None = None   # density at equally spaced radii 1..r_out
    ion_mass: float = 0.0                   # m_i / m_e of ids with bit 31 set (ions)

    def _c(self) -> _Params:
        prof, plen = None, 0
        if self.ion_profile is not None:
            self._prof = np.ascontiguousarray(self.ion_profile, dtype=np.float64)
            if self._prof.ndim != 1 or self._prof.size < 2:
                raise ValueError("ion_profile needs at least 2 nodes")
            prof, plen = self._prof.ctypes.data_as(C.POINTER(C.c_double)), self._prof.size
        return _Params(self.d, self.eps_r, self.r_out, self.dt, self.ntilde, self.ion_density,
                       self.l_max, self.m_mode, self.probe_bc, self.wall_bc, self.seed, prof, plen,
                       self.ion_mass)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_library()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        P = C.POINTER(_Params)
        L.orc_coeffs.argtypes = [C.c_double, C.c_double, C.c_int, dp, dp, dp]
        L.orc_ion_field.argtypes = [P, C.c_double, dp]
        L.orc_ion_field.restype = C.c_double
        L.orc_greens.argtypes = [P, dp, dp, C.c_int, dp, dp]
        L.orc_psi_anti.argtypes = [P, dp, dp, dp]
        L.orc_field.argtypes = [P, C.c_int64, dp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint8),
                                C.c_double, C.c_double, C.c_int64, C.POINTER(C.c_int64), dp, dp]
        L.orc_qdiff.argtypes = [P, C.c_int64, dp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint8)]
        L.orc_qdiff.restype = C.c_double
        L.orc_run.argtypes = [P, C.c_int64, dp, dp, C.POINTER(C.c_uint32), C.POINTER(C.c_uint8),
                              dp, dp, C.c_int64, C.c_int64, dp]
        L.orc_run.restype = C.c_int64
        L.orc_energy.argtypes = [P, C.c_int64, dp, dp, C.POINTER(C.c_uint32),
                                 C.POINTER(C.c_uint8), C.c_double, C.c_double, dp, dp]
        L.orc_energy.restype = C.c_double
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        L.orc_diffuse_dir.argtypes = [C.c_uint64, C.c_uint32, C.c_int64, C.c_int, dp, dp]
        L.orc_diffuse_dir.restype = None
        L.orc_philox4x64_10.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_uint64)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def coeffs(eps_r: float, d: float, l_max: int):
    """(f_l, b^P_l, c_l) for l = 0..l_max."""
    f = np.zeros(l_max + 1)
    b = np.zeros(l_max + 1)
    c = np.zeros(l_max + 1)
    lib().orc_coeffs(eps_r, d, l_max, _dp(f), _dp(b), _dp(c))
    return f, b, c


def greens(p: Params, x, y, x_outer: bool | None = None):
    """G~_L(x, y) and its gradient in x."""
    x = _f64(x, 3)
    y = _f64(y, 3)
    if x_outer is None:
        x_outer = float(np.dot(x, x)) > float(np.dot(y, y))
    G = C.c_double()
    g = np.zeros(3)
    pc = p._c()
    rc = lib().orc_greens(C.byref(pc), _dp(x), _dp(y), int(bool(x_outer)), C.byref(G), _dp(g))
    if rc != 0:
        raise ValueError("oracle: l_max out of range")
    return G.value, g


def psi_anti(p: Params, x):
    x = _f64(x, 3)
    psi = C.c_double()
    g = np.zeros(3)
    pc = p._c()
    lib().orc_psi_anti(C.byref(pc), _dp(x), C.byref(psi), _dp(g))
    return psi.value, g


def _alive_arr(alive, n):
    if alive is None:
        return np.ones(n, dtype=np.uint8)
    return np.ascontiguousarray(alive, dtype=np.uint8)


def field(p: Params, pos, ids=None, alive=None, q_surface: float = 0.0, u_asy: float = 0.0,
          targets=None):
    """Field E (and potential without self term) at every particle or at `targets`."""
    pos = _f64(pos)
    n = pos.shape[0]
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, np.uint32)
    al = _alive_arr(alive, n)
    if targets is None:
        nt, tp = n, None
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = t.shape[0], t.ctypes.data_as(C.POINTER(C.c_int64))
    E = np.zeros((nt, 3))
    phi = np.zeros(nt)
    pc = p._c()
    rc = lib().orc_field(C.byref(pc), n, _dp(pos), ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                         al.ctypes.data_as(C.POINTER(C.c_uint8)), q_surface, u_asy, nt, tp,
                         _dp(E), _dp(phi))
    if rc != 0:
        raise ValueError("oracle: l_max out of range")
    return E, phi


def ion_field(p: Params, r: float) -> tuple:
    """(E_r, Phi) of the immobile ion background at radius r."""
    phi = C.c_double()
    pc = p._c()
    e = lib().orc_ion_field(C.byref(pc), float(r), C.byref(phi))
    return e, phi.value


def qdiff(p: Params, pos, alive=None, ids=None) -> float:
    pos = _f64(pos)
    al = _alive_arr(alive, pos.shape[0])
    idp = None
    if ids is not None:
        ids = np.ascontiguousarray(ids, np.uint32)
        idp = ids.ctypes.data_as(C.POINTER(C.c_uint32))
    pc = p._c()
    return lib().orc_qdiff(C.byref(pc), pos.shape[0], _dp(pos), idp,
                           al.ctypes.data_as(C.POINTER(C.c_uint8)))


@dataclass
class RunResult:
    pos: np.ndarray
    vel: np.ndarray
    alive: np.ndarray
    q_surface: float
    qdiff: np.ndarray
    absorbed: int


def run(p: Params, pos, vel, u_asy, n_steps: int, ids=None, alive=None, q_surface: float = 0.0,
        start_step: int = 0) -> RunResult:
    """Leapfrog for n_steps from absolute step start_step; inputs are copied."""
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    n = pos.shape[0]
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, np.uint32)
    al = _alive_arr(alive, n).copy()
    u = _f64(u_asy)
    if u.shape[0] < start_step + n_steps:
        raise ValueError("u_asy shorter than start_step + n_steps")
    qd = np.zeros(u.shape[0])
    qs = C.c_double(q_surface)
    pc = p._c()
    tot = lib().orc_run(C.byref(pc), n, _dp(pos), _dp(vel),
                        ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                        al.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(qs), _dp(u),
                        start_step, n_steps, _dp(qd))
    if tot < 0:
        raise ValueError("oracle run failed")
    return RunResult(pos, vel, al, qs.value, qd[start_step:start_step + n_steps], int(tot))


def energy(p: Params, pos, v2, ids=None, alive=None, q_surface: float = 0.0, u_asy: float = 0.0):
    """(H, kinetic, potential) with per-particle v.v supplied by the caller."""
    pos = _f64(pos)
    n = pos.shape[0]
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, np.uint32)
    al = _alive_arr(alive, n)
    v2 = _f64(v2)
    ke = C.c_double()
    pe = C.c_double()
    pc = p._c()
    h = lib().orc_energy(C.byref(pc), n, _dp(pos), _dp(v2),
                         ids.ctypes.data_as(C.POINTER(C.c_uint32)),
                         al.ctypes.data_as(C.POINTER(C.c_uint8)), q_surface, u_asy,
                         C.byref(ke), C.byref(pe))
    return h, ke.value, pe.value


def philox4x64_10(counter, key):
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    P = C.POINTER(C.c_uint64)
    lib().orc_philox4x64_10(c.ctypes.data_as(P), k.ctypes.data_as(P), o.ctypes.data_as(P))
    return o


def diffuse_dir(seed: int, pid: int, step: int, wall: int, normal):
    """Direction the diffuse wall rule gives a particle (id, step) reflected
    at `wall` (0 probe, 1 outer wall) with inward unit normal `normal`."""
    n = _f64(normal, 3)
    d = np.zeros(3)
    lib().orc_diffuse_dir(int(seed), int(pid), int(step), int(wall), _dp(n), _dp(d))
    return d


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())
