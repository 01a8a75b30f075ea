"""Thin ctypes binding of libmrpsim.so (C ABI in include/mrpsim.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of csrc/mrpsim.hip.  There is no CPU fallback; if the library is not
built this module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from .build import LIB

SIM_OK, SIM_EINVAL, SIM_ENOMEM, SIM_ERANGE, SIM_ESTATE, SIM_EDEVICE = 0, -1, -2, -3, -4, -5
SIM_BUSY = 1   # sim_query: work still running
SIM_M_FULL, SIM_M_AXISYM = 0, 1
SIM_BC_ABSORB, SIM_BC_SPECULAR, SIM_BC_DIFFUSE = 0, 1, 2
SIM_FP64, SIM_FP32_COMP = 0, 1
# A member occupies whole groups of this many particle slots (four tiles of 64).
SLOT_GROUP = 256

# Every function include/mrpsim.h declares.
EXPORTED = ("sim_params_default", "sim_create", "sim_step", "sim_sync", "sim_query",
            "sim_read_response",
            "sim_read_state", "sim_eval_field", "sim_profile", "sim_num_kernels",
            "sim_kernel_name", "sim_footprint_bytes", "sim_info", "sim_destroy",
            "sim_strerror", "sim_last_error", "sim_member_default", "sim_batch_create",
            "sim_batch_footprint_bytes", "sim_batch_add", "sim_batch_remove", "sim_batch_step",
            "sim_member_info", "sim_member_read_response", "sim_member_read_state",
            "sim_member_eval_field", "sim_member_data_bytes", "sim_member_counts",
            "sim_eval_field_static", "sim_eval_field_static_bytes")


# sim_allocator callbacks: alloc(ctx, bytes, stream) -> device pointer or NULL;
# free(ctx, ptr, bytes, stream)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)


class sim_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class Allocator:
    """A sim_allocator from two Python callables (kept alive with it):
    alloc(nbytes, stream_handle) -> int device pointer (0 on failure) and
    free(ptr, nbytes, stream_handle)."""

    def __init__(self, alloc, free):
        def _a(ctx, nbytes, stream):
            try:
                return int(alloc(int(nbytes), int(stream or 0))) or None
            except Exception:
                return None

        def _f(ctx, ptr, nbytes, stream):
            free(int(ptr), int(nbytes), int(stream or 0))

        self._a, self._f = ALLOC_FN(_a), FREE_FN(_f)
        self.c = sim_allocator(self._a, self._f, None)


def torch_allocator() -> Allocator:
    """Device memory from torch's caching allocator (current device), on the
    handle's stream (stream 0: the handle's own stream, which torch does not
    know; the block is then kept on torch's default stream)."""

    def alloc(nbytes, stream):
        import torch
        return torch.cuda.caching_allocator_alloc(nbytes, torch.cuda.current_device(), stream)

    def free(ptr, nbytes, stream):
        import torch
        torch.cuda.caching_allocator_delete(ptr)

    return Allocator(alloc, free)


def _allocator(spec):
    """None or "hip": hipMalloc inside the library; "torch": torch's caching
    allocator; or an Allocator."""
    if spec is None or spec == "hip":
        return None
    if spec == "torch":
        return torch_allocator()
    if isinstance(spec, Allocator):
        return spec
    raise ValueError(f"unknown allocator {spec!r}")


class sim_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("reserved0", C.c_uint32),
        ("d", C.c_double), ("eps_r", C.c_double), ("r_out", C.c_double), ("dt", C.c_double),
        ("ntilde", C.c_double), ("ion_density", C.c_double), ("q_surface0", C.c_double),
        ("l_max", C.c_int32), ("m_mode", C.c_int32), ("probe_bc", C.c_int32),
        ("wall_bc", C.c_int32), ("precision", C.c_int32), ("tile", C.c_int32),
        ("seed", C.c_uint64), ("mem_limit_bytes", C.c_uint64),
        ("sort_bucket", C.c_int32), ("carry_chunk", C.c_int32),
        ("sort_keys", C.c_int32), ("near_split", C.c_int32),
    ]


class sim_member(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("reserved0", C.c_uint32), ("n", C.c_int64),
        ("pos", C.POINTER(C.c_double)), ("vel", C.POINTER(C.c_double)),
        ("ids", C.POINTER(C.c_uint32)), ("u_asy", C.POINTER(C.c_double)),
        ("n_steps", C.c_int64), ("start_step", C.c_int64),
        ("ntilde", C.c_double), ("ion_density", C.c_double), ("q_surface0", C.c_double),
        ("r_out", C.c_double), ("dt", C.c_double), ("seed", C.c_uint64),
        ("probe_bc", C.c_int32), ("wall_bc", C.c_int32),
        ("ion_profile", C.POINTER(C.c_double)), ("ion_profile_len", C.c_int64),
        ("ion_mass", C.c_double),
    ]


class SimError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (status {code})")
        self.code = code


_lib = None


def lib():
    """Load libmrpsim.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        raise ImportError(f"{LIB} is not built; run __graft_entry__.build() first")
    # The library links the HIP runtime by soname.  Load torch first so the
    # process holds a single HIP runtime (torch's), shared with torch's
    # device memory and streams.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB)
    dp = C.POINTER(C.c_double)
    P = C.POINTER(sim_params)
    H = C.c_void_p
    L.sim_params_default.argtypes = [P]
    L.sim_params_default.restype = None
    A = C.POINTER(sim_allocator)
    L.sim_create.argtypes = [P, C.c_int64, dp, dp, C.POINTER(C.c_uint32), dp, C.c_int64,
                             C.c_int64, C.c_void_p, A, C.POINTER(C.c_void_p)]
    L.sim_step.argtypes = [H, C.c_int64]
    L.sim_sync.argtypes = [H]
    L.sim_query.argtypes = [H]
    L.sim_read_response.argtypes = [H, C.c_int64, C.c_int64, dp]
    L.sim_read_state.argtypes = [H, dp, dp, C.POINTER(C.c_uint8), dp, C.POINTER(C.c_int64)]
    L.sim_eval_field.argtypes = [H, dp]
    L.sim_profile.argtypes = [H, C.c_int64, dp, C.c_int32]
    L.sim_num_kernels.argtypes = []
    L.sim_num_kernels.restype = C.c_int32
    L.sim_kernel_name.argtypes = [C.c_int32]
    L.sim_kernel_name.restype = C.c_char_p
    L.sim_footprint_bytes.argtypes = [P, C.c_int64, C.c_int64]
    L.sim_footprint_bytes.restype = C.c_int64
    L.sim_info.argtypes = [H, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.sim_destroy.argtypes = [H]
    L.sim_destroy.restype = None
    L.sim_strerror.argtypes = [C.c_int]
    L.sim_strerror.restype = C.c_char_p
    L.sim_last_error.argtypes = []
    L.sim_last_error.restype = C.c_char_p
    M = C.POINTER(sim_member)
    i32p, i64p = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.sim_member_default.argtypes = [M]
    L.sim_member_default.restype = None
    L.sim_batch_create.argtypes = [P, C.c_int64, C.c_int32, C.c_int64, C.c_int32, M,
                                   C.c_void_p, A, C.POINTER(C.c_void_p)]
    L.sim_batch_footprint_bytes.argtypes = [P, C.c_int64, C.c_int32, C.c_int64]
    L.sim_batch_footprint_bytes.restype = C.c_int64
    L.sim_member_data_bytes.argtypes = [C.c_int64, C.c_int64]
    L.sim_member_data_bytes.restype = C.c_int64
    L.sim_batch_add.argtypes = [H, M, i32p]
    L.sim_batch_remove.argtypes = [H, C.c_int32]
    L.sim_batch_step.argtypes = [H, C.c_int64]
    L.sim_member_info.argtypes = [H, C.c_int32, i64p, i64p, i64p]
    L.sim_member_read_response.argtypes = [H, C.c_int32, C.c_int64, C.c_int64, dp]
    L.sim_member_read_state.argtypes = [H, C.c_int32, dp, dp, C.POINTER(C.c_uint8), dp, i64p]
    L.sim_member_eval_field.argtypes = [H, C.c_int32, dp]
    L.sim_member_counts.argtypes = [H, C.c_int32, i64p, i64p, i64p]
    L.sim_eval_field_static.argtypes = [P, C.c_int64, C.c_void_p, C.c_double, C.c_double,
                                        C.c_void_p, C.c_void_p]
    L.sim_eval_field_static_bytes.argtypes = [P, C.c_int64]
    L.sim_eval_field_static_bytes.restype = C.c_int64
    for name in EXPORTED:
        if name not in ("sim_params_default", "sim_num_kernels", "sim_kernel_name",
                        "sim_footprint_bytes", "sim_destroy", "sim_strerror", "sim_last_error",
                        "sim_member_default", "sim_batch_footprint_bytes",
                        "sim_member_data_bytes", "sim_eval_field_static_bytes"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != SIM_OK:
        L = lib()
        raise SimError(rc, f"{L.sim_strerror(rc).decode()}: {L.sim_last_error().decode()}")


@dataclass
class SimParams:
    d: float = 0.25
    eps_r: float = 4.0
    r_out: float = 5.0
    dt: float = 0.05
    ntilde: float = 1.0
    ion_density: float = 1.0
    q_surface0: float = 0.0
    l_max: int = 8
    m_mode: int = SIM_M_FULL
    probe_bc: int = SIM_BC_ABSORB
    wall_bc: int = SIM_BC_SPECULAR
    precision: int = SIM_FP64
    tile: int = 0
    seed: int = 0
    mem_limit_bytes: int = 0
    # launch sizes chosen by paper_2111_13072_amd.tune (0: built-in choice)
    sort_bucket: int = 0
    carry_chunk: int = 0
    # where the sort keys are taken: 1 push, -1 own pass, 0 by launch size
    sort_keys: int = 0
    # near-field block: 1 half tiles (32), -1 whole tiles (64), 0 by member
    near_split: int = 0

    def to_c(self) -> sim_params:
        p = sim_params()
        lib().sim_params_default(C.byref(p))
        for f, _ in sim_params._fields_:
            if f in ("struct_size", "reserved0"):
                continue
            setattr(p, f, getattr(self, f))
        return p


def footprint_bytes(params: SimParams, n: int, n_steps: int) -> int:
    p = params.to_c()
    v = lib().sim_footprint_bytes(C.byref(p), n, n_steps)
    if v < 0:
        _check(int(v))
    return int(v)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _counts(handle, index: int) -> dict:
    a, b, st = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().sim_member_counts(handle, index, C.byref(a), C.byref(b), C.byref(st)))
    return dict(alive=a.value, absorbed=b.value, step=st.value)


def _current_torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Sim:
    """One simulation handle (sim_create ... sim_destroy).  Its device memory
    comes from `allocator`: "torch" (torch's caching allocator, the default),
    "hip" (hipMalloc inside the library) or an Allocator."""

    def __init__(self, params: SimParams, pos, vel, u_asy, ids=None, start_step: int = 0,
                 stream=None, use_torch_stream: bool = True, allocator="torch"):
        L = lib()
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        u = np.ascontiguousarray(u_asy, dtype=np.float64)
        n = pos.shape[0]
        if pos.shape != (n, 3) or vel.shape != (n, 3):
            raise ValueError("pos and vel must have shape [n, 3]")
        self.n = n
        self.n_steps = u.shape[0]
        self._ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
        idp = None if self._ids is None else self._ids.ctypes.data_as(C.POINTER(C.c_uint32))
        if stream is None and use_torch_stream:
            stream = _current_torch_stream()
        self._p = params.to_c()
        self._alloc = _allocator(allocator)
        h = C.c_void_p()
        rc = L.sim_create(C.byref(self._p), n, _dp(pos), _dp(vel), idp,
                          _dp(u) if u.size else None, self.n_steps, start_step, stream,
                          C.byref(self._alloc.c) if self._alloc else None, C.byref(h))
        _check(rc)
        self._h = h

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().sim_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if not getattr(self, "_h", None):
            raise SimError(SIM_ESTATE, "simulation is closed")
        return self._h

    # -- calls -------------------------------------------------------------
    def step(self, k: int = 1):
        _check(lib().sim_step(self._handle(), k))

    def sync(self):
        _check(lib().sim_sync(self._handle()))

    def query(self) -> bool:
        """True when all enqueued work has completed (does not wait)."""
        rc = lib().sim_query(self._handle())
        if rc == SIM_BUSY:
            return False
        _check(rc)
        return True

    def read_response(self, first: int, count: int) -> np.ndarray:
        out = np.zeros(count)
        _check(lib().sim_read_response(self._handle(), first, count, _dp(out)))
        return out

    def read_state(self) -> dict:
        pos = np.zeros((self.n, 3))
        vel = np.zeros((self.n, 3))
        alive = np.zeros(self.n, dtype=np.uint8)
        qs = C.c_double()
        st = C.c_int64()
        _check(lib().sim_read_state(self._handle(), _dp(pos), _dp(vel),
                                    alive.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(qs),
                                    C.byref(st)))
        return dict(pos=pos, vel=vel, alive=alive, q_surface=qs.value, step=st.value)

    def eval_field(self) -> np.ndarray:
        E = np.zeros((self.n, 3))
        _check(lib().sim_eval_field(self._handle(), _dp(E)))
        return E

    def profile(self, k: int) -> dict:
        L = lib()
        nk = L.sim_num_kernels()
        ms = np.zeros(nk)
        _check(L.sim_profile(self._handle(), k, _dp(ms), nk))
        return {L.sim_kernel_name(i).decode(): float(ms[i]) for i in range(nk)}

    def counts(self) -> dict:
        """Alive and absorbed particle counts and the step (synchronises)."""
        return _counts(self._handle(), 0)

    def info(self) -> dict:
        n = C.c_int64()
        t = C.c_int32()
        c = C.c_int32()
        _check(lib().sim_info(self._handle(), C.byref(n), C.byref(t), C.byref(c)))
        return dict(n=n.value, tile=t.value, channels=c.value)


def eval_field_static(params: SimParams, pos, E, q_surface: float = 0.0, u_asy: float = 0.0,
                      stream=None):
    """sim_eval_field_static: the field at device-resident positions pos
    (torch tensor [n, 3], float64, on the GPU) into E (same shape), with no
    device allocation (the library's static buffer).  Synchronises."""
    n = int(pos.shape[0])
    if tuple(pos.shape) != (n, 3) or tuple(E.shape) != (n, 3):
        raise ValueError("pos and E must have shape [n, 3]")
    if not (pos.is_contiguous() and E.is_contiguous()):
        raise ValueError("pos and E must be contiguous")
    if str(pos.dtype) != "torch.float64" or str(E.dtype) != "torch.float64":
        raise ValueError("pos and E must be float64")
    if stream is None:
        stream = _current_torch_stream()
    p = params.to_c()
    _check(lib().sim_eval_field_static(C.byref(p), n, C.c_void_p(pos.data_ptr()), q_surface,
                                       u_asy, C.c_void_p(E.data_ptr()), stream))


def eval_field_static_bytes(params: SimParams, n: int) -> int:
    p = params.to_c()
    v = lib().sim_eval_field_static_bytes(C.byref(p), n)
    if v < 0:
        _check(int(v))
    return int(v)


@dataclass
class Member:
    """One simulation of a batch: its particles, drive and per-run parameters
    (everything but the probe geometry, l_max, m_mode and precision, which the
    batch's common SimParams fix)."""
    pos: np.ndarray
    vel: np.ndarray
    u_asy: np.ndarray
    ntilde: float
    ids: np.ndarray | None = None
    start_step: int = 0
    ion_density: float = 1.0
    q_surface0: float = 0.0
    r_out: float = 5.0
    dt: float = 0.05
    seed: int = 0
    probe_bc: int = SIM_BC_ABSORB
    wall_bc: int = SIM_BC_SPECULAR
    ion_profile: np.ndarray | None = None   # densities at equally spaced radii 1..r_out
    ion_mass: float = 0.0                   # m_i / m_e of ids with bit 31 set (mobile ions)

    @staticmethod
    def from_params(params: SimParams, pos, vel, u_asy, ids=None, start_step: int = 0) -> "Member":
        return Member(pos=pos, vel=vel, u_asy=u_asy, ntilde=params.ntilde, ids=ids,
                      start_step=start_step, ion_density=params.ion_density,
                      q_surface0=params.q_surface0, r_out=params.r_out, dt=params.dt,
                      seed=params.seed, probe_bc=params.probe_bc, wall_bc=params.wall_bc)

    def to_c(self):
        """(sim_member, arrays kept alive for the duration of the call)."""
        pos = np.ascontiguousarray(self.pos, dtype=np.float64)
        vel = np.ascontiguousarray(self.vel, dtype=np.float64)
        u = np.ascontiguousarray(self.u_asy, dtype=np.float64)
        n = pos.shape[0]
        if pos.shape != (n, 3) or vel.shape != (n, 3):
            raise ValueError("pos and vel must have shape [n, 3]")
        ids = None if self.ids is None else np.ascontiguousarray(self.ids, dtype=np.uint32)
        m = sim_member()
        lib().sim_member_default(C.byref(m))
        m.n = n
        m.pos = _dp(pos)
        m.vel = _dp(vel)
        m.ids = None if ids is None else ids.ctypes.data_as(C.POINTER(C.c_uint32))
        m.u_asy = _dp(u) if u.size else None
        m.n_steps = u.shape[0]
        m.start_step = self.start_step
        for f in ("ntilde", "ion_density", "q_surface0", "r_out", "dt", "seed", "probe_bc",
                  "wall_bc", "ion_mass"):
            setattr(m, f, getattr(self, f))
        prof = None
        if self.ion_profile is not None:
            prof = np.ascontiguousarray(self.ion_profile, dtype=np.float64)
            m.ion_profile = _dp(prof)
            m.ion_profile_len = prof.size
        return m, (pos, vel, u, ids, prof)


def member_data_bytes(n_steps: int, ion_profile_len: int = 0) -> int:
    """Bytes a member takes of a batch's member data pool."""
    v = lib().sim_member_data_bytes(n_steps, ion_profile_len)
    if v < 0:
        _check(int(v))
    return int(v)


def batch_footprint_bytes(params: SimParams, slot_capacity: int, max_members: int,
                          member_data: int = 0) -> int:
    p = params.to_c()
    v = lib().sim_batch_footprint_bytes(C.byref(p), slot_capacity, max_members, member_data)
    if v < 0:
        _check(int(v))
    return int(v)


class Batch:
    """Many independent simulations stepped by the same kernel launches
    (sim_batch_create ... sim_destroy).  Members may be admitted and retired
    between steps; each member's results equal those of the member run alone."""

    def __init__(self, common: SimParams, members=(), slot_capacity: int = 0,
                 max_members: int = 0, member_data: int = 0, stream=None,
                 use_torch_stream: bool = True, allocator="torch"):
        """member_data: bytes of the member data pool (0: what the initial
        members need; see member_data_bytes)."""
        L = lib()
        self._p = common.to_c()
        cs, keep = [], []
        for mb in members:
            c, k = mb.to_c()
            cs.append(c)
            keep.append(k)
        arr = (sim_member * max(len(cs), 1))(*cs)
        if stream is None and use_torch_stream:
            stream = _current_torch_stream()
        h = C.c_void_p()
        self._alloc = _allocator(allocator)
        _check(L.sim_batch_create(C.byref(self._p), slot_capacity, max_members, member_data,
                                  len(cs), arr if cs else None, stream,
                                  C.byref(self._alloc.c) if self._alloc else None, C.byref(h)))
        self._h = h
        self._n = {i: mb.to_c()[0].n for i, mb in enumerate(members)}

    def close(self):
        if getattr(self, "_h", None):
            lib().sim_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _handle(self):
        if not getattr(self, "_h", None):
            raise SimError(SIM_ESTATE, "batch is closed")
        return self._h

    def add(self, member: Member) -> int:
        c, keep = member.to_c()
        idx = C.c_int32()
        _check(lib().sim_batch_add(self._handle(), C.byref(c), C.byref(idx)))
        self._n[idx.value] = c.n
        del keep
        return idx.value

    def remove(self, index: int):
        _check(lib().sim_batch_remove(self._handle(), index))
        self._n.pop(index, None)

    def step(self, k: int = 1):
        _check(lib().sim_batch_step(self._handle(), k))

    def step_strict(self, k: int = 1):
        _check(lib().sim_step(self._handle(), k))

    def sync(self):
        _check(lib().sim_sync(self._handle()))

    def query(self) -> bool:
        """True when all enqueued work has completed (does not wait)."""
        rc = lib().sim_query(self._handle())
        if rc == SIM_BUSY:
            return False
        _check(rc)
        return True

    def info(self, index: int) -> dict:
        n, st, ns = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().sim_member_info(self._handle(), index, C.byref(n), C.byref(st), C.byref(ns)))
        return dict(n=n.value, step=st.value, n_steps=ns.value)

    def counts(self, index: int) -> dict:
        """Alive and absorbed particle counts and the step (synchronises)."""
        return _counts(self._handle(), index)

    def read_response(self, index: int, first: int, count: int) -> np.ndarray:
        out = np.zeros(count)
        _check(lib().sim_member_read_response(self._handle(), index, first, count, _dp(out)))
        return out

    def read_state(self, index: int) -> dict:
        n = self.info(index)["n"]
        pos = np.zeros((n, 3))
        vel = np.zeros((n, 3))
        alive = np.zeros(n, dtype=np.uint8)
        qs = C.c_double()
        st = C.c_int64()
        _check(lib().sim_member_read_state(self._handle(), index, _dp(pos), _dp(vel),
                                           alive.ctypes.data_as(C.POINTER(C.c_uint8)),
                                           C.byref(qs), C.byref(st)))
        return dict(pos=pos, vel=vel, alive=alive, q_surface=qs.value, step=st.value)

    def eval_field(self, index: int) -> np.ndarray:
        n = self.info(index)["n"]
        E = np.zeros((n, 3))
        _check(lib().sim_member_eval_field(self._handle(), index, _dp(E)))
        return E

    def profile(self, k: int) -> dict:
        L = lib()
        nk = L.sim_num_kernels()
        ms = np.zeros(nk)
        _check(L.sim_profile(self._handle(), k, _dp(ms), nk))
        return {L.sim_kernel_name(i).decode(): float(ms[i]) for i in range(nk)}
