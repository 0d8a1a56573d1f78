"""ctypes binding of libl2t.so (declared in include/l2t.h).

Argument marshalling only: every step of the electronic-temperature path runs
in the library's HIP kernels.  Functions carry the C names; ``Context`` is a
small convenience wrapper over them.  Arrays may be numpy arrays (host) or
torch tensors on the GPU (device); torch is used for device memory and the
current HIP stream only.

Loading fails loudly when the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libl2t.so")

L2T_OK, L2T_WUNSTABLE = 0, 1
L2T_EINVAL, L2T_ENOMEM, L2T_EHIP, L2T_ESTATE, L2T_ERANGE, L2T_ENOTIMPL = -1, -2, -3, -4, -5, -6
L2T_FP64, L2T_FP32C = 0, 1
L2T_HOST, L2T_DEVICE = 0, 1
L2T_FIELD_TE, L2T_FIELD_TL, L2T_FIELD_GATE, L2T_FIELD_NBRS, L2T_FIELD_ELAT = 0, 1, 2, 3, 4
L2T_FIELD_FIXED = 5
L2T_CE_CONST, L2T_CE_LINEAR, L2T_CE_CAPPED = 0, 1, 2
L2T_OPT_PERSISTENT, L2T_OPT_BLOCK, L2T_OPT_RESIDENT_MAX, L2T_OPT_GRAPH, L2T_OPT_AUTOTUNE = 0, 1, 2, 3, 4
L2T_OPT_KERNEL, L2T_OPT_BRICK_EDGE, L2T_OPT_ATOM_LEDGER, L2T_OPT_BATCH_FP64 = 5, 6, 7, 8
L2T_OPT_SWEEP = 9
L2T_OPT_TABLE_STREAM = 10
L2T_XI_INSTANT, L2T_XI_LEDGER = 0, 1

# every symbol the header declares (checked by the CPU test suite)
EXPORTS = ("l2t_create", "l2t_destroy", "l2t_set_positions", "l2t_build_neighbors",
           "l2t_get_neighbors", "l2t_set_params", "l2t_set_field", "l2t_get_field",
           "l2t_set_velocities", "l2t_set_velocities_noalloc", "l2t_advance", "l2t_advance_system", "l2t_advance_recorded",
           "l2t_adjoint", "l2t_energies", "l2t_sync", "l2t_set_option", "l2t_get_option",
           "l2t_coupling", "l2t_damping_step", "l2t_set_mean_field", "l2t_get_params",
           "l2t_set_lattice_fd", "l2t_set_counters", "l2t_set_allocator",
           "l2t_exchange_rate", "l2t_pair_fp32", "l2t_strerror", "l2t_last_error",
           "l2t_version")


# the allocator hook of l2t_set_allocator
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class l2t_system_desc(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("periodic", C.c_int32 * 3),
                ("box_lo", C.c_double * 3), ("box_len", C.c_double * 3)]


class l2t_params(C.Structure):
    _fields_ = [("T_min", C.c_double), ("T_max", C.c_double), ("K", C.c_double),
                ("dt", C.c_double), ("g", C.c_double),
                ("ce_model", C.c_int32), ("laser_on", C.c_int32),
                ("ce_const", C.c_double), ("gamma", C.c_double), ("ce_cap", C.c_double),
                ("ke_eps", C.c_double),
                ("laser_fluence", C.c_double), ("laser_lp", C.c_double),
                ("laser_t0", C.c_double), ("laser_sigma", C.c_double),
                ("laser_x0", C.c_double), ("v_atom", C.c_double)]


class l2t_mean_field(C.Structure):
    _fields_ = [("on", C.c_int32), ("reserved", C.c_int32), ("lambda_", C.c_double),
                ("k_coef", C.c_double)]


class l2t_lattice_fd(C.Structure):
    _fields_ = [("on", C.c_int32), ("reserved", C.c_int32), ("K_lat", C.c_double),
                ("c_lat", C.c_double)]


class l2t_energy_report(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("E_e", C.c_double),
                ("sum_T", C.c_double), ("E_e_to_l", C.c_double), ("E_src", C.c_double),
                ("T_ledger_acc", C.c_double), ("T_max_atom", C.c_double),
                ("T_min_atom", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class L2TError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"l2t status {status}: {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Load libl2t.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "paper_1810_12357_amd.build.build() (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "l2t_create": (C.c_int, [P(vp), i32, P(l2t_system_desc), i32, vp]),
        "l2t_destroy": (None, [vp]),
        "l2t_set_allocator": (C.c_int, [vp, ALLOC_FN, FREE_FN, vp]),
        "l2t_set_positions": (C.c_int, [vp, i32, vp, i32]),
        "l2t_build_neighbors": (C.c_int, [vp, d, P(i32), P(d)]),
        "l2t_get_neighbors": (C.c_int, [vp, i32, vp, vp, i64]),
        "l2t_set_params": (C.c_int, [vp, i32, P(l2t_params)]),
        "l2t_set_field": (C.c_int, [vp, i32, i32, vp, i32]),
        "l2t_get_field": (C.c_int, [vp, i32, i32, vp, i32]),
        "l2t_set_velocities": (C.c_int, [vp, i32, vp, vp, i32, i32]),
        "l2t_set_velocities_noalloc": (C.c_int, [vp, i32, vp, vp, i32]),
        "l2t_advance": (C.c_int, [vp, i32]),
        "l2t_advance_system": (C.c_int, [vp, i32, i32]),
        "l2t_advance_recorded": (C.c_int, [vp, i32, i32]),
        "l2t_adjoint": (C.c_int, [vp, vp, i32, vp, vp, vp]),
        "l2t_energies": (C.c_int, [vp, i32, P(l2t_energy_report)]),
        "l2t_sync": (C.c_int, [vp]),
        "l2t_set_counters": (C.c_int, [vp, i32, i64, d, d, d]),
        "l2t_set_option": (C.c_int, [vp, i32, i64]),
        "l2t_get_option": (C.c_int, [vp, i32, P(i64)]),
        "l2t_coupling": (C.c_int, [vp, i32, i32, d, vp, vp, vp, i32]),
        "l2t_set_mean_field": (C.c_int, [vp, i32, P(l2t_mean_field)]),
        "l2t_get_params": (C.c_int, [vp, i32, P(l2t_params)]),
        "l2t_set_lattice_fd": (C.c_int, [vp, i32, P(l2t_lattice_fd)]),
        "l2t_damping_step": (C.c_int, [vp, i32, d, vp, vp, vp, vp, i32]),
        "l2t_exchange_rate": (d, [d, d, i32, d]),
        "l2t_pair_fp32": (C.c_int, [vp, vp, vp, i64, vp]),
        "l2t_strerror": (C.c_char_p, [C.c_int]),
        "l2t_last_error": (C.c_char_p, [vp]),
        "l2t_version": (C.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---- argument marshalling ----------------------------------------------------
def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


# per context handle: atom count of every system and the HIP device, recorded
# by l2t_create so that array arguments can be checked before the call
_CTX_INFO: dict = {}


def _sys_n(ctx, sys: int):
    info = _CTX_INFO.get(getattr(ctx, "value", ctx))
    if info is None or not (0 <= sys < len(info[0])):
        return None
    return info[0][sys]


def _ctx_device(ctx):
    info = _CTX_INFO.get(getattr(ctx, "value", ctx))
    return None if info is None else info[1]


def _ptr(a, dtype=np.float64, n=None, out=False, ctx=None):
    """(pointer, mem, keepalive) for a numpy array or a torch tensor.

    n: required element count (None = unchecked).  out: the library writes
    the buffer, so it must already have the dtype and layout (no copy).
    ctx: a device tensor must live on the context's GPU."""
    if _is_torch(a):
        import torch
        want = {np.float64: torch.float64, np.float32: torch.float32,
                np.int32: torch.int32, np.int64: torch.int64}[dtype]
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        if n is not None and a.numel() != n:
            raise ValueError(f"tensor has {a.numel()} elements, expected {n}")
        if a.is_cuda and ctx is not None:
            dev = _ctx_device(ctx)
            if dev is not None and a.device.index != dev:
                raise ValueError(f"tensor on cuda:{a.device.index}, context on cuda:{dev}")
        return C.c_void_p(a.data_ptr()), (L2T_DEVICE if a.is_cuda else L2T_HOST), a
    if out:
        if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags.c_contiguous
                and a.flags.writeable):
            raise TypeError(f"output must be a writeable contiguous {np.dtype(dtype)} array")
        arr = a
    else:
        arr = np.ascontiguousarray(a, dtype=dtype)
    if n is not None and arr.size != n:
        raise ValueError(f"array has {arr.size} elements, expected {n}")
    return C.c_void_p(arr.ctypes.data), L2T_HOST, arr


def _stream(stream):
    if stream is not None:
        return C.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return C.c_void_p(0)


def make_params(p: dict) -> l2t_params:
    return l2t_params(**{k: p[k] for k, _ in l2t_params._fields_})


def _check(ctx, rc: int, allow_warn: bool = True) -> int:
    if rc == L2T_OK or (allow_warn and rc > 0):
        return rc
    lib = load()
    msg = lib.l2t_last_error(ctx).decode() if ctx else ""
    if not msg:
        msg = lib.l2t_strerror(rc).decode()
    raise L2TError(rc, msg)


# ---- functions with the C names ----------------------------------------------
def l2t_version() -> int:
    return load().l2t_version()


def l2t_strerror(status: int) -> str:
    return load().l2t_strerror(status).decode()


def l2t_exchange_rate(kappa_e: float, C_e: float, dim: int, lattice_sum: float) -> float:
    return load().l2t_exchange_rate(kappa_e, C_e, dim, lattice_sum)


def l2t_create(descs, precision: int, stream=None):
    arr = (l2t_system_desc * len(descs))(*descs)
    h = C.c_void_p()
    _check(None, load().l2t_create(C.byref(h), len(descs), arr, precision, _stream(stream)))
    dev = None
    try:
        import torch
        if torch.cuda.is_available():
            dev = torch.cuda.current_device()
    except Exception:
        pass
    _CTX_INFO[h.value] = ([int(d.n_atoms) for d in descs], dev)
    return h


def l2t_destroy(ctx) -> None:
    _CTX_INFO.pop(getattr(ctx, "value", ctx), None)
    load().l2t_destroy(ctx)


def l2t_set_allocator(ctx, alloc, free_, user=None) -> int:
    """alloc, free_: ALLOC_FN / FREE_FN objects (or None for both, which restores
    hipMalloc / hipFree).  The caller keeps them alive while the context lives."""
    a = C.cast(None, ALLOC_FN) if alloc is None else alloc
    f = C.cast(None, FREE_FN) if free_ is None else free_
    return _check(ctx, load().l2t_set_allocator(ctx, a, f, user))


def torch_allocator(device=None, stream=None):
    """(alloc, free_) hooks that take the context's device memory from
    PyTorch's caching allocator on the context's stream (the HIP stream
    handle given to l2t_create; None or 0 = the device's null stream), so
    that the caching allocator orders the reuse of a block after the library's
    work on it."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    h = int(stream or 0)
    s = (torch.cuda.ExternalStream(h, device=dev) if h
         else torch.cuda.default_stream(dev))

    def _alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, s)
        except Exception:
            return None

    def _free(ptr, _user):
        torch.cuda.caching_allocator_delete(int(ptr))

    return ALLOC_FN(_alloc), FREE_FN(_free)


def l2t_set_positions(ctx, sys: int, xyz) -> int:
    n = _sys_n(ctx, sys)
    p, mem, keep = _ptr(xyz, n=None if n is None else 3 * n, ctx=ctx)
    return _check(ctx, load().l2t_set_positions(ctx, sys, p, mem))


def l2t_build_neighbors(ctx, r_cut: float):
    mx = C.c_int32()
    mean = C.c_double()
    _check(ctx, load().l2t_build_neighbors(ctx, r_cut, C.byref(mx), C.byref(mean)))
    return mx.value, mean.value


def l2t_get_neighbors(ctx, sys: int, n: int):
    row = np.zeros(n + 1, dtype=np.int64)
    lib = load()
    _check(ctx, lib.l2t_get_neighbors(ctx, sys, row.ctypes.data, None, 0))
    col = np.zeros(max(int(row[-1]), 1), dtype=np.int32)
    _check(ctx, lib.l2t_get_neighbors(ctx, sys, row.ctypes.data, col.ctypes.data, col.size))
    return row, col[:int(row[-1])]


def l2t_set_params(ctx, sys: int, params: dict) -> int:
    pp = make_params(params)
    return _check(ctx, load().l2t_set_params(ctx, sys, C.byref(pp)))


def l2t_set_field(ctx, sys: int, field: int, src) -> int:
    p, mem, keep = _ptr(src, n=_sys_n(ctx, sys), ctx=ctx)
    return _check(ctx, load().l2t_set_field(ctx, sys, field, p, mem))


def l2t_get_field(ctx, sys: int, field: int, dst):
    p, mem, keep = _ptr(dst, n=_sys_n(ctx, sys), out=True, ctx=ctx)
    _check(ctx, load().l2t_get_field(ctx, sys, field, p, mem))
    return dst


def l2t_set_velocities(ctx, sys: int, v, mass, global_com: bool = False) -> int:
    n = _sys_n(ctx, sys)
    pv, mem, kv = _ptr(v, n=None if n is None else 3 * n, ctx=ctx)
    pm, mem2, km = _ptr(mass, n=n, ctx=ctx)
    if mem != mem2:
        raise TypeError("velocities and masses must live in the same memory space")
    return _check(ctx, load().l2t_set_velocities(ctx, sys, pv, pm, mem, int(bool(global_com))))


def l2t_set_velocities_noalloc(ctx, sys: int, v, mass, global_com: bool = False) -> int:
    """Eq. 4 as l2t_set_velocities, allocating nothing; v and mass are device
    tensors (float64, contiguous)."""
    for t in (v, mass):
        if not (_is_torch(t) and t.is_cuda):
            raise TypeError("l2t_set_velocities_noalloc takes device tensors")
    n = _sys_n(ctx, sys)
    pv, _, kv = _ptr(v, n=None if n is None else 3 * n, ctx=ctx)
    pm, _, km = _ptr(mass, n=n, ctx=ctx)
    return _check(ctx, load().l2t_set_velocities_noalloc(ctx, sys, pv, pm, int(bool(global_com))))


def l2t_advance(ctx, n_substeps: int) -> int:
    return _check(ctx, load().l2t_advance(ctx, n_substeps))


def l2t_advance_system(ctx, sys: int, n_substeps: int) -> int:
    return _check(ctx, load().l2t_advance_system(ctx, sys, n_substeps))


def l2t_advance_recorded(ctx, n_substeps: int, ckpt_every: int) -> int:
    return _check(ctx, load().l2t_advance_recorded(ctx, n_substeps, ckpt_every))


def l2t_adjoint(ctx, dL_dTN, n_systems: int, dL_dT0=None):
    info = _CTX_INFO.get(getattr(ctx, "value", ctx))
    N = None if info is None else sum(info[0])
    pw, mem, kw = _ptr(dL_dTN, n=N, ctx=ctx)
    dK = np.zeros(n_systems)
    dg = np.zeros(n_systems)
    p0 = None
    if dL_dT0 is not None:
        p0, mem0, k0 = _ptr(dL_dT0, n=N, out=True, ctx=ctx)
        if mem0 != mem:
            raise TypeError("dL_dTN and dL_dT0 must live in the same memory space")
    _check(ctx, load().l2t_adjoint(ctx, pw, mem, dK.ctypes.data, dg.ctypes.data, p0))
    return dK, dg


def l2t_set_mean_field(ctx, sys: int, on: bool, lambda_atom: float = 0.0,
                       k_coef: float = 0.0) -> int:
    """Mean-field parameter mode of Section 2 (see l2t.h)."""
    mf = l2t_mean_field(on=int(bool(on)), reserved=0, lambda_=float(lambda_atom),
                        k_coef=float(k_coef))
    return _check(ctx, load().l2t_set_mean_field(ctx, sys, C.byref(mf)))


def l2t_set_lattice_fd(ctx, sys: int, on: bool, K_lat: float = 0.0, c_lat: float = 1.0) -> int:
    """Two-temperature lattice mode of Section 3.1 (see l2t.h)."""
    lf = l2t_lattice_fd(on=int(bool(on)), reserved=0, K_lat=float(K_lat), c_lat=float(c_lat))
    return _check(ctx, load().l2t_set_lattice_fd(ctx, sys, C.byref(lf)))


def l2t_get_params(ctx, sys: int) -> dict:
    """Parameters in effect (K, ce_model, ce_const after a mean-field refresh)."""
    p = l2t_params()
    _check(ctx, load().l2t_get_params(ctx, sys, C.byref(p)))
    return {k: getattr(p, k) for k, _ in p._fields_}


def l2t_coupling(ctx, sys: int, mode: int, dt_md: float, v, mass, xi):
    """Eq. 8 coupling coefficient into xi (see l2t.h)."""
    n = _sys_n(ctx, sys)
    pv, mem, kv = _ptr(v, n=None if n is None else 3 * n, ctx=ctx)
    pm, mem2, km = _ptr(mass, n=n, ctx=ctx)
    px, mem3, kx = _ptr(xi, n=n, out=True, ctx=ctx)
    if not (mem == mem2 == mem3):
        raise TypeError("v, mass and xi must live in the same memory space")
    _check(ctx, load().l2t_coupling(ctx, sys, mode, float(dt_md), pv, pm, px, mem))
    return xi


def l2t_damping_step(ctx, sys: int, dt_md: float, xi, force, mass, v):
    """One explicit step of Eq. 5 on v in place (see l2t.h)."""
    n = _sys_n(ctx, sys)
    n3 = None if n is None else 3 * n
    px, mem, kx = _ptr(xi, n=n, ctx=ctx)
    pm, mem2, km = _ptr(mass, n=n, ctx=ctx)
    pv, mem3, kv = _ptr(v, n=n3, out=True, ctx=ctx)
    pf, kf = None, None
    if force is not None:
        pf, mem4, kf = _ptr(force, n=n3, ctx=ctx)
        if mem4 != mem:
            raise TypeError("force must live in the same memory space as v")
    if not (mem == mem2 == mem3):
        raise TypeError("xi, mass and v must live in the same memory space")
    _check(ctx, load().l2t_damping_step(ctx, sys, float(dt_md), px, pf, pm, pv, mem))
    return v


def l2t_energies(ctx, sys: int, check: bool = True) -> dict:
    e = l2t_energy_report()
    rc = load().l2t_energies(ctx, sys, C.byref(e))
    if check:
        _check(ctx, rc)
    d = e.as_dict()
    d["status"] = rc
    return d


def l2t_sync(ctx) -> int:
    return _check(ctx, load().l2t_sync(ctx))


def l2t_set_counters(ctx, sys: int, step: int, E_e_to_l: float, E_src: float,
                     T_ledger_acc: float) -> int:
    """Restore a system's sub-step counter and ledger totals (see l2t.h)."""
    return _check(ctx, load().l2t_set_counters(ctx, sys, int(step), float(E_e_to_l),
                                               float(E_src), float(T_ledger_acc)))


def l2t_set_option(ctx, option: int, value: int) -> int:
    return _check(ctx, load().l2t_set_option(ctx, option, value))


def l2t_get_option(ctx, option: int) -> int:
    v = C.c_int64()
    _check(ctx, load().l2t_get_option(ctx, option, C.byref(v)))
    return v.value


def l2t_pair_fp32(ti, tj, out, stream=None) -> None:
    """Device FP32 tensors ti, tj, out of equal length."""
    for t in (ti, tj, out):
        if not (_is_torch(t) and t.is_cuda):
            raise TypeError("l2t_pair_fp32 takes device tensors")
    n = out.numel()
    _check(None, load().l2t_pair_fp32(C.c_void_p(ti.data_ptr()), C.c_void_p(tj.data_ptr()),
                                      C.c_void_p(out.data_ptr()), n, _stream(stream)))


# ---- convenience wrapper -------------------------------------------------------
def desc_of(system) -> l2t_system_desc:
    d = l2t_system_desc()
    d.n_atoms = system.n
    for k in range(3):
        d.periodic[k] = int(system.periodic[k])
        d.box_lo[k] = float(system.box_lo[k])
        d.box_len[k] = float(system.box_len[k])
    return d


class Context:
    """Owns one l2t context holding a list of independent systems."""

    def __init__(self, systems, precision: int = L2T_FP32C, stream=None,
                 torch_memory: bool = False):
        self.systems = list(systems)
        self.precision = precision
        hs = _stream(stream)
        self.h = l2t_create([desc_of(s) for s in self.systems], precision, hs.value or 0)
        self._hooks = None
        if torch_memory:
            # device buffers from PyTorch's caching allocator, on the stream
            # the context works on; the hooks live as long as the context
            self._hooks = torch_allocator(stream=hs.value or 0)
            l2t_set_allocator(self.h, *self._hooks)

    def close(self):
        if self.h:
            l2t_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, r_cut: float, use_velocities: bool = True):
        """Positions, neighbours, parameters, T_e and T_lat of every system."""
        for s, sy in enumerate(self.systems):
            l2t_set_positions(self.h, s, sy.pos.reshape(-1))
        mx, mean = l2t_build_neighbors(self.h, r_cut)
        warn = 0
        for s, sy in enumerate(self.systems):
            warn |= l2t_set_params(self.h, s, sy.params)
            l2t_set_field(self.h, s, L2T_FIELD_TE, sy.T_e0)
            if use_velocities and sy.vel is not None:
                l2t_set_velocities(self.h, s, sy.vel.reshape(-1), sy.mass)
            elif sy.T_l is not None:
                l2t_set_field(self.h, s, L2T_FIELD_TL, sy.T_l)
        return mx, mean, warn

    def get(self, sys: int, field: int = L2T_FIELD_TE) -> np.ndarray:
        out = np.empty(self.systems[sys].n)
        l2t_get_field(self.h, sys, field, out)
        return out

    def advance(self, n: int) -> int:
        return l2t_advance(self.h, n)

    def energies(self, sys: int, check: bool = True) -> dict:
        return l2t_energies(self.h, sys, check)
