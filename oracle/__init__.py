"""Plain FP64 CPU oracle for the electronic-temperature sub-step path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the GPU library.  The arithmetic lives in ``oracle.c``
(plain C, FP64, no FMA contraction); this module only marshals numpy arrays.

Function map (paper passages):
  neighbors          neighbour sets within the cut-off, minimum image
                     (Section 2, cut-off of Eq. 4; Section 2.1)
  lattice_temperature  Eq. 4 with centre-of-mass removal + the K_i < eps gate
                     (remark after Eq. 8)
  pair               the pair term of Eq. 2, literal two-exponential form
  run                forward-Euler sub-steps of Eq. 2 with coupling and Eq. 10
                     source (Section 2.1), ledgers of Eq. 6 (per system and,
                     optionally, per atom)
  mean_field         mean-field heat capacity and exchange rate (Section 2)
  run_2t             two-temperature bar: Eq. 2 electrons with a finite-
                     difference Fourier lattice in the same step (Section 3.1)
  coupling           Eq. 8 coupling coefficient of the damping force
  damping_step       one explicit velocity step of Eq. 5
  energies           sum of the per-atom electronic energy and of T
  adjoint            discrete adjoint of ``run`` (derived from Eq. 2)
  run_cs             complex-step forward run (directional derivatives)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CE_MODELS = {"const": 0, "linear": 1, "capped": 2}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("T_min", C.c_double), ("T_max", C.c_double), ("K", C.c_double),
                ("dt", C.c_double), ("g", C.c_double),
                ("ce_model", C.c_int32), ("laser_on", C.c_int32),
                ("ce_const", C.c_double), ("gamma", C.c_double), ("ce_cap", C.c_double),
                ("ke_eps", C.c_double),
                ("laser_fluence", C.c_double), ("laser_lp", C.c_double),
                ("laser_t0", C.c_double), ("laser_sigma", C.c_double),
                ("laser_x0", C.c_double), ("v_atom", C.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        pd, pi32, pi64 = P(d), P(i32), P(i64)
        lib.or_pair.restype = d
        lib.or_pair.argtypes = [d, d]
        lib.or_pair_batch.argtypes = [i64, pd, pd, pd]
        lib.or_laser_q_at.restype = d
        lib.or_laser_q_at.argtypes = [P(Params), d, d]
        lib.or_neighbors.restype = i64
        lib.or_neighbors.argtypes = [i32, pd, pd, pd, pd, pd, pi32, d, i32, pi64, pi32, i64]
        lib.or_lattice_temp.argtypes = [i32, pi64, pi32, pd, pd, pd, pd, d, i32, pd, pi32]
        lib.or_run.restype = i64
        lib.or_run.argtypes = [i32, pi64, pi32, pd, pd, pi32, pd, P(Params), i64, i32, pd, pd,
                               pi32]
        lib.or_mean_field.argtypes = [i32, pd, pd, d, d, pd]
        lib.or_run_2t.restype = i64
        lib.or_run_2t.argtypes = [i32, pi64, pi32, pd, pd, P(Params), d, d, i64, i32, pd]
        lib.or_coupling.argtypes = [i32, i32, pd, pd, pi32, pd, d, d, d, pd, pd, pd, pd, pd]
        lib.or_damping_step.argtypes = [i32, d, pd, pd, pd, pd, pd, pd, pd, pd]
        lib.or_energies.argtypes = [i32, pd, P(Params), pd]
        lib.or_adjoint.restype = C.c_int
        lib.or_adjoint.argtypes = [i32, pi64, pi32, pd, pd, pi32, pd, P(Params), i64, i32,
                                   pd, pd, pd, pd]
        lib.or_run_cs.argtypes = [i32, pi64, pi32, pd, pd, pi32, pd, P(Params),
                                  d, d, d, d, i64, i32]
        _lib = lib
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(p: dict) -> Params:
    ce = p["ce_model"]
    ce = CE_MODELS[ce] if isinstance(ce, str) else int(ce)
    return Params(T_min=p["T_min"], T_max=p["T_max"], K=p["K"], dt=p["dt"], g=p["g"],
                  ce_model=ce, laser_on=int(p["laser_on"]), ce_const=p["ce_const"],
                  gamma=p["gamma"], ce_cap=p["ce_cap"], ke_eps=p["ke_eps"],
                  laser_fluence=p["laser_fluence"], laser_lp=p["laser_lp"],
                  laser_t0=p["laser_t0"], laser_sigma=p["laser_sigma"],
                  laser_x0=p["laser_x0"], v_atom=p["v_atom"])


def _gomp():
    _load()                      # the oracle library pulls in the OpenMP runtime
    return C.CDLL("libgomp.so.1")


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_gomp().omp_get_max_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's parallel loops (results do
    not depend on it: every sum runs serially in a fixed order)."""
    _gomp().omp_set_num_threads(int(n))


def pair(ti, tj):
    """Literal pair term of Eq. 2 for arrays of normalised temperatures."""
    ti = _f64(np.atleast_1d(ti))
    tj = _f64(np.broadcast_to(np.atleast_1d(tj), ti.shape))
    out = np.empty_like(ti)
    _load().or_pair_batch(ti.size, _p(ti, C.c_double), _p(tj, C.c_double), _p(out, C.c_double))
    return out


def laser_q(params: dict, x: float, t: float) -> float:
    pp = make_params(params)
    return _load().or_laser_q_at(C.byref(pp), float(x), float(t))


def neighbors(pos, box_lo, box_len, periodic, r_cut, method: str = "auto"):
    """Rows N(i) sorted by ascending j: returns (row_ptr int64[N+1], col int32)."""
    pos = _f64(pos)
    n = pos.shape[1]
    x, y, z = (np.ascontiguousarray(pos[d]) for d in range(3))
    lo = _f64(box_lo)
    ln = _f64(box_len)
    per = np.ascontiguousarray(periodic, dtype=np.int32)
    m = {"brute": 0, "cells": 1, "auto": 0 if n <= 3000 else 1}[method]
    lib = _load()
    row = np.zeros(n + 1, dtype=np.int64)
    args = (n, _p(x, C.c_double), _p(y, C.c_double), _p(z, C.c_double), _p(lo, C.c_double),
            _p(ln, C.c_double), _p(per, C.c_int32), float(r_cut), m, _p(row, C.c_int64))
    nnz = lib.or_neighbors(*args, None, 0)
    if nnz < 0:
        raise MemoryError("oracle neighbour count failed")
    col = np.empty(max(nnz, 1), dtype=np.int32)
    nnz2 = lib.or_neighbors(*args, _p(col, C.c_int32), nnz)
    if nnz2 != nnz:
        raise RuntimeError("oracle neighbour fill failed")
    return row, col[:nnz]


def lattice_temperature(row, col, vel, mass, ke_eps=1e-5, global_com=False):
    """Eq. 4 over {i} U N(i) and the kinetic-energy gate: (T_lat, gated)."""
    vel = _f64(vel)
    n = vel.shape[1]
    vx, vy, vz = (np.ascontiguousarray(vel[d]) for d in range(3))
    m = _f64(mass)
    T = np.empty(n)
    gated = np.empty(n, dtype=np.int32)
    _load().or_lattice_temp(n, _p(row, C.c_int64), _p(col, C.c_int32), _p(vx, C.c_double),
                            _p(vy, C.c_double), _p(vz, C.c_double), _p(m, C.c_double),
                            float(ke_eps), int(bool(global_com)), _p(T, C.c_double),
                            _p(gated, C.c_int32))
    return T, gated


def _opt(a, dtype, n):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=dtype)
    assert a.shape == (n,)
    return a, _p(a, C.c_double if dtype == np.float64 else C.c_int32)


def run(row, col, T, T_lat, params: dict, n_steps: int, step0: int = 0, gated=None,
        x=None, ledger=None, e_atom=None, fixed=None):
    """Forward-Euler sub-steps.  Returns (T_new, ledger[3], n_out_of_range).

    ledger = [energy to lattice (eV), source energy (eV), temperature ledger (K)],
    accumulated onto the ``ledger`` argument when given.  ``e_atom`` (float64
    array [n], optional) accumulates in place each atom's energy to the
    lattice, sum over sub-steps of g (T_i - T_lat,i) dt (Eq. 6).  ``fixed``
    (int array [n], optional): atoms that hold their electronic temperature
    (Dirichlet boundary); the exchange they would receive goes to the
    temperature ledger."""
    T = _f64(T).copy()
    n = T.size
    Tl = _f64(T_lat)
    g, gp = _opt(gated, np.int32, n)
    fx, fp = _opt(fixed, np.int32, n)
    xx, xp = _opt(x, np.float64, n)
    led = np.zeros(3) if ledger is None else _f64(ledger).copy()
    if e_atom is not None:
        assert e_atom.dtype == np.float64 and e_atom.shape == (n,) and e_atom.flags.c_contiguous
    pp = make_params(params)
    bad = _load().or_run(n, _p(row, C.c_int64), _p(col, C.c_int32), _p(T, C.c_double),
                         _p(Tl, C.c_double), gp, xp, C.byref(pp), int(step0), int(n_steps),
                         _p(led, C.c_double), None if e_atom is None else _p(e_atom, C.c_double),
                         fp)
    if bad < 0:
        raise MemoryError("oracle run allocation failed")
    return T, led, int(bad)


def run_2t(row, col, T, T_lat, params: dict, K_lat: float, c_lat: float, n_steps: int,
           step0: int = 0, ledger=None):
    """Two-temperature bar (Section 3.1): electrons by Eq. 2 and the lattice by
    the Fourier law K_lat sum_j (T_l,j - T_l,i) + (g/c_lat)(T - T_l), one
    forward-Euler step for both.  Returns (T, T_lat, ledger[3], n_out_of_range)."""
    T = _f64(T).copy()
    Tl = _f64(T_lat).copy()
    led = np.zeros(3) if ledger is None else _f64(ledger).copy()
    pp = make_params(params)
    bad = _load().or_run_2t(T.size, _p(row, C.c_int64), _p(col, C.c_int32), _p(T, C.c_double),
                            _p(Tl, C.c_double), C.byref(pp), float(K_lat), float(c_lat),
                            int(step0), int(n_steps), _p(led, C.c_double))
    if bad < 0:
        raise MemoryError("oracle run allocation failed")
    return T, Tl, led, int(bad)


def mean_field(T, T_lat, lambda_atom, k_coef):
    """Mean-field parameters of Section 2: (c, K) = (lambda_atom mean(T_e),
    k_coef / mean(T_lat))."""
    T = _f64(T)
    Tl = _f64(T_lat)
    out = np.zeros(2)
    _load().or_mean_field(T.size, _p(T, C.c_double), _p(Tl, C.c_double), float(lambda_atom),
                          float(k_coef), _p(out, C.c_double))
    return float(out[0]), float(out[1])


XI_INSTANT, XI_LEDGER = 0, 1


def coupling(mode, T, T_lat, gated, e_atom, g, dt_md, ke_eps, vel, mass):
    """Eq. 8 coupling coefficient xi_i = P_i / (2 K_i), K_i = 1/2 m_i |v_i|^2:
    P_i = g (T_i - T_lat,i) (mode XI_INSTANT) or e_atom_i / dt_md (XI_LEDGER);
    0 where gated or K_i < ke_eps.  vel is (3, n) A/fs, mass amu."""
    T = _f64(T)
    n = T.size
    Tl = _f64(T_lat)
    g_, gp = _opt(gated, np.int32, n)
    e = _f64(e_atom if e_atom is not None else np.zeros(n))
    vel = _f64(vel)
    vx, vy, vz = (np.ascontiguousarray(vel[d]) for d in range(3))
    m = _f64(mass)
    xi = np.empty(n)
    _load().or_coupling(n, int(mode), _p(T, C.c_double), _p(Tl, C.c_double), gp,
                        _p(e, C.c_double), float(g), float(dt_md), float(ke_eps),
                        _p(vx, C.c_double), _p(vy, C.c_double), _p(vz, C.c_double),
                        _p(m, C.c_double), _p(xi, C.c_double))
    return xi


def damping_step(dt_md, xi, force, mass, vel):
    """One explicit step of Eq. 5: v + dt_md (F/m + xi v).  force (3, n) eV/A or
    None; returns the new (3, n) velocities."""
    xi = _f64(xi)
    n = xi.size
    m = _f64(mass)
    v = np.array(_f64(vel), copy=True)
    vx, vy, vz = (np.ascontiguousarray(v[d]) for d in range(3))
    if force is None:
        fx = fy = fz = None
    else:
        force = _f64(force)
        fx, fy, fz = (np.ascontiguousarray(force[d]) for d in range(3))
    fp = [None if a is None else _p(a, C.c_double) for a in (fx, fy, fz)]
    _load().or_damping_step(n, float(dt_md), _p(xi, C.c_double), *fp, _p(m, C.c_double),
                            _p(vx, C.c_double), _p(vy, C.c_double), _p(vz, C.c_double))
    return np.stack([vx, vy, vz])


def energies(T, params: dict):
    """(sum_i E(T_i), sum_i T_i) with E the integral of c from 0 to T."""
    T = _f64(T)
    out = np.zeros(2)
    pp = make_params(params)
    _load().or_energies(T.size, _p(T, C.c_double), C.byref(pp), _p(out, C.c_double))
    return float(out[0]), float(out[1])


def adjoint(row, col, T0, T_lat, params: dict, n_steps: int, w, step0: int = 0,
            gated=None, x=None):
    """Discrete adjoint: returns (dL/dT0, dL/dK, dL/dg) for dL/dT^N = w."""
    T0 = _f64(T0)
    n = T0.size
    Tl = _f64(T_lat)
    w = _f64(w)
    g, gp = _opt(gated, np.int32, n)
    xx, xp = _opt(x, np.float64, n)
    lam = np.empty(n)
    dK = C.c_double()
    dg = C.c_double()
    pp = make_params(params)
    rc = _load().or_adjoint(n, _p(row, C.c_int64), _p(col, C.c_int32), _p(T0, C.c_double),
                            _p(Tl, C.c_double), gp, xp, C.byref(pp), int(step0), int(n_steps),
                            _p(w, C.c_double), _p(lam, C.c_double), C.byref(dK), C.byref(dg))
    if rc != 0:
        raise MemoryError("oracle adjoint allocation failed")
    return lam, dK.value, dg.value


def run_cs(row, col, T, T_lat, params: dict, n_steps: int, K=None, g=None, step0: int = 0,
           gated=None, x=None):
    """Complex-step run: T complex128 in, complex128 out; K and g complex."""
    T = np.ascontiguousarray(T, dtype=np.complex128).copy()
    n = T.size
    Tl = _f64(T_lat)
    g_, gp = _opt(gated, np.int32, n)
    xx, xp = _opt(x, np.float64, n)
    K = complex(params["K"] if K is None else K)
    gg = complex(params["g"] if g is None else g)
    pp = make_params(params)
    _load().or_run_cs(n, _p(row, C.c_int64), _p(col, C.c_int32),
                      T.ctypes.data_as(C.POINTER(C.c_double)), _p(Tl, C.c_double), gp, xp,
                      C.byref(pp), K.real, K.imag, gg.real, gg.imag, int(step0), int(n_steps))
    return T
