"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: each compares the oracle with a
closed form, an invariant, a special case, a high-precision evaluation, an
independent library routine or brute force, chosen so that a dropped term, a
wrong sign or index, a transposed operand or a unit slip fails one of them.
"""
import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _nbrs(sys_, rc, method="auto"):
    return oracle.neighbors(sys_.pos, sys_.box_lo, sys_.box_len, sys_.periodic, rc, method)


# --------------------------------------------------------------------- P7 ----
def _pair_decimal(ti, tj):
    """Eq. 2 pair term evaluated in 60-digit decimal arithmetic."""
    getcontext().prec = 60
    a, b = Decimal(ti), Decimal(tj)
    return float(b * (1 - a) * (a - b).exp() - a * (1 - b) * (b - a).exp())


def test_pair_special_values():
    # f(0,1) = exp(-1), f(1,0) = -exp(-1), f(t,t) = 0, f(0,t) = t exp(-t)
    assert oracle.pair(0.0, 1.0)[0] == pytest.approx(math.exp(-1.0), rel=1e-15)
    assert oracle.pair(1.0, 0.0)[0] == pytest.approx(-math.exp(-1.0), rel=1e-15)
    t = np.linspace(0, 1, 101)
    assert np.all(oracle.pair(t, t) == 0.0)
    np.testing.assert_allclose(oracle.pair(np.zeros_like(t), t), t * np.exp(-t), rtol=1e-15)


def test_pair_against_high_precision_and_product_form():
    rng = np.random.default_rng(7)
    ti = rng.uniform(0, 1, 400)
    tj = np.concatenate([rng.uniform(0, 1, 200), ti[200:] + rng.normal(0, 1e-3, 200).clip(-0.5, 0.5)])
    tj = tj.clip(0, 1)
    f = oracle.pair(ti, tj)
    ref = np.array([_pair_decimal(a, b) for a, b in zip(ti, tj)])
    np.testing.assert_allclose(f, ref, rtol=0, atol=4e-16)
    # cancellation-free product form derived from Eq. 2: with d = tj - ti and
    # m = (ti + tj)/2, f = d cosh d - (2 m (1 - m) + d^2/2) sinh d
    d = tj - ti
    m = 0.5 * (ti + tj)
    prod = d * np.cosh(d) - (2 * m * (1 - m) + d * d / 2) * np.sinh(d)
    np.testing.assert_allclose(f, prod, rtol=0, atol=4e-16)
    # exact antisymmetry of the literal form
    assert np.all(oracle.pair(tj, ti) == -f)


def test_pair_linear_limit_sign():
    # f ~ (1 - 2 m (1 - m)) d for small d: heat flows from hot to cold with the
    # printed sign of Delta e (the opposite sign would give 1 + 2 m (1 - m))
    for m in (0.05, 0.3, 0.5, 0.9):
        d = 1e-6
        f = oracle.pair(m - d / 2, m + d / 2)[0]
        assert f / d == pytest.approx(1 - 2 * m * (1 - m), rel=1e-8)


# --------------------------------------------------------------------- P6 ----
def test_neighbour_shell_counts_perfect_fcc():
    pos, L = W.fcc(5, 5, 5)
    s = W.System(pos=pos, box_lo=np.zeros(3), box_len=L, periodic=np.ones(3, np.int32),
                 T_e0=np.zeros(pos.shape[1]), params=W.default_params())
    for rc, expect in ((0.75 * W.A_LAT, 12), (1.1 * W.A_LAT, 18), (1.2 * W.A_LAT, 18)):
        row, col = _nbrs(s, rc, "cells")
        assert np.all(np.diff(row) == expect)


def test_neighbours_brute_vs_cells_vs_kdtree():
    from scipy.spatial import cKDTree
    w = W.c3(n_cells=6, n_substeps=1)
    s = w.systems[0]
    rb, cb = _nbrs(s, w.r_cut, "brute")
    rcl, ccl = _nbrs(s, w.r_cut, "cells")
    assert np.array_equal(rb, rcl) and np.array_equal(cb, ccl)
    counts = np.diff(rb)
    assert 18 <= counts.min() and counts.max() <= 27
    assert 19.5 < counts.mean() < 21.0         # jittered 1.2a: ~20.2
    # independent library routine: periodic k-d tree pairs
    tree = cKDTree(s.pos.T, boxsize=s.box_len)
    pairs = tree.query_pairs(w.r_cut, output_type="ndarray")
    mine = set()
    for i in range(s.n):
        for j in cb[rb[i]:rb[i + 1]]:
            if i < j:
                mine.add((i, int(j)))
    assert mine == set(map(tuple, pairs.tolist()))


@pytest.mark.parametrize("cells", [2, 3])
def test_neighbours_in_boxes_of_two_and_three_cells(cells):
    """Periodic axes only two or three cells long, where the cell stencil
    wraps onto itself, beside a free axis: the cell list equals brute force,
    and both equal a k-d tree's pairs (its free axis given a period far
    beyond the box, so no pair wraps there)."""
    from scipy.spatial import cKDTree
    rc = 1.1 * W.A_LAT
    rng = np.random.default_rng(40 + cells)
    box = np.array([cells * rc * 1.02, cells * rc * 1.02, 20.0 * rc])
    n = int(4.0 / W.A_LAT ** 3 * np.prod(box))      # the density of FCC nickel
    pos = rng.uniform(0.0, 1.0, (3, n)) * box[:, None]
    per = np.array([1, 1, 0], np.int32)
    rb, cb = oracle.neighbors(pos, np.zeros(3), box, per, rc, method="brute")
    rcl, ccl = oracle.neighbors(pos, np.zeros(3), box, per, rc, method="cells")
    assert np.array_equal(rb, rcl) and np.array_equal(cb, ccl)
    tree = cKDTree(pos.T, boxsize=np.array([box[0], box[1], 10.0 * box[2]]))
    pairs = set(map(tuple, tree.query_pairs(rc, output_type="ndarray").tolist()))
    mine = set((i, int(j)) for i in range(n) for j in cb[rb[i]:rb[i + 1]] if i < j)
    assert mine == pairs and len(pairs) > n


def test_neighbours_free_axis_and_symmetry():
    s = W.c4_slab(900, 0.1)
    row, col = _nbrs(s, 1.1 * W.A_LAT, "cells")
    rb, cb = _nbrs(s, 1.1 * W.A_LAT, "brute")
    assert np.array_equal(row, rb) and np.array_equal(col, cb)
    counts = np.diff(row)
    x = s.pos[0]
    assert np.all(counts[(x > 2 * W.A_LAT) & (x < x.max() - 2 * W.A_LAT)] == 18)
    assert counts[x == 0].max() < 18           # free surface
    # the relation is symmetric
    ii = np.repeat(np.arange(s.n), counts)
    a = set(zip(ii.tolist(), col.tolist()))
    assert a == set((j, i) for i, j in a)


# --------------------------------------------------------------- Eq. 4 ----
def test_lattice_temperature_two_body_closed_form():
    # two atoms in an open box, within the cut-off of each other: the kinetic
    # energy in the centre-of-mass frame is mu |v1 - v2|^2 / 2
    pos = np.array([[0.0, 2.5], [0.0, 0.0], [0.0, 0.0]])
    m = np.array([58.6934, 12.011])
    v = np.array([[0.01, -0.004], [0.002, 0.003], [-0.001, 0.0]])
    row, col = oracle.neighbors(pos, [-10, -10, -10], [30, 30, 30], [0, 0, 0], 3.0)
    T, gated = oracle.lattice_temperature(row, col, v, m, ke_eps=0.0)
    mu = m[0] * m[1] / (m[0] + m[1])
    dv2 = float(((v[:, 0] - v[:, 1]) ** 2).sum())
    ke = 0.5 * mu * dv2 * W.AMU_A2_PER_FS2_IN_EV
    expect = ke / (1.5 * W.K_B * 2)
    np.testing.assert_allclose(T, [expect, expect], rtol=1e-13)
    # the gate compares K_i = 1/2 m_i |v_i - v_com|^2 with epsilon
    K1 = 0.5 * m[0] * (m[1] / (m[0] + m[1])) ** 2 * dv2 * W.AMU_A2_PER_FS2_IN_EV
    _, g_hi = oracle.lattice_temperature(row, col, v, m, ke_eps=K1 * 1.0001)
    _, g_lo = oracle.lattice_temperature(row, col, v, m, ke_eps=K1 * 0.9999)
    assert g_hi[0] == 1 and g_lo[0] == 0


def test_lattice_temperature_translation_and_maxwell():
    w = W.c3(n_cells=8, n_substeps=1)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    # uniform translation carries no thermal energy
    v = np.tile(np.array([[0.013], [-0.002], [0.007]]), (1, s.n))
    T, gated = oracle.lattice_temperature(row, col, v, s.mass)
    assert np.abs(T).max() < 1e-20 and gated.all()
    # Maxwell at 300 K: removing the local COM of N_j atoms leaves
    # (N_j - 1)/N_j of the equipartition energy on average
    v = W.remove_com(W.maxwell_velocities(s.n, 300.0, s.mass, seed=11), s.mass)
    T, _ = oracle.lattice_temperature(row, col, v, s.mass)
    Nj = np.diff(row) + 1.0
    ratio = T / (300.0 * (Nj - 1) / Nj)
    assert abs(ratio.mean() - 1.0) < 0.02
    Tg, _ = oracle.lattice_temperature(row, col, v, s.mass, global_com=True)
    assert abs(Tg.mean() / 300.0 - 1.0) < 0.02


# ------------------------------------------------------------------ P1/P2 ----
def test_uniform_field_is_stationary():
    w = W.c1(n_cells=5)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    p = dict(s.params, g=0.0)
    T0 = np.full(s.n, 1234.5)
    T, _, _ = oracle.run(row, col, T0, s.T_l, p, 200)
    assert np.array_equal(T, T0)
    # with coupling and T_l equal to T_e nothing moves either
    p = dict(s.params, g=1e-3)
    T, _, _ = oracle.run(row, col, T0, T0, p, 200)
    assert np.array_equal(T, T0)


def test_exchange_conserves_sum_T():
    w = W.c3(n_cells=6, n_substeps=1)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    rng = np.random.default_rng(3)
    T0 = rng.uniform(300, 9000, s.n)
    p = dict(s.params, g=0.0, ce_model=W.CE_CONST, ce_const=W.C_NI)
    T, led, bad = oracle.run(row, col, T0, np.full(s.n, 300.0), p, 2000)
    assert bad == 0
    assert abs(T.sum() - T0.sum()) / T0.sum() < 1e-13
    assert T.std() < 0.2 * T0.std()            # it did diffuse


# --------------------------------------------------------------------- P3 ----
def test_coupling_relaxation_constant_c_closed_form():
    w = W.c1(n_cells=4)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    g, c = 2e-4, 0.05
    p = dict(s.params, g=g, ce_model=W.CE_CONST, ce_const=c)
    n = 3000
    T, led, _ = oracle.run(row, col, np.full(s.n, 5000.0), np.full(s.n, 300.0), p, n)
    expect = 300.0 + 4700.0 * (1.0 - p["dt"] * g / c) ** n
    np.testing.assert_allclose(T, expect, rtol=1e-12)
    # the energy handed to the lattice equals the electronic energy lost
    assert led[0] == pytest.approx(c * s.n * (5000.0 - expect), rel=1e-10)


def test_coupling_relaxation_linear_c_implicit_closed_form():
    w = W.c1(n_cells=4)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    gamma, g, Tl, T0 = 1e-4, 1e-3, 300.0, 5000.0
    p = dict(s.params, g=g, ce_model=W.CE_LINEAR, gamma=gamma, dt=0.01)
    n = 40000
    T, _, _ = oracle.run(row, col, np.full(s.n, T0), np.full(s.n, Tl), p, n)
    Tn = T[0]
    assert np.all(T == Tn)
    # gamma T dT/dt = -g (T - T_l)  =>  t = (gamma/g)[(T0 - T) + T_l ln((T0-T_l)/(T-T_l))]
    t = (gamma / g) * ((T0 - Tn) + Tl * math.log((T0 - Tl) / (Tn - Tl)))
    assert t == pytest.approx(n * p["dt"], rel=2e-4)
    assert Tn < 0.5 * T0


# --------------------------------------------------------------------- P4 ----
def test_two_atom_scalar_map():
    pos = np.array([[0.0, 2.6], [0.0, 0.0], [0.0, 0.0]])
    row, col = oracle.neighbors(pos, [-10, -10, -10], [30, 30, 30], [0, 0, 0], 3.0)
    assert np.array_equal(np.diff(row), [1, 1])
    K, dt, Tmax = 0.9465, 0.05, 20000.0
    p = W.default_params(K=K, dt=dt, T_max=Tmax, g=0.0)
    T0 = np.array([2000.0, 14000.0])
    th = T0 / Tmax
    m = th.mean()
    D = th[1] - th[0]
    T = T0.copy()
    for n in range(60):
        T, _, _ = oracle.run(row, col, T, np.zeros(2), p, 1, step0=n)
        # Delta <- Delta - 2 K dt [Delta cosh Delta - (2m(1-m) + Delta^2/2) sinh Delta]
        D = D - 2 * K * dt * (D * math.cosh(D) - (2 * m * (1 - m) + D * D / 2) * math.sinh(D))
        th = T / Tmax
        assert th.mean() == pytest.approx(m, abs=1e-15)
        assert th[1] - th[0] == pytest.approx(D, abs=2e-14)
    # linear limit: small Delta decays at rate 2K(1 - 2m(1-m))
    T0 = np.array([4000.0, 4000.2])
    T, _, _ = oracle.run(row, col, T0, np.zeros(2), p, 100)
    m = T0.mean() / Tmax
    rate = 2 * K * (1 - 2 * m * (1 - m))
    assert (T[1] - T[0]) / 0.2 == pytest.approx((1 - dt * rate) ** 100, rel=1e-7)


# --------------------------------------------------------------------- P5 ----
def _fourier_amplitude(T, x, Lx):
    k = 2 * np.pi / Lx
    return 2.0 / T.size * np.sum((T - T.mean()) * np.sin(k * x))


@pytest.mark.parametrize("amp,tol", [(1.0, 1e-8), (500.0, 2e-4)])
def test_sinusoid_decays_at_lattice_sum_rate(amp, tol):
    # reduced y/z extent: the profile only varies along x
    w = W.c2(nx=200, ny=3, nz=3, amplitude=amp, n_substeps=5000, precision="fp64")
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    T, led, bad = oracle.run(row, col, s.T_e0, s.T_l, s.params, w.n_substeps)
    assert bad == 0
    a = W.A_LAT
    k = 2 * np.pi / s.box_len[0]
    # 1.1a shell: 8 of the 12 nearest neighbours have |r_x| = a/2, 2 of the 6
    # second neighbours have |r_x| = a
    lat = 8 * (1 - math.cos(k * a / 2)) + 2 * (1 - math.cos(k * a))
    th0 = 1000.0 / s.params["T_max"]
    lam = s.params["K"] * (1 - 2 * th0 * (1 - th0)) * lat
    expect = amp * (1 - s.params["dt"] * lam) ** w.n_substeps
    got = _fourier_amplitude(T, s.pos[0], s.box_len[0])
    assert got == pytest.approx(expect, rel=tol)
    if amp == 500.0:
        assert expect == pytest.approx(327.64, abs=0.01)
    assert abs(T.sum() - s.T_e0.sum()) / s.T_e0.sum() < 1e-13


# --------------------------------------------------------------------- P8 ----
def test_laser_source_total_energy_closed_form():
    s = W.c4_slab(2000, 0.3)
    p = dict(s.params, g=0.0, K=0.0)
    row, col = _nbrs(s, 1.1 * W.A_LAT)
    n_steps = 6000                     # t in [0, 300) fs around t0 = 150 fs
    T, led, _ = oracle.run(row, col, s.T_e0, s.T_l, p, n_steps, x=s.pos[0])
    F, lp, sig, t0, dt = p["laser_fluence"], p["laser_lp"], p["laser_sigma"], p["laser_t0"], p["dt"]
    A_yz = s.box_len[1] * s.box_len[2]
    h = W.A_LAT / 2                     # spacing of the (100) atomic planes
    n_planes = int(round((s.pos[0].max() / h))) + 1
    depth = (h / lp) / (1 - math.exp(-h / lp)) * (1 - math.exp(-n_planes * h / lp))
    frac = 0.5 * (math.erf((n_steps * dt - t0) / (math.sqrt(2) * sig))
                  - math.erf((0.0 - t0) / (math.sqrt(2) * sig)))
    assert led[1] == pytest.approx(F * A_yz * depth * frac, rel=1e-6)
    # with K = G = 0 each atom's electronic energy rises by exactly its source
    E0, _ = oracle.energies(s.T_e0, p)
    E1, _ = oracle.energies(T, p)
    assert E1 - E0 == pytest.approx(led[1], rel=2e-3)   # Euler in T, c = gamma T


# ------------------------------------------------------------------ P9/P10 ----
def test_energy_ledger_constant_uniform_c():
    w = W.c1(n_cells=5)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    p = dict(s.params, ce_model=W.CE_CONST, ce_const=W.C_NI, g=5e-6,
             laser_on=1, laser_fluence=0.1, laser_t0=20.0, laser_sigma=10.0, laser_x0=0.0)
    E0, _ = oracle.energies(s.T_e0, p)
    T = s.T_e0
    led = np.zeros(3)
    for k in range(4):
        T, led, _ = oracle.run(row, col, T, s.T_l, p, 250, step0=250 * k, x=s.pos[0], ledger=led)
        E, _ = oracle.energies(T, p)
        assert E + led[0] - led[1] == pytest.approx(E0, rel=1e-12)
    assert led[0] > 0 and led[1] > 0


@pytest.mark.parametrize("model", ["const", "linear", "capped"])
def test_electronic_energy_is_the_integral_of_the_heat_capacity(model):
    """E(T) = integral_0^T c dT' (the electronic energy whose rate of change
    Eq. 6 balances), checked against adaptive quadrature of c itself.  For the
    capped model c = min(gamma T, cap) this fixes the gamma T*^2/2 - cap T*
    offset above T* = cap / gamma, which no energy difference sees."""
    from scipy.integrate import quad
    gamma, cap, c0 = 1e-4, 3.0 * W.K_B, W.C_NI
    c_of = {"const": lambda t: c0, "linear": lambda t: gamma * t,
            "capped": lambda t: min(gamma * t, cap)}[model]
    ce = {"const": W.CE_CONST, "linear": W.CE_LINEAR, "capped": W.CE_CAPPED}[model]
    p = W.default_params(ce_model=ce, ce_const=c0, gamma=gamma, ce_cap=cap)
    Ts = cap / gamma                                   # 2.585 K: where the cap engages
    temps = [0.5 * Ts, Ts, 1.5 * Ts, 300.0, 8036.0, 19999.0]
    for T in temps:
        pts = [Ts] if (model == "capped" and T > Ts) else None
        ref, _ = quad(c_of, 0.0, T, points=pts, epsabs=0.0, epsrel=1e-13, limit=200)
        E, S = oracle.energies(np.array([T]), p)
        assert S == T
        assert E == pytest.approx(ref, rel=1e-12), (model, T)
    if model == "capped":
        # continuous at T*, slope c on both sides (no kink in E, only in c)
        h = 1e-7 * Ts
        lo, _ = oracle.energies(np.array([Ts - h]), p)
        at, _ = oracle.energies(np.array([Ts]), p)
        hi, _ = oracle.energies(np.array([Ts + h]), p)
        assert at == pytest.approx(0.5 * cap * Ts, rel=1e-15)
        assert (at - lo) / h == pytest.approx(cap, rel=1e-6)
        assert (hi - at) / h == pytest.approx(cap, rel=1e-6)
        # the C3 field: every T_e is above T*, so E_e = cap sum T - N cap T*/2
        s = W.c3(n_cells=4).systems[0]
        E, S = oracle.energies(s.T_e0, s.params)
        assert E == pytest.approx(cap * S - s.n * cap * Ts / 2.0, rel=1e-14)


def test_temperature_ledger_any_c():
    s = W.c4_slab(3000, 0.4)
    row, col = _nbrs(s, 1.1 * W.A_LAT)
    p = dict(s.params, g=2e-6)
    T = s.T_e0 + np.linspace(0, 500, s.n)
    S0 = T.sum()
    T, led, bad = oracle.run(row, col, T, s.T_l, p, 3000, x=s.pos[0])
    assert bad == 0
    assert T.sum() + led[2] == pytest.approx(S0, rel=1e-13)


# -------------------------------------------------------------------- P11 ----
def _small_adjoint_case(ce_model):
    w = W.c1(n_cells=3)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    p = dict(s.params, K=0.3, g=3e-4, ce_model=ce_model, ce_const=0.04, gamma=2e-5,
             ce_cap=0.06, laser_on=1, laser_fluence=50.0, laser_t0=2.0, laser_sigma=3.0)
    rng = np.random.default_rng(5)
    T0 = 300.0 + 5000.0 * rng.uniform(0, 1, s.n)
    Tl = 300.0 + 100 * rng.uniform(0, 1, s.n)
    gated = (rng.uniform(0, 1, s.n) < 0.2).astype(np.int32)
    return s, row, col, p, T0, Tl, gated


@pytest.mark.parametrize("ce_model", [W.CE_CONST, W.CE_LINEAR, W.CE_CAPPED])
def test_adjoint_dot_product_and_parameter_gradients(ce_model):
    s, row, col, p, T0, Tl, gated = _small_adjoint_case(ce_model)
    n_steps = 40
    rng = np.random.default_rng(9)
    v = rng.normal(size=s.n)
    wv = rng.normal(size=s.n)
    lam, dK, dg = oracle.adjoint(row, col, T0, Tl, p, n_steps, wv, gated=gated, x=s.pos[0])
    h = 1e-20
    Jv = oracle.run_cs(row, col, T0 + 1j * h * v, Tl, p, n_steps, gated=gated, x=s.pos[0]).imag / h
    assert np.dot(wv, Jv) == pytest.approx(np.dot(lam, v), rel=1e-12)
    dTK = oracle.run_cs(row, col, T0, Tl, p, n_steps, K=p["K"] + 1j * h, gated=gated,
                        x=s.pos[0]).imag / h
    dTg = oracle.run_cs(row, col, T0, Tl, p, n_steps, g=p["g"] + 1j * h, gated=gated,
                        x=s.pos[0]).imag / h
    assert dK == pytest.approx(np.dot(wv, dTK), rel=1e-11)
    assert dg == pytest.approx(np.dot(wv, dTg), rel=1e-11)
    # central finite differences on the real forward run
    def L(pp):
        T, _, _ = oracle.run(row, col, T0, Tl, pp, n_steps, gated=gated, x=s.pos[0])
        return float(np.dot(wv, T))
    eK = 1e-6 * p["K"]
    fdK = (L(dict(p, K=p["K"] + eK)) - L(dict(p, K=p["K"] - eK))) / (2 * eK)
    eg = 1e-6 * p["g"]
    fdg = (L(dict(p, g=p["g"] + eg)) - L(dict(p, g=p["g"] - eg))) / (2 * eg)
    assert dK == pytest.approx(fdK, rel=1e-6)
    assert dg == pytest.approx(fdg, rel=1e-6)


def test_adjoint_conservation_special_case():
    # G = 0 and no source: sum T^N = sum T^0 for every K, so with L = sum T^N
    # dL/dT0 = 1 exactly and dL/dK = 0 up to rounding
    s, row, col, p, T0, Tl, gated = _small_adjoint_case(W.CE_CONST)
    p = dict(p, g=0.0, laser_on=0)
    lam, dK, dg = oracle.adjoint(row, col, T0, Tl, p, 30, np.ones(s.n))
    assert np.all(lam == 1.0)
    assert abs(dK) < 1e-9 * np.abs(T0).sum()


# -------------------------------------------------------------------- P12 ----
def test_fcc_laplacian_spectrum_and_euler_stability_bound():
    w = W.c1(n_cells=4)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    A = np.zeros((s.n, s.n))
    A[np.repeat(np.arange(s.n), np.diff(row)), col] = 1.0
    lap = np.diag(A.sum(1)) - A
    lam_max = np.linalg.eigvalsh(lap).max()
    assert lam_max == pytest.approx(24.0, abs=1e-9)
    rng = np.random.default_rng(1)
    T0 = 100.0 + 1e-3 * rng.normal(size=s.n)    # theta ~ 0: c(theta) ~ 1
    for kdt, grows in ((2.2 / lam_max, True), (1.8 / lam_max, False)):
        p = dict(s.params, K=kdt / s.params["dt"], g=0.0)
        T, _, _ = oracle.run(row, col, T0, s.T_l, p, 50)
        dev0 = np.abs(T0 - T0.mean()).max()
        dev = np.abs(T - T.mean()).max()
        assert (dev > 100 * dev0) if grows else (dev < 0.5 * dev0)


# ---------------------------------------------------- paper constants (Eq. 3) ----
def test_paper_constants_give_per_atom_values():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    a = W.A_LAT * 1e-10
    v_atom = a ** 3 / 4
    eV = 1.602176634e-19
    g = c["G_W_per_m3K"]["value"] * v_atom / eV * 1e-15
    ce = c["Ce_J_per_m3K"]["value"] * v_atom / eV
    assert g == pytest.approx(W.G_NI, rel=1e-4)
    assert ce == pytest.approx(W.C_NI, rel=1e-4)
    # Eq. 3: K = 2 kappa d / (C_e Z b^2); for a multi-shell cut-off Z b^2 is
    # the lattice sum of |r|^2 over the neighbour set, 12 a^2 at 1.1a
    pos, L = W.fcc(3, 3, 3)
    row, col = oracle.neighbors(pos, np.zeros(3), L, [1, 1, 1], 1.1 * W.A_LAT)
    d = pos[:, col[row[0]:row[1]]] - pos[:, [0]]
    d -= L[:, None] * np.round(d / L[:, None])
    lat = float((d ** 2).sum()) * 1e-20
    assert lat == pytest.approx(12 * a * a, rel=1e-12)
    K = 2 * c["kappa_e_W_per_mK"]["value"] * c["d_md"]["value"] / (c["Ce_J_per_m3K"]["value"] * lat)
    assert K * 1e-15 == pytest.approx(W.K_NI, rel=1e-4)


# ------------------------------------------------- lattice side: Eq. 5, Eq. 8 ----
MVV2E = W.AMU_A2_PER_FS2_IN_EV


def _kinetic(vel, mass):
    """1/2 m |v|^2 per atom in eV (vel (3, n) A/fs, mass amu)."""
    return 0.5 * mass * (vel * vel).sum(axis=0) * MVV2E


def _isolated_atoms(n=300, seed=11):
    """Atoms farther apart than the cut-off: no exchange, pure relaxation."""
    rng = np.random.default_rng(seed)
    T0 = rng.uniform(500.0, 8000.0, n)
    Tl = rng.uniform(100.0, 3000.0, n)
    gated = (rng.uniform(0, 1, n) < 0.15).astype(np.int32)
    row = np.zeros(n + 1, np.int64)
    col = np.zeros(0, np.int32)
    return row, col, T0, Tl, gated


def test_atom_ledger_isolated_atoms_closed_form():
    row, col, T0, Tl, gated = _isolated_atoms()
    g, c, n = 3e-4, 0.05, 700
    p = W.default_params(g=g, ce_model=W.CE_CONST, ce_const=c)
    e = np.zeros(T0.size)
    T, led, bad = oracle.run(row, col, T0, Tl, p, n, gated=gated, e_atom=e)
    assert bad == 0
    # T_i^n = T_l + (T_0 - T_l)(1 - a)^n with a = dt g / c; the energy handed
    # over is the heat-capacity drop c (T_0 - T^n); gated atoms keep T_0
    decay = (1.0 - p["dt"] * g / c) ** n
    free = gated == 0
    np.testing.assert_allclose(e[free], c * (T0 - Tl)[free] * (1.0 - decay), rtol=1e-11)
    assert np.all(e[~free] == 0.0) and np.array_equal(T[~free], T0[~free])
    assert led[0] == pytest.approx(e.sum(), rel=1e-12)


def test_xi_ledger_mode_one_substep_is_eq8_before_the_step():
    # after one sub-step the recorded energy is g (T_0 - T_l) dt, so the
    # ledger form over dt_md = dt equals Eq. 8 evaluated on the state T_0
    row, col, T0, Tl, gated = _isolated_atoms(seed=12)
    p = W.default_params(g=2e-4, ce_model=W.CE_LINEAR, gamma=1e-4)
    mass = np.full(T0.size, W.MASS_NI)
    vel = W.maxwell_velocities(T0.size, 600.0, mass, seed=13)
    vel[:, :5] *= 1e-4                         # kinetic energy below epsilon
    e = np.zeros(T0.size)
    oracle.run(row, col, T0, Tl, p, 1, gated=gated, e_atom=e)
    xl = oracle.coupling(oracle.XI_LEDGER, T0, Tl, gated, e, p["g"], p["dt"], p["ke_eps"], vel, mass)
    xi = oracle.coupling(oracle.XI_INSTANT, T0, Tl, gated, None, p["g"], p["dt"], p["ke_eps"], vel,
                         mass)
    np.testing.assert_allclose(xl, xi, rtol=1e-13, atol=0)
    K = _kinetic(vel, mass)
    off = (gated == 1) | (K < p["ke_eps"])
    assert off[:5].all() and np.all(xi[off] == 0.0) and np.all(xi[~off] != 0.0)
    # heating where T_e > T_l, cooling where T_e < T_l
    assert np.array_equal(np.sign(xi[~off]), np.sign((T0 - Tl)[~off]))


def _coupled_md_step():
    w = W.c3(n_cells=5, n_substeps=1)
    s = w.systems[0]
    row, col = _nbrs(s, w.r_cut)
    p = dict(s.params, g=4e-5, ce_model=W.CE_CONST, ce_const=W.C_NI * 40)
    Tl, gated = oracle.lattice_temperature(row, col, s.vel, s.mass, p["ke_eps"])
    return s, row, col, p, Tl, gated


def test_damping_work_matches_atom_ledger_exactly():
    # one explicit step v' = v (1 + xi dt_md) without forces changes the
    # kinetic energy by K ((1 + xi dt_md)^2 - 1) = 2 xi K dt_md + (xi dt_md)^2 K,
    # which with xi = E / (2 K dt_md) is E + E^2 / (4 K): the energy the atom's
    # electrons handed over, plus a second-order remainder
    s, row, col, p, Tl, gated = _coupled_md_step()
    n_sub = 10
    dt_md = n_sub * p["dt"]
    e = np.zeros(s.n)
    T, led, bad = oracle.run(row, col, s.T_e0, Tl, p, n_sub, gated=gated, e_atom=e)
    assert bad == 0
    xi = oracle.coupling(oracle.XI_LEDGER, T, Tl, gated, e, p["g"], dt_md, p["ke_eps"], s.vel,
                         s.mass)
    v1 = oracle.damping_step(dt_md, xi, None, s.mass, s.vel)
    K0, K1 = _kinetic(s.vel, s.mass), _kinetic(v1, s.mass)
    on = xi != 0.0
    assert on.sum() > 0.9 * s.n
    np.testing.assert_allclose((K1 - K0)[on], (e + e * e / (4.0 * K0))[on], rtol=1e-9)
    assert np.array_equal(v1[:, ~on], s.vel[:, ~on])
    assert np.all(e[~on] == 0.0)


def test_md_step_energy_balance_second_order_remainder():
    # constant uniform c, no source: the exchange conserves sum T, so the
    # electrons lose exactly sum_i E_i; the damped lattice gains
    # sum_i E_i + E_i^2 / (4 K_i).  The total changes by the remainder only.
    s, row, col, p, Tl, gated = _coupled_md_step()
    p = dict(p, g=4e-6)                    # xi dt_md well below 1: a small remainder
    n_sub = 20
    dt_md = n_sub * p["dt"]
    E0, _ = oracle.energies(s.T_e0, p)
    e = np.zeros(s.n)
    T, led, _ = oracle.run(row, col, s.T_e0, Tl, p, n_sub, gated=gated, e_atom=e)
    E1, _ = oracle.energies(T, p)
    xi = oracle.coupling(oracle.XI_LEDGER, T, Tl, gated, e, p["g"], dt_md, p["ke_eps"], s.vel,
                         s.mass)
    v1 = oracle.damping_step(dt_md, xi, None, s.mass, s.vel)
    K0 = _kinetic(s.vel, s.mass)
    dKE = _kinetic(v1, s.mass).sum() - K0.sum()
    rem = np.where(xi != 0.0, e * e / (4.0 * K0), 0.0).sum()
    assert (E1 - E0) == pytest.approx(-e.sum(), rel=1e-10)
    assert (E1 - E0) + dKE == pytest.approx(rem, rel=1e-6, abs=1e-12 * abs(E1 - E0))
    assert 0.0 < rem < 5e-2 * abs(E1 - E0)


def test_damping_step_force_obeys_newton_in_md_units():
    # without damping, the momentum change over dt_md is dt_md * sum F in
    # amu A/fs, with F in eV/A converted by 1 amu A^2/fs^2 = 103.6427 eV
    rng = np.random.default_rng(21)
    n = 500
    mass = rng.uniform(20.0, 200.0, n)
    vel = rng.normal(0.0, 0.01, (3, n))
    force = rng.normal(0.0, 0.5, (3, n))
    dt = 0.7
    v1 = oracle.damping_step(dt, np.zeros(n), force, mass, vel)
    dp = ((v1 - vel) * mass[None, :]).sum(axis=1)
    np.testing.assert_allclose(dp, dt * force.sum(axis=1) / MVV2E, rtol=1e-12)
    # a uniform xi scales every velocity by (1 + xi dt) and leaves directions
    v2 = oracle.damping_step(dt, np.full(n, 0.05), None, mass, vel)
    np.testing.assert_allclose(v2, vel * (1.0 + 0.05 * dt), rtol=1e-15)


# ---------------------- Section 2 mean-field mode, Section 4 fixed electrons ----
def _bar(nx=16, nyz=3):
    """FCC bar, periodic in y and z, free in x."""
    pos, L = W.fcc(nx, nyz, nyz)
    lo = np.array([-0.25 * W.A_LAT, 0.0, 0.0])
    box = np.array([L[0] + 0.5 * W.A_LAT, L[1], L[2]])
    return pos, lo, box, np.array([0, 1, 1], np.int32)


def test_fixed_atoms_hold_and_temperature_ledger_books_their_exchange():
    s = W.c4_slab(3000, 0.4)
    row, col = _nbrs(s, 1.1 * W.A_LAT)
    p = dict(s.params, g=2e-6)
    x = s.pos[0]
    T0 = s.T_e0 + np.linspace(0, 500, s.n)
    fixed = ((x < x.min() + W.A_LAT) | (x > x.max() - W.A_LAT)).astype(np.int32)
    assert 0 < fixed.sum() < s.n // 2
    T, led, bad = oracle.run(row, col, T0, s.T_l, p, 3000, x=x, fixed=fixed)
    assert bad == 0
    held = fixed == 1
    assert np.array_equal(T[held], T0[held])
    assert not np.allclose(T[~held], T0[~held])
    # the exchange sums to zero over all atoms, so the held atoms' share booked
    # in the temperature ledger keeps sum T + ledger invariant
    assert T.sum() + led[2] == pytest.approx(T0.sum(), rel=1e-13)


def test_fixed_ends_relax_bar_to_the_linear_steady_profile():
    # small amplitude around 3,000 K, no coupling: the linearised exchange on a
    # centrosymmetric lattice annihilates any linear profile, so with the two
    # end cells held on a line the free atoms converge onto that line
    pos, lo, box, per = _bar()
    row, col = oracle.neighbors(pos, lo, box, per, 1.1 * W.A_LAT)
    x = pos[0]
    delta = 5.0
    line = 3000.0 + delta * (2.0 * (x - x.min()) / (x.max() - x.min()) - 1.0)
    fixed = ((x < x.min() + 0.9 * W.A_LAT) | (x > x.max() - 0.9 * W.A_LAT)).astype(np.int32)
    rng = np.random.default_rng(41)
    T0 = np.where(fixed == 1, line, 3000.0 + rng.uniform(-delta, delta, x.size))
    p = W.default_params(g=0.0, ce_model=W.CE_CONST, ce_const=W.C_NI)
    T1, _, _ = oracle.run(row, col, T0, np.full(x.size, 300.0), p, 6000, fixed=fixed)
    T2, _, _ = oracle.run(row, col, T1, np.full(x.size, 300.0), p, 2000, step0=6000, fixed=fixed)
    free = fixed == 0
    assert np.max(np.abs(T2 - T1)[free]) < 1e-6 * delta          # converged
    # the O((dT/T_max)^2) nonlinearity of the pair term bends it by < 1e-3 delta
    assert np.max(np.abs(T2 - line)[free]) < 1e-3 * delta


def test_mean_field_rate_drops_mean_Te_and_matches_eq3_in_si():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    a = W.A_LAT * 1e-10
    v_atom = a ** 3 / 4
    eV = 1.602176634e-19
    lam = c["lambda_J_per_m3K2"]["value"]
    kap0 = c["kappa_e_W_per_mK"]["value"]
    d = c["d_md"]["value"]
    S = 12 * a * a                        # lattice sum of the 1.1a shell (pinned above)
    lam_atom = lam * v_atom / eV          # eV/K^2 per atom
    k_coef = 2 * d * kap0 / (lam * S) * 1e-15   # K/fs
    rng = np.random.default_rng(43)
    Tl = rng.uniform(250.0, 350.0, 400)
    Ks = []
    for Te_mean in (400.0, 3000.0, 9000.0):
        T = rng.normal(Te_mean, 40.0, 400)
        cc, K = oracle.mean_field(T, Tl, lam_atom, k_coef)
        # Eq. 3 in SI with the Section 2 relations kappa_e = kappa_0 Te / Tl, C_e = lambda Te
        Te_b, Tl_b = T.mean(), Tl.mean()
        K_si = 2 * (kap0 * Te_b / Tl_b) * d / ((lam * Te_b) * S)
        assert K == pytest.approx(K_si * 1e-15, rel=1e-12)
        assert cc == pytest.approx(lam * Te_b * v_atom / eV, rel=1e-12)
        Ks.append(K)
    assert Ks[0] == pytest.approx(Ks[1], rel=1e-14) == pytest.approx(Ks[2], rel=1e-14)
    # at T_e = T_lat = C_e / lambda the mean-field rate is the Section 3.1 constant K
    Teq = c["Ce_J_per_m3K"]["value"] / lam
    _, K_eq = oracle.mean_field(np.full(10, Teq), np.full(10, Teq), lam_atom, k_coef)
    assert K_eq == pytest.approx(W.K_NI, rel=1e-4)


def test_mean_field_heat_capacity_sets_relaxation_of_uniform_system():
    row, col, _, _, _ = _isolated_atoms(n=50)
    T0, Tl = np.full(50, 5000.0), np.full(50, 300.0)
    cc, K = oracle.mean_field(T0, Tl, 1e-5, 300.0)
    p = W.default_params(g=2e-4, K=K, ce_model=W.CE_CONST, ce_const=cc)
    T, led, _ = oracle.run(row, col, T0, Tl, p, 500)
    # c = lambda mean(T_e) = 0.05 eV/K held over the advance
    np.testing.assert_allclose(T, 300.0 + 4700.0 * (1.0 - p["dt"] * 2e-4 / 0.05) ** 500, rtol=1e-12)


# ------------------------------------------- two-temperature bar, Section 3.1 ----
def _bar_system():
    w = W.c6(n_bars=1)
    s = w.systems[0]
    row, col = oracle.neighbors(s.pos, s.box_lo, s.box_len, s.periodic, w.r_cut)
    assert np.all(np.diff(row) == 2)                  # the chain's two neighbours
    return w, s, row, col


def test_bar_means_relax_to_the_papers_equilibrium_in_closed_form():
    # the electron exchange and the lattice stencil both conserve their sums,
    # so D = mean(T_e) - mean(T_l) obeys D_n = D_0 (1 - dt (g/c_e + g/c_l))^n
    # and c_e mean(T_e) + c_l mean(T_l) is conserved: both means approach
    # T_eq = (C_e <T_e0> + rho C_l <T_l0>) / (C_e + rho C_l) (Section 3.1)
    w, s, row, col = _bar_system()
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    Ce = c["Ce_J_per_m3K"]["value"]
    rhoCl = 8890.0 * 400.0                       # Section 3.1: rho = 8890 kg/m^3, C_l = 400 J/kg/K
    Teq = (Ce * s.T_e0.mean() + rhoCl * s.T_l.mean()) / (Ce + rhoCl)
    n = 12000
    T, Tl, led, bad = oracle.run_2t(row, col, s.T_e0, s.T_l, s.params, w.extra["K_lat"],
                                    w.extra["c_lat"], n)
    assert bad == 0
    g, ce, cl, dt = s.params["g"], s.params["ce_const"], w.extra["c_lat"], s.params["dt"]
    Dn = (s.T_e0.mean() - s.T_l.mean()) * (1.0 - dt * (g / ce + g / cl)) ** n
    assert T.mean() == pytest.approx(Teq + rhoCl / (Ce + rhoCl) * Dn, rel=1e-12)
    assert Tl.mean() == pytest.approx(Teq - Ce / (Ce + rhoCl) * Dn, rel=1e-12)
    # the energy the lattice received is the electrons' loss
    assert cl * (Tl.mean() - s.T_l.mean()) * s.n == pytest.approx(led[0], rel=1e-11)


def test_bar_lattice_fourier_modes_decay_at_the_stencil_rate():
    # no coupling: the lattice alone is the forward-Euler three-point Fourier
    # law on a ring, whose cosines decay by 1 - dt K_l (2 - 2 cos(2 pi k / N))
    w, s, row, col = _bar_system()
    N = s.n
    x = np.arange(N)
    p = dict(s.params, g=0.0)
    for k in (1, 5, 40):
        Tl0 = 300.0 + 20.0 * np.cos(2 * np.pi * k * x / N)
        _, Tl, _, _ = oracle.run_2t(row, col, np.full(N, 300.0), Tl0, p, w.extra["K_lat"],
                                    w.extra["c_lat"], 3000)
        r = (1.0 - p["dt"] * w.extra["K_lat"] * (2.0 - 2.0 * np.cos(2 * np.pi * k / N))) ** 3000
        np.testing.assert_allclose(Tl, 300.0 + 20.0 * r * np.cos(2 * np.pi * k * x / N),
                                   rtol=0, atol=1e-10)
