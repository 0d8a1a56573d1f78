"""GPU parity of the electronic energy E_e = sum_i integral_0^{T_i} c dT
(the energy whose balance Eq. 6 states) and of the energy ledger.

Each case runs the library and the FP64 oracle from the same seeded input and
compares:
  - the library's E_e with the oracle's energy of the oracle's own state, to
    the trajectory tolerance (FP64 1e-12; FP32C 2e-5, since E grows like T^2
    under c = gamma T, so a 1e-5 relative error in T can double);
  - the library's E_e with the oracle's energy of the library's own state, to
    FP64 summation order (1e-12): this isolates the device reduction and the
    per-atom energy, including the capped branch gamma T*^2/2 + cap (T - T*);
  - with a constant uniform c, E_e + E_e->l - E_src against its initial value
    (the balance of Eq. 6 with the Eq. 10 source): 1e-12 in FP64, 1e-6 in
    FP32C, whose ledger terms are FP32 per lane with FP32 wave sums.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_context, gpu_trajectory, oracle_trajectory

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1810_12357_amd.l2t")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(model):
    if model == "const":          # C2 recipe, reduced in y and z
        w = W.c2(nx=60, ny=3, nz=3, amplitude=500.0, n_substeps=1500)
        cps = [500, 1500]
    elif model == "linear":       # C1 recipe
        w = W.c1(n_cells=6, n_substeps=600)
        cps = [100, 600]
    else:                         # C3 recipe (capped c), reduced
        w = W.c3(n_cells=8, n_substeps=800)
        cps = [200, 800]
    return w, cps


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
@pytest.mark.parametrize("model", ["const", "linear", "capped"])
def test_electronic_energy_equals_oracle(model, precision):
    w, cps = _case(model)
    sy = w.systems[0]
    p = sy.params
    assert p["ce_model"] == {"const": W.CE_CONST, "linear": W.CE_LINEAR,
                             "capped": W.CE_CAPPED}[model]
    traj, led, bad = oracle_trajectory(sy, w.r_cut, cps)
    assert bad == 0
    prec = L.L2T_FP64 if precision == "fp64" else L.L2T_FP32C
    ctx = gpu_context(w, prec)
    e0 = ctx.energies(0)
    E_init, _ = oracle.energies(sy.T_e0, p)
    assert e0["E_e"] == pytest.approx(E_init, rel=1e-12)
    tol = 1e-12 if precision == "fp64" else 2e-5
    step = 0
    for c, To in zip(cps, traj):
        ctx.advance(c - step)
        step = c
        e = ctx.energies(0)
        Tg = ctx.get(0)
        E_or, S_or = oracle.energies(To, p)
        assert e["E_e"] == pytest.approx(E_or, rel=tol), (model, precision, c)
        E_own, S_own = oracle.energies(Tg, p)
        assert e["E_e"] == pytest.approx(E_own, rel=1e-12)
        assert e["sum_T"] == pytest.approx(S_own, rel=1e-12)
        assert e["T_max_atom"] == Tg.max() and e["T_min_atom"] == Tg.min()
    if model == "capped":
        # every atom sits above T* = cap/gamma, so the energy is affine in T
        cap, Ts = p["ce_cap"], p["ce_cap"] / p["gamma"]
        assert Tg.min() > Ts
        assert e["E_e"] == pytest.approx(cap * e["sum_T"] - sy.n * cap * Ts / 2, rel=1e-12)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_energy_balance_constant_uniform_c(precision):
    """P9: with one constant c for every atom, E_e + E_e->l - E_src holds its
    initial value through coupling and laser heating."""
    w = W.c1(n_cells=6, n_substeps=1000)
    sy = w.systems[0]
    sy.params = dict(sy.params, ce_model=W.CE_CONST, ce_const=W.C_NI, g=5e-6, laser_on=1,
                     laser_fluence=0.1, laser_t0=20.0, laser_sigma=10.0, laser_x0=0.0)
    prec = L.L2T_FP64 if precision == "fp64" else L.L2T_FP32C
    ctx = gpu_context(w, prec)
    E0 = ctx.energies(0)["E_e"]
    E_init, _ = oracle.energies(sy.T_e0, sy.params)
    assert E0 == pytest.approx(E_init, rel=1e-12)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for k in range(4):
        ctx.advance(250)
        e = ctx.energies(0)
        assert e["E_e"] + e["E_e_to_l"] - e["E_src"] == pytest.approx(E0, rel=tol), k
    assert e["E_e_to_l"] > 0 and e["E_src"] > 0
    # and the ledger totals are the oracle's
    traj, led, bad = oracle_trajectory(sy, w.r_cut, [1000])
    lt = 1e-10 if precision == "fp64" else 1e-5
    assert e["E_e_to_l"] == pytest.approx(led[0], rel=lt)
    assert e["E_src"] == pytest.approx(led[1], rel=lt)
    ctx.close()


def test_energy_of_a_batch_each_system_its_own_model():
    """Three systems with the three heat-capacity models in one FP32C context:
    each report is the oracle's energy of that system's state."""
    systems = [_case(m)[0].systems[0] for m in ("const", "linear", "capped")]
    # one cut-off for the batch: the largest
    r_cut = max(_case(m)[0].r_cut for m in ("const", "linear", "capped"))
    ctx = L.Context(systems, L.L2T_FP32C)
    ctx.setup(r_cut)
    ctx.advance(300)
    for s, sy in enumerate(systems):
        e = ctx.energies(s)
        E_own, _ = oracle.energies(ctx.get(s), sy.params)
        assert e["E_e"] == pytest.approx(E_own, rel=1e-12), s
    ctx.close()
