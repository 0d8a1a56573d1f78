"""Full-size batch and gradient workloads, launched as the benchmark launches
them, checked on sampled systems against the FP64 oracle and on every system
against properties that hold at any size."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_context, max_rel, oracle_lattice, oracle_neighbors, oracle_trajectory

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

L = pytest.importorskip("paper_1810_12357_amd.l2t")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _laser_energy_closed_form(sy, n_steps):
    """Energy a slab absorbs from the Eq. 10 source over n_steps sub-steps:
    the depth sum over (100) planes spaced a/2 is a geometric series and the
    Gaussian time factor integrates to the error-function window."""
    p = sy.params
    F, lp, sig, t0, dt = p["laser_fluence"], p["laser_lp"], p["laser_sigma"], p["laser_t0"], p["dt"]
    A_yz = sy.box_len[1] * sy.box_len[2]
    h = W.A_LAT / 2
    n_planes = int(round(sy.pos[0].max() / h)) + 1
    depth = (h / lp) / (1 - math.exp(-h / lp)) * (1 - math.exp(-n_planes * h / lp))
    frac = 0.5 * (math.erf((n_steps * dt - t0) / (math.sqrt(2) * sig))
                  - math.erf((0.0 - t0) / (math.sqrt(2) * sig)))
    return F * A_yz * depth * frac


def test_c4_full_batch_sampled_systems_and_ledgers():
    w = W.c4()                                   # 256 slabs, 7.9M atoms, 6,000 sub-steps
    ctx = gpu_context(w, L.L2T_FP32C)
    ctx.advance(w.n_substeps)
    L.l2t_sync(ctx.h)
    sizes = np.array([sy.n for sy in w.systems])
    for s, sy in enumerate(w.systems):
        e = ctx.energies(s)
        assert e["step"] == w.n_substeps
        assert e["sum_T"] + e["T_ledger_acc"] == pytest.approx(sy.T_e0.sum(), rel=1e-7)
        assert e["E_src"] == pytest.approx(_laser_energy_closed_form(sy, w.n_substeps), rel=2e-4)
        assert 300.0 <= e["T_min_atom"] and e["T_max_atom"] < 1000.0
    # oracle trajectories over the whole length: the five smallest systems, the
    # median one and the largest (200,704 atoms), every atom
    order = np.argsort(sizes, kind="stable")
    for s in list(order[:5]) + [order[len(order) // 2], order[-1]]:
        sy = w.systems[int(s)]
        traj, led, bad = oracle_trajectory(sy, w.r_cut, [w.n_substeps])
        assert bad == 0
        assert max_rel(ctx.get(int(s)), traj[0]) < 1e-5, (int(s), sy.n)
        e = ctx.energies(int(s))
        assert e["E_src"] == pytest.approx(led[1], rel=1e-5)
        assert e["E_e_to_l"] == pytest.approx(led[0], rel=1e-5)


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_c2_full_size_every_atom_against_the_oracle(precision):
    """Fourier-limit workload at its full size (200 x 8 x 8 cells, 51,200
    atoms) over all 5,000 sub-steps, every atom against the oracle at three
    points, plus the energy of the state (constant c: E_e = c sum T)."""
    w = W.c2(precision=precision)
    sy = w.systems[0]
    cps = [1000, 2500, 5000]
    traj, led, bad = oracle_trajectory(sy, w.r_cut, cps)
    assert bad == 0
    ctx = gpu_context(w, L.L2T_FP64 if precision == "fp64" else L.L2T_FP32C)
    tol = 1e-12 if precision == "fp64" else 1e-5
    step = 0
    for c, To in zip(cps, traj):
        ctx.advance(c - step)
        step = c
        assert max_rel(ctx.get(0), To) < tol, c
    e = ctx.energies(0)
    E_or, S_or = oracle.energies(traj[-1], sy.params)
    assert e["E_e"] == pytest.approx(E_or, rel=tol)
    assert e["sum_T"] == pytest.approx(sy.T_e0.sum(), rel=1e-12 if precision == "fp64" else 1e-8)
    ctx.close()


def test_c5_full_adjoint_sampled_systems():
    w = W.c5()                                   # 64 x 32,000 atoms, 2,000 sub-steps
    n, ck = w.n_substeps, w.checkpoint_every
    ctx = L.Context(w.systems, L.L2T_FP32C)
    ctx.setup(w.r_cut)
    L.l2t_advance_recorded(ctx.h, n, ck)
    TN = [ctx.get(s) for s in range(len(w.systems))]
    sampled = (0, 21, 37, 63)
    N = sum(sy.n for sy in w.systems)
    targets = {}
    for s in sampled:
        sy = w.systems[s]
        row, col = oracle_neighbors(sy, w.r_cut)
        K, g = w.extra["target_params"][s]
        targets[s], _, _ = oracle.run(row, col, sy.T_e0, sy.T_l, dict(sy.params, K=K, g=g), n)
    # the systems not compared take their initial field as target
    dL = np.concatenate([2.0 * (TN[s] - targets.get(s, w.systems[s].T_e0)) / N
                         for s in range(len(w.systems))])
    dT0 = np.zeros(N)
    dK, dg = L.l2t_adjoint(ctx.h, dL, len(w.systems), dL_dT0=dT0)
    off = np.cumsum([0] + [sy.n for sy in w.systems])
    for s in sampled:
        sy = w.systems[s]
        row, col = oracle_neighbors(sy, w.r_cut)
        lam, oK, og = oracle.adjoint(row, col, sy.T_e0, sy.T_l, sy.params, n,
                                     dL[off[s]:off[s + 1]])
        assert dK[s] == pytest.approx(oK, rel=1e-4)
        assert dg[s] == pytest.approx(og, rel=1e-4)
        seg = dT0[off[s]:off[s + 1]]
        assert np.max(np.abs(seg - lam)) < 1e-4 * np.abs(lam).max()
    # the loss falls along -grad for the sampled systems (sanity of direction)
    assert np.isfinite(dK).all() and np.isfinite(dg).all()


def test_c3_full_length_sampled_against_the_stored_oracle_run():
    """The 4,000,000-atom system over all 10,000 sub-steps of the benchmark, in
    the benchmark's launch configuration, against the FP64 oracle's states of
    sampled atoms and its system energy and ledger at 1,000, 2,500, 5,000 and
    10,000 sub-steps (tests/golden/c3_long.json, written by make_c3_long.py
    from the oracle alone)."""
    with open(os.path.join(GOLDEN, "c3_long.json")) as fh:
        ref = json.load(fh)
    w = W.c3()
    ctx = gpu_context(w, L.L2T_FP32C)
    idx = np.asarray(ref["atoms"], dtype=np.int64)
    step = 0
    for cp in ref["checkpoints"]:
        assert cp["out_of_range"] == 0
        ctx.advance(cp["step"] - step)
        step = cp["step"]
        T = ctx.get(0)
        To = np.asarray(cp["T"])
        assert max_rel(T[idx], To) < 1e-5, step
        e = ctx.energies(0)
        assert e["E_e"] == pytest.approx(cp["E_e"], rel=1e-5)
        assert e["sum_T"] == pytest.approx(cp["sum_T"], rel=1e-8)
        assert e["E_e_to_l"] == pytest.approx(cp["E_e_to_l"], rel=1e-5)
        assert e["sum_T"] + e["T_ledger_acc"] == pytest.approx(cp["sum_T"] + cp["T_ledger"],
                                                                rel=1e-9)
        assert e["T_max_atom"] == pytest.approx(cp["T_max"], rel=1e-5)
        assert e["T_min_atom"] == pytest.approx(cp["T_min"], rel=1e-5)
    ctx.close()
