"""Fixed electronic temperatures (the Dirichlet electronic boundary of
Section 4) and the mean-field parameter mode of Section 2, through the C ABI
against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_context, max_rel, oracle_neighbors

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1810_12357_amd.l2t")

TOL = {0: 1e-12, 1: 1e-5}             # FP64, FP32C
LEDGER_TOL = {0: 1e-12, 1: 1e-7}
LAMBDA_ATOM = 1065.0 * (W.V_ATOM * 1e-30) / 1.602176634e-19     # eV/K^2 per atom (Section 3.2)
K_COEF = 2 * 3 * 91.0 / (1065.0 * 12 * (W.A_LAT * 1e-10) ** 2) * 1e-15   # K/fs


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _slab_with_held_ends():
    w = W.c4(n_systems=2, n_substeps=2000, size_lo=2000, size_hi=5000)
    fixed = []
    for sy in w.systems:
        sy.params = dict(sy.params, g=2e-6)
        x = sy.pos[0]
        sy.T_e0 = sy.T_e0 + np.linspace(0.0, 800.0, sy.n)
        fixed.append(((x < x.min() + W.A_LAT) | (x > x.max() - W.A_LAT)).astype(np.int32))
    return w, fixed


@pytest.mark.parametrize("precision", [L.L2T_FP64, L.L2T_FP32C])
def test_held_atoms_match_oracle_and_keep_the_ledger(precision):
    w, fixed = _slab_with_held_ends()
    ctx = gpu_context(w, precision)
    for s in range(len(w.systems)):
        L.l2t_set_field(ctx.h, s, L.L2T_FIELD_FIXED, fixed[s].astype(np.float64))
        assert np.array_equal(ctx.get(s, L.L2T_FIELD_FIXED), fixed[s].astype(np.float64))
    n = w.n_substeps
    # the stored state (FP64, or the FP32C hi and its 16-bit low part) the held atoms keep
    start = [ctx.get(s) for s in range(len(w.systems))]
    if precision == L.L2T_FP64:
        for s in range(len(w.systems)):
            L.l2t_advance_system(ctx.h, s, n)
    else:
        ctx.advance(n)
    for s, sy in enumerate(w.systems):
        row, col = oracle_neighbors(sy, w.r_cut)
        T, led, bad = oracle.run(row, col, sy.T_e0, sy.T_l, sy.params, n, x=sy.pos[0],
                                 fixed=fixed[s])
        got = ctx.get(s)
        held = fixed[s] == 1
        assert np.array_equal(got[held], start[s][held])
        assert max_rel(got, T) < TOL[precision]
        e = ctx.energies(s)
        assert e["sum_T"] + e["T_ledger_acc"] == pytest.approx(sy.T_e0.sum(),
                                                               rel=LEDGER_TOL[precision])
        assert e["T_ledger_acc"] == pytest.approx(led[2], rel=1e-5 if precision else 1e-10)
    ctx.close()


def test_held_atoms_bitwise_equal_across_launch_forms():
    w = W.c3(n_cells=9, n_substeps=1)
    sy = w.systems[0]
    r2 = ((sy.pos - (sy.box_len / 2)[:, None]) ** 2).sum(0)
    fixed = (r2 > 12.0 ** 2).astype(np.float64)
    runs = []
    for kernel, persistent, graph in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 0, 1)):
        ctx = gpu_context(w, L.L2T_FP32C, graph=graph)
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
        if persistent:
            L.l2t_set_option(ctx.h, L.L2T_OPT_PERSISTENT, 1)
        L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_FIXED, fixed)
        start = ctx.get(0)
        ctx.advance(37)
        ctx.advance(64)
        runs.append(ctx.get(0))
        ctx.close()
    for r in runs[1:]:
        assert np.array_equal(runs[0], r)
    assert np.array_equal(runs[0][fixed == 1], start[fixed == 1])


def _oracle_mean_field(row, col, T, Tl, params, advances, n, gated=None, fixed=None, x=None):
    out, ck = [], []
    step = 0
    for _ in range(advances):
        c, K = oracle.mean_field(T, Tl, LAMBDA_ATOM, K_COEF)
        p = dict(params, ce_model=W.CE_CONST, ce_const=c, K=K)
        T, _, bad = oracle.run(row, col, T, Tl, p, n, step0=step, gated=gated, fixed=fixed, x=x)
        assert bad == 0
        step += n
        out.append(T.copy())
        ck.append((c, K))
    return out, ck


@pytest.mark.parametrize("precision", [L.L2T_FP64, L.L2T_FP32C])
def test_mean_field_mode_matches_oracle(precision):
    w = W.c1(n_cells=8, n_substeps=100)
    sy = w.systems[0]
    sy.params = dict(sy.params, g=5e-6)
    ctx = gpu_context(w, precision)
    L.l2t_set_mean_field(ctx.h, 0, True, LAMBDA_ATOM, K_COEF)
    row, col = oracle_neighbors(sy, w.r_cut)
    want, ck = _oracle_mean_field(row, col, sy.T_e0, sy.T_l, sy.params, 5, 100)
    for k in range(5):
        ctx.advance(100)
        assert max_rel(ctx.get(0), want[k]) < TOL[precision]
        p = L.l2t_get_params(ctx.h, 0)
        assert p["ce_model"] == L.L2T_CE_CONST
        assert p["ce_const"] == pytest.approx(ck[k][0], rel=TOL[precision])
        assert p["K"] == pytest.approx(ck[k][1], rel=1e-12)       # mean T_lat is fixed
    # switched off, the system runs on its own parameters again
    L.l2t_set_mean_field(ctx.h, 0, False)
    assert L.l2t_get_params(ctx.h, 0)["K"] == sy.params["K"]
    ctx.close()


def test_mean_field_error_paths_and_no_adjoint():
    w = W.c1(n_cells=5, n_substeps=10)
    sy = w.systems[0]
    ctx = gpu_context(w, L.L2T_FP32C)
    with pytest.raises(L.L2TError) as ex:
        L.l2t_set_mean_field(ctx.h, 0, True, 0.0, K_COEF)
    assert ex.value.status == L.L2T_EINVAL
    L.l2t_set_mean_field(ctx.h, 0, True, LAMBDA_ATOM, K_COEF)
    with pytest.raises(L.L2TError) as ex:
        L.l2t_advance_recorded(ctx.h, 10, 5)
    assert ex.value.status == L.L2T_ENOTIMPL
    # a zero mean lattice temperature cannot set K: reported, never divided by
    L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_TL, np.zeros(sy.n))
    ctx.advance(4)
    with pytest.raises(L.L2TError) as ex:
        L.l2t_sync(ctx.h)
    assert ex.value.status == L.L2T_ERANGE
    L.l2t_set_mean_field(ctx.h, 0, False)
    L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_FIXED, np.ones(sy.n))
    with pytest.raises(L.L2TError) as ex:
        L.l2t_advance_recorded(ctx.h, 10, 5)
    assert ex.value.status == L.L2T_ENOTIMPL
    ctx.close()


def test_full_size_held_shell_and_mean_field(c3_full):
    """4M atoms in the benchmark's launch configuration: a shell of held atoms
    around the hot core and the mean-field parameters refreshed at each of two
    advances of 6 sub-steps.  The oracle runs the whole system."""
    w, sy, row, col = c3_full
    r2 = ((sy.pos - (sy.box_len / 2)[:, None]) ** 2).sum(0)
    fixed = ((r2 > 60.0 ** 2) & (r2 < 64.0 ** 2)).astype(np.int32)
    ctx = gpu_context(w, L.L2T_FP32C)
    L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_FIXED, fixed.astype(np.float64))
    L.l2t_set_mean_field(ctx.h, 0, True, LAMBDA_ATOM, K_COEF)
    start = ctx.get(0)
    Tl, gated = oracle.lattice_temperature(row, col, sy.vel, sy.mass, sy.params["ke_eps"])
    want, ck = _oracle_mean_field(row, col, sy.T_e0, Tl, sy.params, 2, 6, gated=gated,
                                  fixed=fixed)
    for k in range(2):
        ctx.advance(6)
        got = ctx.get(0)
        assert max_rel(got, want[k]) < 1e-5
        assert L.l2t_get_params(ctx.h, 0)["K"] == pytest.approx(ck[k][1], rel=1e-6)
    held = fixed == 1
    assert np.array_equal(got[held], start[held])
    e = ctx.energies(0)
    assert e["sum_T"] + e["T_ledger_acc"] == pytest.approx(sy.T_e0.sum(), rel=1e-7)
    ctx.close()


def test_fp64_brick_and_global_forms_are_bitwise_equal():
    """The FP64 sub-step through LDS brick tiles and through global gathers
    on a 400,000-atom laser slab with held end cells (more bricks than CUs,
    so the brick form runs), the per-atom record on, two advances of odd
    length, per-system and batched launches, graphs on and off: states,
    records and ledgers are bitwise equal, and match the oracle."""
    sy = W.c4_slab(4.0e5, 0.2)
    sy.params = dict(sy.params, g=2e-6)
    x = sy.pos[0]
    sy.T_e0 = sy.T_e0 + np.linspace(0.0, 800.0, sy.n)
    fixed = ((x < x.min() + W.A_LAT) | (x > x.max() - W.A_LAT)).astype(np.int32)
    w = W.Workload("slab_400k_fp64", [sy], r_cut=1.1 * W.A_LAT, n_substeps=300,
                   precision="fp64")
    n1, n2 = 137, 163
    runs = []
    for kernel, batch, graph in ((1, 0, 1), (0, 0, 1), (1, 1, 1), (0, 1, 0), (1, 1, 0)):
        ctx = gpu_context(w, L.L2T_FP64)
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
        L.l2t_set_option(ctx.h, L.L2T_OPT_GRAPH, graph)
        L.l2t_set_option(ctx.h, L.L2T_OPT_BATCH_FP64, batch)
        L.l2t_set_option(ctx.h, L.L2T_OPT_ATOM_LEDGER, 1)
        L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_FIXED, fixed.astype(np.float64))
        ctx.advance(n1)
        ctx.advance(n2)
        runs.append((ctx.get(0), ctx.get(0, L.L2T_FIELD_ELAT), ctx.energies(0)))
        ctx.close()
    for T, E, en in runs[1:]:
        assert np.array_equal(T, runs[0][0])
        assert np.array_equal(E, runs[0][1])
        for k in ("E_e_to_l", "E_src", "T_ledger_acc", "sum_T"):
            assert en[k] == runs[0][2][k]
    row, col = oracle_neighbors(sy, w.r_cut)
    T, _, bad = oracle.run(row, col, sy.T_e0, sy.T_l, sy.params, n1 + n2, x=sy.pos[0],
                           fixed=fixed)
    assert bad == 0
    assert max_rel(runs[0][0], T) < 1e-12
