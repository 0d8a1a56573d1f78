"""Degenerate and ragged inputs through the C ABI against the FP64 oracle:
atoms without a neighbour inside the cut-off, one batch of systems of 1, 2,
63, 64, 65 and 200 atoms beside a lattice, periodic axes only two or three
cells long, and a temperature step that puts the pair term on its top tier,
in every launch form."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_context, max_rel, oracle_neighbors

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1810_12357_amd.l2t")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _params():
    return W.default_params(g=5e-6, ce_model=W.CE_CONST, ce_const=W.C_NI)


def _grid_system(m=8, spacing=5.0, seed=21):
    """m^3 atoms on a periodic cubic grid 5 A apart: no pair within 4 A."""
    rng = np.random.default_rng(seed)
    g = (np.arange(m) + 0.5) * spacing
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).copy()
    n = pos.shape[1]
    return W.System(pos=pos, box_lo=np.zeros(3), box_len=np.full(3, m * spacing),
                    periodic=np.ones(3, np.int32), T_e0=300.0 + 3000.0 * rng.uniform(0, 1, n),
                    params=_params(), T_l=300.0 + 200.0 * rng.uniform(0, 1, n))


def _gas(n, box, seed):
    """n atoms uniform in a free (non-periodic) box."""
    rng = np.random.default_rng(seed)
    return W.System(pos=rng.uniform(0.05, box - 0.05, (3, n)), box_lo=np.zeros(3),
                    box_len=np.full(3, box), periodic=np.zeros(3, np.int32),
                    T_e0=300.0 + 2500.0 * rng.uniform(0, 1, n), params=_params(),
                    T_l=300.0 + 100.0 * rng.uniform(0, 1, n))


@pytest.mark.parametrize("precision", [L.L2T_FP64, L.L2T_FP32C])
def test_atoms_without_neighbours_relax_by_the_closed_form(precision):
    """With no neighbour inside the cut-off only the coupling acts:
    T_n - T_l = (T_0 - T_l) (1 - dt g / c)^n, and the energy handed to the
    lattice is c (sum T_0 - sum T_n)."""
    sy = _grid_system()
    w = W.Workload("grid", [sy], 4.0, 400, "fp64")
    ctx = gpu_context(w, precision)
    n = 400
    ctx.advance(n)
    p = sy.params
    want = sy.T_l + (sy.T_e0 - sy.T_l) * (1.0 - p["dt"] * p["g"] / p["ce_const"]) ** n
    got = ctx.get(0)
    assert max_rel(got, want) < (1e-12 if precision == L.L2T_FP64 else 1e-5)
    row, col = oracle_neighbors(sy, w.r_cut)
    assert row[-1] == 0
    T, led, _ = oracle.run(row, col, sy.T_e0, sy.T_l, p, n)
    assert max_rel(got, T) < (1e-12 if precision == L.L2T_FP64 else 1e-5)
    e = ctx.energies(0)
    ref = p["ce_const"] * (sy.T_e0.sum() - T.sum())
    assert e["E_e_to_l"] == pytest.approx(ref, rel=1e-9 if precision == L.L2T_FP64 else 1e-5)
    ctx.close()


def _ragged():
    systems = [_gas(n, box, 30 + k) for k, (n, box) in
               enumerate([(1, 9.0), (2, 5.0), (63, 12.0), (64, 12.0), (65, 12.0), (200, 20.0)])]
    systems.append(W.c1(n_cells=4).systems[0])
    return W.Workload("ragged", systems, 4.0, 300, "fp32c")


def _oracle_states(w, n):
    out = []
    for sy in w.systems:
        row, col = oracle_neighbors(sy, w.r_cut)
        T, _, bad = oracle.run(row, col, sy.T_e0, sy.T_l, sy.params, n)
        assert bad == 0
        out.append(T)
    return out


def test_ragged_batch_fp32c_every_launch_form():
    w = _ragged()
    n = 300
    want = _oracle_states(w, n)
    runs = []
    for kernel, persistent, graph in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 0, 1)):
        ctx = gpu_context(w, L.L2T_FP32C, graph=graph)
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
        if persistent:
            L.l2t_set_option(ctx.h, L.L2T_OPT_PERSISTENT, 1)
        ctx.advance(137)
        ctx.advance(n - 137)
        runs.append([ctx.get(s) for s in range(len(w.systems))])
        ctx.close()
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)
    for got, T in zip(runs[0], want):
        assert max_rel(got, T) < 1e-5


def test_ragged_batch_fp64_resident_and_per_substep():
    w = _ragged()
    n = 300
    want = _oracle_states(w, n)
    runs = []
    for batch, res in ((0, 0), (1, -1), (1, 0)):
        ctx = gpu_context(w, L.L2T_FP64)
        L.l2t_set_option(ctx.h, L.L2T_OPT_BATCH_FP64, batch)
        L.l2t_set_option(ctx.h, L.L2T_OPT_RESIDENT_MAX, res)
        ctx.advance(137)
        ctx.advance(n - 137)
        runs.append([ctx.get(s) for s in range(len(w.systems))])
        ctx.close()
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)
    for got, T in zip(runs[0], want):
        assert max_rel(got, T) < 1e-12


@pytest.mark.parametrize("precision", [L.L2T_FP64, L.L2T_FP32C])
def test_uniform_temperature_is_stationary_and_g0_conserves(precision):
    """T_e = T_lat uniform: every pair term and the coupling are exactly zero,
    so the state does not move at all.  With G = 0 and constant c the
    antisymmetric exchange keeps sum T (the ledger records no energy to the
    lattice)."""
    w = W.c1(n_cells=6, n_substeps=500)
    sy = w.systems[0]
    sy.params = dict(sy.params, ce_model=W.CE_CONST, ce_const=W.C_NI)
    flat = W.System(pos=sy.pos, box_lo=sy.box_lo, box_len=sy.box_len, periodic=sy.periodic,
                    T_e0=np.full(sy.n, 1234.5), params=sy.params, T_l=np.full(sy.n, 1234.5))
    ctx = gpu_context(W.Workload("flat", [flat], w.r_cut, 500, "fp64"), precision)
    ctx.advance(500)
    assert np.array_equal(ctx.get(0), flat.T_e0)
    ctx.close()
    hot = W.System(pos=sy.pos, box_lo=sy.box_lo, box_len=sy.box_len, periodic=sy.periodic,
                   T_e0=sy.T_e0, params=dict(sy.params, g=0.0), T_l=sy.T_l)
    ctx = gpu_context(W.Workload("g0", [hot], w.r_cut, 500, "fp64"), precision)
    ctx.advance(500)
    T = ctx.get(0)
    assert np.max(np.abs(T - hot.T_e0)) > 100.0             # the hotspot did spread
    assert T.sum() == pytest.approx(hot.T_e0.sum(), rel=1e-13 if precision == L.L2T_FP64 else 1e-9)
    assert ctx.energies(0)["E_e_to_l"] == 0.0
    ctx.close()


def test_measured_brick_edge_near_the_model_cached_and_exact():
    """A layout with more bricks than CUs (64 systems of 32,000 atoms): the
    build measures the model's brick edge against its neighbours and keeps
    one of the three, and times the sweep order and the table-load policy; a
    second build of the same shape reuses all three choices; both layouts
    give the oracle's trajectory on a sampled system.  Without the autotuner
    the build keeps the fixed order and cached table loads."""
    w = W.c5(n_substeps=40)
    ctx_m = L.Context(w.systems, L.L2T_FP32C)
    L.l2t_set_option(ctx_m.h, L.L2T_OPT_AUTOTUNE, 0)     # the model's edge only
    ctx_m.setup(w.r_cut)
    e_m = L.l2t_get_option(ctx_m.h, L.L2T_OPT_BRICK_EDGE)
    assert L.l2t_get_option(ctx_m.h, L.L2T_OPT_SWEEP) == 1
    assert L.l2t_get_option(ctx_m.h, L.L2T_OPT_TABLE_STREAM) == 1
    ctx_t = L.Context(w.systems, L.L2T_FP32C)
    ctx_t.setup(w.r_cut)
    e_t = L.l2t_get_option(ctx_t.h, L.L2T_OPT_BRICK_EDGE)
    assert abs(e_t - e_m) <= 1
    choice = [L.l2t_get_option(ctx_t.h, o) for o in (L.L2T_OPT_SWEEP, L.L2T_OPT_TABLE_STREAM)]
    assert all(v in (1, 2) for v in choice)
    ctx_2 = L.Context(w.systems, L.L2T_FP32C)
    ctx_2.setup(w.r_cut)
    assert L.l2t_get_option(ctx_2.h, L.L2T_OPT_BRICK_EDGE) == e_t
    assert [L.l2t_get_option(ctx_2.h, o)
            for o in (L.L2T_OPT_SWEEP, L.L2T_OPT_TABLE_STREAM)] == choice
    ctx_2.close()
    sy = w.systems[5]
    row, col = oracle_neighbors(sy, w.r_cut)
    ref, _, _ = oracle.run(row, col, sy.T_e0, sy.T_l, sy.params, w.n_substeps)
    for ctx in (ctx_m, ctx_t):
        ctx.advance(w.n_substeps)
        assert max_rel(ctx.get(5), ref) < 1e-5
        ctx.close()


def test_graph_or_direct_launches_timed_cached_and_bitwise_equal():
    """The FP32C autotuner times the tuned shape's probe as direct launches
    and as a graph replay and keeps the faster (L2T_OPT_GRAPH = 2, the
    default): the choice reads back as 0 or 1, a second context of the same
    shape reuses it, and default, direct and graph-replayed advances give the
    same states bit for bit.  Without the autotuner the advance replays
    graphs; values outside 0..2 are refused."""
    w = W.c5(n_substeps=37)
    states, choice = [], []
    for graph in (None, None, 0, 1):
        ctx = gpu_context(w, L.L2T_FP32C, graph=graph)
        ctx.advance(w.n_substeps)
        choice.append(L.l2t_get_option(ctx.h, L.L2T_OPT_GRAPH))
        states.append(np.concatenate([ctx.get(s) for s in (0, 31, 63)]))
        ctx.close()
    assert choice[0] in (0, 1) and choice[1] == choice[0] and choice[2:] == [0, 1]
    for st in states[1:]:
        assert np.array_equal(st, states[0])
    ctx = L.Context(w.systems, L.L2T_FP32C)
    L.l2t_set_option(ctx.h, L.L2T_OPT_AUTOTUNE, 0)
    ctx.setup(w.r_cut)
    ctx.advance(3)
    assert L.l2t_get_option(ctx.h, L.L2T_OPT_GRAPH) == 1
    with pytest.raises(L.L2TError):
        L.l2t_set_option(ctx.h, L.L2T_OPT_GRAPH, 3)
    ctx.close()


def test_autotune_cache_file_records_the_timed_choice(tmp_path, monkeypatch):
    """With L2T_AUTOTUNE_CACHE set, the first tuning of a problem shape
    appends one line for it: the shape key, then kernel, persistent, block
    and the timed graph choice; the context uses what the line records."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("L2T_AUTOTUNE_CACHE", str(path))
    sy = _grid_system(m=9, spacing=2.9, seed=44)   # a shape no other test tunes
    w = W.Workload("grid9", [sy], 4.4, 10, "fp32c")
    ctx = gpu_context(w, L.L2T_FP32C)
    ctx.advance(10)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    key, vals = lines[0].split("|")
    assert key.startswith("n_int=") and " sys=1 " in key
    k, pers, block, graph = (int(v) for v in vals.split())
    assert k == L.l2t_get_option(ctx.h, L.L2T_OPT_KERNEL)
    assert pers == 0 and block == L.l2t_get_option(ctx.h, L.L2T_OPT_BLOCK)
    assert graph == L.l2t_get_option(ctx.h, L.L2T_OPT_GRAPH) and graph in (0, 1)
    ctx.close()


def _step_system(n_cells=10, hot=19000.0, cold=300.0, seed=31):
    """FCC n^3 cells, periodic, jittered 0.05 A: T_e = hot where x < L/2 and
    cold beyond, so neighbours across the two planes of the step differ by up
    to 18,700 K and their pair terms run on the top tier of the FP32 form."""
    pos, box = W.fcc(n_cells, n_cells, n_cells)
    per = np.ones(3, np.int32)
    pos = W.wrap_periodic(W.jitter(pos, 0.05, seed), np.zeros(3), box, per)
    n = pos.shape[1]
    p = W.default_params(ce_model=W.CE_LINEAR, gamma=1e-4)
    return W.System(pos=pos, box_lo=np.zeros(3), box_len=box, periodic=per,
                    T_e0=np.where(pos[0] < box[0] / 2.0, hot, cold), params=p,
                    T_l=np.full(n, 300.0))


def test_steep_step_on_the_top_tier_in_every_launch_form():
    """A temperature step of 18,700 K, compared after 7, 37 and 400 sub-steps
    (the top tier carries the exchange through the first ~40): every FP32C
    launch form (global gathers, persistent, LDS bricks with and without
    graphs) gives the same states bit for bit and matches the oracle to
    1e-5; FP64 to 1e-12."""
    sy = _step_system()
    w = W.Workload("step", [sy], 1.1 * W.A_LAT, 400, "fp32c")
    p = sy.params
    row, col = oracle_neighbors(sy, w.r_cut)
    own = np.repeat(np.arange(sy.n), np.diff(row))
    u = ((sy.T_e0[col] - sy.T_e0[own]) / (p["T_max"] - p["T_min"])) ** 2
    assert u.max() > 0.8 and np.count_nonzero(u > 1e-2) > 1000   # the top tier is reached
    checkpoints = (7, 37, 400)
    want, T, step = [], sy.T_e0, 0
    for c in checkpoints:
        T, _, bad = oracle.run(row, col, T, sy.T_l, p, c - step)
        assert bad == 0
        want.append(T)
        step = c

    def states(ctx):
        out, step = [], 0
        for c in checkpoints:
            ctx.advance(c - step)
            step = c
            out.append(ctx.get(0))
        ctx.close()
        return out

    runs = []
    for kernel, persistent, graph in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 0, 1)):
        ctx = gpu_context(w, L.L2T_FP32C, graph=graph)
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
        if persistent:
            L.l2t_set_option(ctx.h, L.L2T_OPT_PERSISTENT, 1)
        runs.append(states(ctx))
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            assert np.array_equal(a, b)
    f64 = states(gpu_context(w, L.L2T_FP64))
    for c, got, got64, T in zip(checkpoints, runs[0], f64, want):
        err, err64 = max_rel(got, T), max_rel(got64, T)
        print(f"step of 18,700 K after {c} sub-steps: FP32C {err:.2e}, FP64 {err64:.2e}")
        assert err < 1e-5 and err64 < 1e-12


def _short_box(cells, seed):
    """Atoms uniform at the density of FCC nickel in a box whose periodic x
    and y axes are only `cells` cells long (the cell stencil and a brick's
    shell wrap onto themselves) and whose z axis is free and 20 cells long.
    The exchange rate is lowered to 0.2 / fs: random placement gives up to
    ~40 neighbours, and forward Euler stays stable for K dt (2 n_max) < 2."""
    rc = 1.1 * W.A_LAT
    rng = np.random.default_rng(seed)
    box = np.array([cells * rc * 1.02, cells * rc * 1.02, 20.0 * rc])
    n = int(4.0 / W.A_LAT ** 3 * np.prod(box))
    p = W.default_params(g=5e-6, ce_model=W.CE_CONST, ce_const=W.C_NI, K=0.2)
    return W.System(pos=rng.uniform(0.0, 1.0, (3, n)) * box[:, None], box_lo=np.zeros(3),
                    box_len=box, periodic=np.array([1, 1, 0], np.int32),
                    T_e0=300.0 + 4000.0 * rng.uniform(0, 1, n), params=p,
                    T_l=300.0 + 100.0 * rng.uniform(0, 1, n))


def test_periodic_axes_of_two_and_three_cells_every_launch_form():
    """Neighbour sets equal the oracle's where a periodic axis is only two or
    three cells long; after 7, 137 and 300 sub-steps the states of every
    FP32C launch form are bitwise equal and match the oracle (1e-5), FP64 to
    1e-12."""
    systems = [_short_box(2, 52), _short_box(3, 53)]
    rc = 1.1 * W.A_LAT
    w = W.Workload("short", systems, rc, 300, "fp32c")
    checkpoints = (7, 137, 300)
    want = []
    for sy in systems:
        row, col = oracle_neighbors(sy, rc)
        T, step, states = sy.T_e0, 0, []
        for c in checkpoints:
            T, _, bad = oracle.run(row, col, T, sy.T_l, sy.params, c - step)
            assert bad == 0
            states.append(T)
            step = c
        want.append(states)

    def states(ctx):
        out, step = [], 0
        for c in checkpoints:
            ctx.advance(c - step)
            step = c
            out.append([ctx.get(s) for s in range(len(systems))])
        ctx.close()
        return out

    runs = []
    for kernel, persistent, graph in ((0, 0, 0), (0, 1, 0), (1, 0, 0), (1, 0, 1)):
        ctx = gpu_context(w, L.L2T_FP32C, graph=graph)
        if not runs:
            for s, sy in enumerate(systems):
                r, c = L.l2t_get_neighbors(ctx.h, s, sy.n)
                r0, c0 = oracle_neighbors(sy, rc)
                assert np.array_equal(r, r0) and np.array_equal(c, c0)
        L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
        if persistent:
            L.l2t_set_option(ctx.h, L.L2T_OPT_PERSISTENT, 1)
        runs.append(states(ctx))
    for r in runs[1:]:
        for a, b in zip(runs[0], r):
            for x, y in zip(a, b):
                assert np.array_equal(x, y)
    f64 = states(gpu_context(w, L.L2T_FP64))
    for k, c in enumerate(checkpoints):
        for s in range(len(systems)):
            err = max_rel(runs[0][k][s], want[s][k])
            err64 = max_rel(f64[k][s], want[s][k])
            print(f"{['two', 'three'][s]} cells, {c} sub-steps: FP32C {err:.2e}, FP64 {err64:.2e}")
            assert err < 1e-5 and err64 < 1e-12
