"""GPU adjoint (reverse sub-step kernel with checkpointed recomputation)
against the FP64 oracle adjoint, and through torch.autograd."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import oracle_lattice, oracle_neighbors

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1810_12357_amd.l2t")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _targets(sy, r_cut, n, K, g):
    """Target T^N from the oracle with perturbed parameters."""
    row, col = oracle_neighbors(sy, r_cut)
    Tl, gated = oracle_lattice(sy, row, col)
    T, _, _ = oracle.run(row, col, sy.T_e0, Tl, dict(sy.params, K=K, g=g), n, gated=gated)
    return T


def _oracle_grad(sy, r_cut, n, w, params=None):
    row, col = oracle_neighbors(sy, r_cut)
    Tl, gated = oracle_lattice(sy, row, col)
    p = sy.params if params is None else params
    x = sy.pos[0] if p["laser_on"] else None
    return oracle.adjoint(row, col, sy.T_e0, Tl, p, n, w, gated=gated, x=x)


@pytest.mark.parametrize("ckpt", [1, 7, 50, 1000])
def test_adjoint_matches_oracle_reduced_c5(ckpt):
    """Checkpoints every 7 (a ragged last segment) and every 50 sub-steps, and
    the two degenerate schedules: every state stored (segments of one reverse
    sub-step, nothing recomputed) and one checkpoint longer than the run (the
    whole forward recomputed in one segment)."""
    w = W.c5(n_systems=3, n_cells=7, n_substeps=300)
    n = w.n_substeps
    ctx = L.Context(w.systems, L.L2T_FP32C)
    ctx.setup(w.r_cut)
    L.l2t_advance_recorded(ctx.h, n, ckpt)
    TN = [ctx.get(s) for s in range(3)]
    tgt = [_targets(sy, w.r_cut, n, *w.extra["target_params"][s]) for s, sy in enumerate(w.systems)]
    N = sum(sy.n for sy in w.systems)
    dL = np.concatenate([2.0 * (TN[s] - tgt[s]) / N for s in range(3)])
    dT0 = np.zeros(N)
    dK, dg = L.l2t_adjoint(ctx.h, dL, 3, dL_dT0=dT0)
    off = 0
    for s, sy in enumerate(w.systems):
        lam, oK, og = _oracle_grad(sy, w.r_cut, n, dL[off:off + sy.n])
        assert dK[s] == pytest.approx(oK, rel=1e-4)
        assert dg[s] == pytest.approx(og, rel=1e-4)
        scale = np.abs(lam).max()
        assert np.max(np.abs(dT0[off:off + sy.n] - lam)) < 1e-4 * scale
        off += sy.n
    # recorded forward equals a plain forward
    ctx2 = L.Context(w.systems, L.L2T_FP32C)
    ctx2.setup(w.r_cut)
    L.l2t_set_option(ctx2.h, L.L2T_OPT_PERSISTENT, 1)
    ctx2.advance(n)
    for s in range(3):
        assert np.array_equal(ctx2.get(s), TN[s])


def test_adjoint_linear_c_laser_gate():
    """Every local term: linear heat capacity, laser source, gated atoms."""
    s4 = W.c4_slab(1500, 0.4)
    s4.params = dict(s4.params, laser_t0=20.0, laser_sigma=8.0, g=5e-6)
    rng = np.random.default_rng(2)
    s4.T_l = 300.0 + 200 * rng.uniform(0, 1, s4.n)
    w = W.Workload("slab", [s4], 1.1 * W.A_LAT, 400, "fp32c")
    ctx = L.Context(w.systems, L.L2T_FP32C)
    ctx.setup(w.r_cut)
    gate = (rng.uniform(0, 1, s4.n) < 0.1).astype(np.float64)
    L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_GATE, gate)
    L.l2t_advance_recorded(ctx.h, 400, 64)
    wv = rng.normal(size=s4.n) * 1e-3
    dT0 = np.zeros(s4.n)
    dK, dg = L.l2t_adjoint(ctx.h, wv, 1, dL_dT0=dT0)
    row, col = oracle_neighbors(s4, w.r_cut)
    lam, oK, og = oracle.adjoint(row, col, s4.T_e0, s4.T_l, s4.params, 400, wv,
                                 gated=gate.astype(np.int32), x=s4.pos[0])
    assert dK[0] == pytest.approx(oK, rel=1e-4)
    assert dg[0] == pytest.approx(og, rel=1e-4)
    assert np.max(np.abs(dT0 - lam)) < 1e-4 * np.abs(lam).max()


def test_autograd_function_gradients():
    import torch
    from paper_1810_12357_amd import autograd as A
    w = W.c5(n_systems=2, n_cells=6, n_substeps=200)
    ctx = L.Context(w.systems, L.L2T_FP32C)
    ctx.setup(w.r_cut)
    T0 = torch.from_numpy(np.concatenate([sy.T_e0 for sy in w.systems])).cuda()
    K = torch.tensor([W.C5_K0, W.C5_K0 * 1.1], dtype=torch.float64, device="cuda",
                     requires_grad=True)
    g = torch.tensor([W.C5_G0, W.C5_G0 * 0.9], dtype=torch.float64, device="cuda",
                     requires_grad=True)
    T0.requires_grad_(True)
    TN = A.advance(T0, K, g, ctx, 200, 50)
    tgt = torch.full_like(TN, 500.0)
    loss = ((TN - tgt) ** 2).mean()
    loss.backward()
    # finite differences of the same GPU forward in K for system 0
    def f(Kv):
        with torch.no_grad():
            out = A.advance(T0.detach(), torch.tensor([Kv, K[1].item()], dtype=torch.float64,
                                                      device="cuda"), g.detach(), ctx, 200, 50)
            return float(((out - tgt) ** 2).mean())
    eps = 1e-3 * W.C5_K0
    fd = (f(W.C5_K0 + eps) - f(W.C5_K0 - eps)) / (2 * eps)
    assert K.grad[0].item() == pytest.approx(fd, rel=2e-3)
    # and the oracle's adjoint for system 0
    sy = w.systems[0]
    n0 = sy.n
    wv = (2.0 * (TN.detach() - tgt) / TN.numel()).cpu().numpy()[:n0]
    lam, oK, og = _oracle_grad(sy, w.r_cut, 200, wv, dict(sy.params, K=W.C5_K0, g=W.C5_G0))
    assert K.grad[0].item() == pytest.approx(oK, rel=1e-4)
    assert g.grad[0].item() == pytest.approx(og, rel=1e-4)
    assert np.max(np.abs(T0.grad.cpu().numpy()[:n0] - lam)) < 1e-4 * np.abs(lam).max()
    # a later recorded forward replaces the recording: the earlier graph refuses backward
    T1 = A.advance(T0, K, g, ctx, 50, 25)
    T2 = A.advance(T0, K, g, ctx, 50, 25)
    with pytest.raises(RuntimeError):
        T1.sum().backward()
    T2.sum().backward()


def _adjoint_run(w, kernel, dL_fn, gate=None, graph=1):
    ctx = L.Context(w.systems, L.L2T_FP32C)
    ctx.setup(w.r_cut)
    L.l2t_set_option(ctx.h, L.L2T_OPT_KERNEL, kernel)
    L.l2t_set_option(ctx.h, L.L2T_OPT_GRAPH, graph)
    if gate is not None:
        L.l2t_set_field(ctx.h, 0, L.L2T_FIELD_GATE, gate)
    L.l2t_advance_recorded(ctx.h, w.n_substeps, w.checkpoint_every)
    TN = np.concatenate([ctx.get(s) for s in range(len(w.systems))])
    dL = dL_fn(TN)
    dT0 = np.zeros(TN.size)
    dK, dg = L.l2t_adjoint(ctx.h, dL, len(w.systems), dL_dT0=dT0)
    return ctx, TN, dT0, dK, dg


@pytest.mark.parametrize("case", ["c5", "laser_slab"])
def test_adjoint_brick_and_global_forms_agree(case):
    """The LDS-brick reverse step (with the brick recomputation) and the
    global-gather one evaluate the same per-atom terms in the same order:
    lambda is bitwise equal; the gradient sums differ only in grouping.  The
    segments replayed from captured graphs equal the directly launched ones."""
    gate = None
    if case == "c5":
        w = W.c5(n_systems=3, n_cells=7, n_substeps=300)
        w.checkpoint_every = 50
    else:
        s4 = W.c4_slab(1500, 0.4)
        s4.params = dict(s4.params, laser_t0=20.0, laser_sigma=8.0, g=5e-6)
        rng = np.random.default_rng(2)
        s4.T_l = 300.0 + 200 * rng.uniform(0, 1, s4.n)
        gate = (rng.uniform(0, 1, s4.n) < 0.1).astype(np.float64)
        w = W.Workload("slab", [s4], 1.1 * W.A_LAT, 400, "fp32c", checkpoint_every=64)
    rng = np.random.default_rng(7)
    wv = rng.normal(size=w.n_atoms) * 1e-3
    runs = [_adjoint_run(w, k, lambda TN: wv, gate, graph) for k, graph in ((0, 1), (1, 1), (1, 0))]
    for r in runs:
        r[0].close()
    (_, TN0, l0, K0, g0), (_, TN1, l1, K1, g1), (_, TN2, l2, K2, g2) = runs
    assert np.array_equal(TN1, TN2) and np.array_equal(l1, l2)
    assert np.array_equal(K1, K2) and np.array_equal(g1, g2)
    assert np.array_equal(TN0, TN1)
    assert np.array_equal(l0, l1)
    np.testing.assert_allclose(K1, K0, rtol=1e-12)
    np.testing.assert_allclose(g1, g0, rtol=1e-12)


def test_full_size_c5_adjoint_forms_and_finite_difference():
    """64 systems of 32,000 atoms, 2,000 sub-steps, a checkpoint every 100 (the
    benchmark's differentiation workload): both launch forms give the same
    lambda, and dL/dK of system 0 matches a central difference of the GPU
    forward."""
    w = W.c5()
    n = w.n_substeps
    tw = W.c5()
    for s, sy in enumerate(tw.systems):
        K, g = tw.extra["target_params"][s]
        sy.params = dict(sy.params, K=K, g=g)
    ct = L.Context(tw.systems, L.L2T_FP32C)
    ct.setup(tw.r_cut)
    ct.advance(n)
    tgt = np.concatenate([ct.get(s) for s in range(len(tw.systems))])
    ct.close()
    N = w.n_atoms
    loss = lambda TN: float(np.mean((TN - tgt) ** 2))
    dL_fn = lambda TN: 2.0 * (TN - tgt) / N
    ctx1, TN1, l1, K1, g1 = _adjoint_run(w, 1, dL_fn)
    ctx0, TN0, l0, K0, g0 = _adjoint_run(w, 0, dL_fn)
    ctx0.close()
    assert np.array_equal(TN0, TN1)
    assert np.array_equal(l0, l1)
    np.testing.assert_allclose(K1, K0, rtol=1e-12)
    np.testing.assert_allclose(g1, g0, rtol=1e-12)
    sy0 = w.systems[0]
    eps = 1e-3 * sy0.params["K"]

    def run_K(Kv):
        L.l2t_set_params(ctx1.h, 0, dict(sy0.params, K=Kv))
        for s, sy in enumerate(w.systems):
            L.l2t_set_field(ctx1.h, s, L.L2T_FIELD_TE, sy.T_e0)
        ctx1.advance(n)
        return loss(np.concatenate([ctx1.get(s) for s in range(len(w.systems))]))

    fd = (run_K(sy0.params["K"] + eps) - run_K(sy0.params["K"] - eps)) / (2 * eps)
    assert K1[0] == pytest.approx(fd, rel=2e-3)
    ctx1.close()
