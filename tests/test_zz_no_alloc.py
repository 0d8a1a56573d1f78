"""The allocation-free Eq. 4 entry point, l2t_set_velocities_noalloc, against
l2t_set_velocities: same T^lat and gate bit for bit, on two calls in a row
(the second on a smaller system, so stale staging from the first would
show), with the local and the global centre of mass, and against the oracle.
Sizes beyond the static staging array are refused."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import oracle_neighbors

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_1810_12357_amd.l2t")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision", ["fp64", "fp32c"])
def test_noalloc_lattice_temperature_equals_the_allocating_entry_point(torch, precision):
    big = W.c3(n_cells=9, n_substeps=1)        # 2,916 atoms
    small = W.c3(n_cells=6, n_substeps=1)      # 864 atoms
    systems = [big.systems[0], small.systems[0]]
    prec = L.L2T_FP64 if precision == "fp64" else L.L2T_FP32C
    ctx = L.Context(systems, prec)
    ctx.setup(big.r_cut, use_velocities=False)
    vel = [_dev(torch, sy.vel.reshape(-1)) for sy in systems]
    mass = [_dev(torch, sy.mass) for sy in systems]
    for gcom in (False, True):
        ref = []
        for s in range(2):
            L.l2t_set_velocities(ctx.h, s, vel[s], mass[s], gcom)
            ref.append((ctx.get(s, L.L2T_FIELD_TL), ctx.get(s, L.L2T_FIELD_GATE)))
        for s in range(2):                     # clear, so nothing is left over
            L.l2t_set_field(ctx.h, s, L.L2T_FIELD_TL, np.zeros(systems[s].n))
        # two calls in a row, the second on the smaller system
        for s in (0, 1):
            L.l2t_set_velocities_noalloc(ctx.h, s, vel[s], mass[s], gcom)
            Tl = ctx.get(s, L.L2T_FIELD_TL)
            gate = ctx.get(s, L.L2T_FIELD_GATE)
            assert np.array_equal(Tl, ref[s][0]), (s, gcom)
            assert np.array_equal(gate, ref[s][1]), (s, gcom)
            sy = systems[s]
            row, col = oracle_neighbors(sy, big.r_cut)
            To, go = oracle.lattice_temperature(row, col, sy.vel, sy.mass, sy.params["ke_eps"],
                                                global_com=gcom)
            tol = 1e-13 if precision == "fp64" else 6e-8
            assert np.max(np.abs(Tl - To) / To) < tol
            assert np.array_equal(gate.astype(np.int32), go)
    # the state it leaves drives the sub-steps like the allocating call's
    ctx.advance(20)
    T_a = [ctx.get(s) for s in range(2)]
    ctx.close()
    ctx = L.Context(systems, prec)
    ctx.setup(big.r_cut, use_velocities=False)
    for s in range(2):
        L.l2t_set_velocities(ctx.h, s, vel[s], mass[s], True)
    ctx.advance(20)
    for s in range(2):
        assert np.array_equal(ctx.get(s), T_a[s])
    ctx.close()


def test_noalloc_refuses_host_arrays_and_oversized_systems(torch):
    w = W.c3(n_cells=5, n_substeps=1)
    sy = w.systems[0]
    ctx = L.Context([sy], L.L2T_FP64)
    ctx.setup(w.r_cut, use_velocities=False)
    v = np.ascontiguousarray(sy.vel.reshape(-1))
    with pytest.raises(TypeError):
        L.l2t_set_velocities_noalloc(ctx.h, 0, v, sy.mass)
    ctx.close()
    # 1,048,576 atoms need 4 * 1,048,576 + 4 doubles: over 32 MiB
    n = 1 << 20
    d = L.l2t_system_desc()
    d.n_atoms = n
    for k in range(3):
        d.periodic[k] = 1
        d.box_len[k] = 400.0
    h = L.l2t_create([d], L.L2T_FP64)
    vd = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    md = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(L.L2TError) as e:
        L.l2t_set_velocities_noalloc(h, 0, vd, md)
    assert e.value.status == L.L2T_EINVAL
    L.l2t_destroy(h)
