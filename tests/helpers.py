"""Shared drivers for the parity tests: the same seeded workload is run by the
FP64 CPU oracle and by the HIP library (through the C ABI)."""
from __future__ import annotations

import numpy as np

import oracle


def oracle_neighbors(sy, r_cut):
    return oracle.neighbors(sy.pos, sy.box_lo, sy.box_len, sy.periodic, r_cut)


def oracle_lattice(sy, row, col):
    """(T_lat, gated) as the oracle derives them for a system."""
    if sy.vel is not None:
        return oracle.lattice_temperature(row, col, sy.vel, sy.mass, sy.params["ke_eps"])
    return np.asarray(sy.T_l, dtype=np.float64), None


def oracle_trajectory(sy, r_cut, checkpoints, params=None):
    """Oracle states at the given sub-step counts, plus the ledger at the end."""
    p = sy.params if params is None else params
    row, col = oracle_neighbors(sy, r_cut)
    Tl, gated = oracle_lattice(sy, row, col)
    x = sy.pos[0] if p["laser_on"] else None
    T = np.array(sy.T_e0, dtype=np.float64)
    led = np.zeros(3)
    step = 0
    out = []
    bad_total = 0
    for c in checkpoints:
        T, led, bad = oracle.run(row, col, T, Tl, p, c - step, step0=step, gated=gated, x=x,
                                 ledger=led)
        bad_total += bad
        step = c
        out.append(T.copy())
    return out, led, bad_total


def gpu_context(workload, precision, persistent=None, block=None, graph=None, systems=None):
    from paper_1810_12357_amd import l2t as L
    ctx = L.Context(workload.systems if systems is None else systems, precision)
    ctx.setup(workload.r_cut)
    if persistent is not None:
        L.l2t_set_option(ctx.h, L.L2T_OPT_PERSISTENT, int(persistent))
    if block is not None:
        L.l2t_set_option(ctx.h, L.L2T_OPT_BLOCK, int(block))
    if graph is not None:
        L.l2t_set_option(ctx.h, L.L2T_OPT_GRAPH, int(graph))
    return ctx


def gpu_trajectory(ctx, checkpoints):
    out = []
    step = 0
    for c in checkpoints:
        ctx.advance(c - step)
        step = c
        out.append([ctx.get(s) for s in range(len(ctx.systems))])
    return out


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def light_cone(row, col, seeds, hops):
    """Atoms within `hops` neighbour hops of the seed atoms (sorted)."""
    n = row.size - 1
    mark = np.zeros(n, dtype=bool)
    mark[seeds] = True
    frontier = np.asarray(seeds, dtype=np.int64)
    for _ in range(hops):
        if frontier.size == 0:
            break
        starts = row[frontier]
        lens = row[frontier + 1] - starts
        idx = np.repeat(starts - np.cumsum(np.r_[0, lens[:-1]]), lens) + np.arange(lens.sum())
        nb = np.unique(col[idx])
        nb = nb[~mark[nb]]
        mark[nb] = True
        frontier = nb
    return np.flatnonzero(mark)


def sub_problem(row, col, keep):
    """Neighbour rows restricted to the atoms in `keep` (re-indexed)."""
    n = row.size - 1
    remap = -np.ones(n, dtype=np.int64)
    remap[keep] = np.arange(keep.size)
    starts = row[keep]
    lens = row[keep + 1] - starts
    idx = np.repeat(starts - np.cumsum(np.r_[0, lens[:-1]]), lens) + np.arange(lens.sum())
    nb = remap[col[idx]]
    owner = np.repeat(np.arange(keep.size), lens)
    ok = nb >= 0
    nb = nb[ok]
    owner = owner[ok]
    counts = np.bincount(owner, minlength=keep.size)
    r = np.zeros(keep.size + 1, dtype=np.int64)
    r[1:] = np.cumsum(counts)
    order = np.lexsort((nb, owner))
    return r, nb[order].astype(np.int32)
