// Geometry kernels: cell binning, the brick-ordered internal layout, neighbour
// sets in wavefront-sliced column-major tables (global int32 indices and
// brick-local uint16 indices with per-brick halo lists), per-atom field
// permutation, the local lattice temperature (Eq. 4) with the kinetic-energy
// gate, and the per-atom depth weights of the laser source (Eq. 10).
//
// Internal order of one system: cells are grouped into bricks of up to
// b x b x b cells; bricks in x-major order, cells inside a brick z-fastest,
// atoms inside a cell by caller index.  Every brick owns a slot range padded
// to a multiple of 64, so no 64-lane slice straddles two bricks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <thread>
#include <vector>

#include "l2t_internal.h"
#include "state_fp32c.h"

namespace l2t {
namespace {

struct Grid {
    int32_t nc[3];
    int32_t periodic[3];
    double lo[3], len[3];
};

__device__ inline double wrap_coord(double x, double lo, double len, int32_t periodic) {
    double s = x - lo;
    if (periodic) s -= len * floor(s / len);
    return s;
}

__device__ inline int32_t cell_coord(double s, double len, int32_t nc) {
    int32_t k = (int32_t)floor(s / len * (double)nc);
    return k < 0 ? 0 : (k >= nc ? nc - 1 : k);
}

// distinct cell coordinates c-1, c, c+1 along one axis (wrapped or clipped),
// with the offset that first produced each
__device__ inline int axis_cells(int32_t c, int32_t nc, int32_t periodic, int32_t out[3],
                                 int32_t off[3]) {
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int32_t k = c + o;
        if (periodic) {
            k = (k % nc + nc) % nc;
        } else if (k < 0 || k >= nc) {
            continue;
        }
        bool dup = false;
        for (int q = 0; q < m; ++q) dup |= (out[q] == k);
        if (!dup) {
            off[m] = o;
            out[m++] = k;
        }
    }
    return m;
}

// Positions on a periodic axis lie in [lo, lo + len), so |d| < len and the
// nearest image is at most one box length away: the shift of
// d - len * rint(d / len) without its division, equal to it except where d is
// within an ulp of half a box length (a tie of measure zero).
__device__ inline double min_image(double d, double len, int32_t periodic) {
    if (!periodic) return d;
    const double h = 0.5 * len;
    return d > h ? d - len : (d < -h ? d + len : d);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Rank maps of one system's cells.  Bricks are ordered X, Y, Z and the cells
// inside a brick x, y, z; a brick's extents are clipped at the grid's end, and
// bc0 holds the first rank of every brick.
__global__ void k_rank_maps(int64_t ncell, int32_t nc1, int32_t nc2, int32_t b0, int32_t b1,
                            int32_t b2, int32_t nb1, int32_t nb2, const int32_t *bc0,
                            int32_t brick0, int32_t *rank_of_cell, int32_t *cell_of_rank,
                            int32_t *brick_of_rank) {
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ncell) return;
    const int32_t x = (int32_t)(cell / ((int64_t)nc1 * nc2));
    const int32_t y = (int32_t)((cell / nc2) % nc1), z = (int32_t)(cell % nc2);
    const int32_t X = x / b0, Y = y / b1, Z = z / b2;
    const int32_t e1 = min(b1, nc1 - Y * b1), e2 = min(b2, nc2 - Z * b2);
    const int32_t bidx = (X * nb1 + Y) * nb2 + Z;
    const int32_t r = bc0[bidx] + ((x - X * b0) * e1 + (y - Y * b1)) * e2 + (z - Z * b2);
    rank_of_cell[cell] = r;
    cell_of_rank[r] = (int32_t)cell;
    brick_of_rank[r] = brick0 + bidx;
}

// bin the atoms of one system (caller order); cell_of receives the cell's
// rank in brick order
__global__ void k_bin(const double *px, const double *py, const double *pz, int32_t n, Grid g,
                      const int32_t *rank_of_cell, int32_t *cell_of, int32_t *count,
                      unsigned *err) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double p[3] = {px[i], py[i], pz[i]};
    int32_t ic[3];
    for (int d = 0; d < 3; ++d) {
        double s = wrap_coord(p[d], g.lo[d], g.len[d], g.periodic[d]);
        if (!g.periodic[d] && !(s >= 0.0 && s <= g.len[d])) atomicOr(err, kErrBox);
        ic[d] = cell_coord(s, g.len[d], g.nc[d]);
    }
    const int32_t r = rank_of_cell[(ic[0] * g.nc[1] + ic[1]) * g.nc[2] + ic[2]];
    cell_of[i] = r;
    atomicAdd(&count[r], 1);
}

// exclusive prefix sum of n int32 values with out[n] = total; one workgroup,
// fixed chunking, so the result is deterministic
__global__ void k_scan_excl(const int32_t *in, int32_t *out, int64_t n) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x, T = blockDim.x;
    int64_t chunk = (n + T - 1) / T;
    int64_t b = (int64_t)t * chunk, e = b + chunk < n ? b + chunk : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t acc = 0;
        for (int k = 0; k < T; ++k) {
            int64_t v = part[k];
            part[k] = acc;
            acc += v;
        }
        out[n] = (int32_t)acc;
    }
    __syncthreads();
    int64_t acc = part[t];
    for (int64_t i = b; i < e; ++i) {
        int32_t v = in[i];
        out[i] = (int32_t)acc;
        acc += v;
    }
}

// Multi-block exclusive scan of the cell counts: tile sums, a scan of the tile
// sums (k_scan_excl on the short array), then each tile's local scan.
constexpr int kScanPer = 8, kScanThreads = 256, kScanTile = kScanPer * kScanThreads;

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const int32_t *in, int64_t n,
                                                            int32_t *bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t s = 0;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (base + k < n) s += in[base + k];
    __shared__ int32_t sh[kScanThreads];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kScanThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kScanThreads) void k_tile_scan(const int32_t *in, int64_t n,
                                                            const int32_t *boff, int32_t *out) {
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
    int32_t v[kScanPer], s = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        v[u] = base + u < n ? in[base + u] : 0;
        s += v[u];
    }
    __shared__ int32_t sh[kScanThreads];
    sh[t] = s;
    __syncthreads();
    for (int w = 1; w < kScanThreads; w <<= 1) {   // inclusive scan of the thread sums
        const int32_t add = t >= w ? sh[t - w] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int32_t acc = boff[blockIdx.x] + sh[t] - s;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        if (base + u < n) out[base + u] = acc;
        acc += v[u];
    }
    if (blockIdx.x == 0 && t == 0) out[n] = boff[gridDim.x];
}

__global__ void k_scatter(const int32_t *cell_of, int32_t n, const int32_t *start, int32_t *fill,
                          int32_t *sorted) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t c = cell_of[i];
    int32_t pos = start[c] + atomicAdd(&fill[c], 1);
    sorted[pos] = i;
}

// order the atoms inside every cell by caller index (makes the order
// independent of the atomic scatter)
__global__ void k_sort_cells(const int32_t *start, int64_t ncell, int32_t *sorted) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int32_t b = start[c], e = start[c + 1];
    for (int32_t i = b + 1; i < e; ++i) {
        int32_t v = sorted[i];
        int32_t j = i - 1;
        while (j >= b && sorted[j] > v) {
            sorted[j + 1] = sorted[j];
            --j;
        }
        sorted[j + 1] = v;
    }
}

// padding slots of one system: no atom
__global__ void k_init_slots(int32_t atom_off, int32_t n_pad, int32_t *perm, int32_t *cell_int,
                             double *qx, double *qy, double *qz, int32_t *cnt) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    const int32_t s = atom_off + k;
    perm[s] = -1;
    cell_int[s] = -1;
    cnt[s] = 0;
    qx[s] = qy[s] = qz[s] = 0.0;
}

// final slot of the atom at cell-order position k: its brick's first slot
// plus its offset inside the brick.  The wrapped position is written by slot
// (qx, qy, qz) and by cell order (sx, sy, sz: what the neighbour search reads)
__global__ void k_assign(const int32_t *sorted, int32_t n, int32_t atom_off, int64_t caller_off,
                         const double *px, const double *py, const double *pz,
                         const int32_t *cell_of, const int32_t *brick_of_rank,
                         const BrickInfo *bricks, const int32_t *brick_atom0, Grid g,
                         int32_t *perm, int32_t *inv, int32_t *cell_int, int32_t *pos_slot,
                         double *qx, double *qy, double *qz, double *sx, double *sy, double *sz) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t i = sorted[k];
    const int32_t r = cell_of[i];
    const int32_t b = brick_of_rank[r];
    const int32_t slot = bricks[b].slot0 + (k - brick_atom0[b]);
    perm[slot] = (int32_t)(caller_off + i);
    inv[caller_off + i] = slot;
    cell_int[slot] = r;
    pos_slot[k] = slot;
    const double x = g.lo[0] + wrap_coord(px[i], g.lo[0], g.len[0], g.periodic[0]);
    const double y = g.lo[1] + wrap_coord(py[i], g.lo[1], g.len[1], g.periodic[1]);
    const double z = g.lo[2] + wrap_coord(pz[i], g.lo[2], g.len[2], g.periodic[2]);
    qx[slot] = x;
    qy[slot] = y;
    qz[slot] = z;
    sx[k] = x;
    sy[k] = y;
    sz[k] = z;
    (void)atom_off;
}

// Count (FILL = false) or write (FILL = true) the neighbour set of every atom
// of one system.  Rows visit the distinct cells of the 3x3x3 stencil in a
// fixed order and each cell's atoms in cell order; both tables hold the same
// entries in the same order: col the global slot, col16 the index into the
// brick's LDS tile (own slots first, then the halo list).  Thread k is the
// atom at cell-order position k; positions are read in cell order (cx, cy,
// cz), so a candidate's distance needs no slot lookup, and the slot is read
// only for an accepted neighbour of the FILL pass.
template <bool FILL>
__global__ void k_neighbors(int32_t n, const int32_t *pos_slot, const double *cx,
                            const double *cy, const double *cz, const int32_t *cell_int,
                            const int32_t *start, const int32_t *rank_of_cell,
                            const int32_t *cell_of_rank, const int32_t *brick_of_rank,
                            const BrickInfo *bricks, const int32_t *shell, Grid g, double rc2,
                            int32_t *cnt, const SliceInfo *slices, int32_t *col,
                            uint16_t *colh) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int32_t self = pos_slot[k];
    const double xi = cx[k], yi = cy[k], zi = cz[k];
    const int32_t rank0 = cell_int[self];
    const int32_t cell0 = cell_of_rank[rank0];
    int32_t ic[3] = {cell0 / (g.nc[1] * g.nc[2]), (cell0 / g.nc[2]) % g.nc[1], cell0 % g.nc[2]};
    int32_t sx[3], sy[3], sz[3], ox[3], oy[3], oz[3];
    int mx = axis_cells(ic[0], g.nc[0], g.periodic[0], sx, ox);
    int my = axis_cells(ic[1], g.nc[1], g.periodic[1], sy, oy);
    int mz = axis_cells(ic[2], g.nc[2], g.periodic[2], sz, oz);
    int32_t m = 0;
    int64_t base = 0, basew = 0;
    int32_t width = 0;
    BrickInfo bi{};
    if (FILL) {
        const SliceInfo si = slices[self / kWave];
        base = (int64_t)si.col_base64 * kWave + (self & (kWave - 1));
        basew = (int64_t)si.colw_base64 * kWave + (self & (kWave - 1));
        width = si.width;
        bi = bricks[brick_of_rank[rank0]];
    }
    for (int a = 0; a < mx; ++a)
        for (int b = 0; b < my; ++b)
            for (int e = 0; e < mz; ++e) {
                const int32_t cell = (sx[a] * g.nc[1] + sy[b]) * g.nc[2] + sz[e];
                const int32_t rk = rank_of_cell[cell];
                int32_t hbase = 0;
                bool own = true;
                if (FILL) {
                    const int32_t p0 = ic[0] - bi.o[0] + ox[a] + 1;
                    const int32_t p1 = ic[1] - bi.o[1] + oy[b] + 1;
                    const int32_t p2 = ic[2] - bi.o[2] + oz[e] + 1;
                    const int32_t h = shell[bi.shell_off + (p0 * bi.sh[1] + p1) * bi.sh[2] + p2];
                    own = (h == -1);
                    hbase = bi.n_own_pad + h;
                }
                for (int32_t q = start[rk]; q < start[rk + 1]; ++q) {
                    if (q == k) continue;
                    double dx = min_image(cx[q] - xi, g.len[0], g.periodic[0]);
                    double dy = min_image(cy[q] - yi, g.len[1], g.periodic[1]);
                    double dz = min_image(cz[q] - zi, g.len[2], g.periodic[2]);
                    if (dx * dx + dy * dy + dz * dz <= rc2) {
                        if (FILL && m < width) {
                            const int32_t j = pos_slot[q];
                            col[base + (int64_t)m * kWave] = j;
                            const int32_t loc = own ? j - bi.slot0 : hbase + (q - start[rk]);
                            colh[2 * (basew + (int64_t)(m >> 1) * kWave) + (m & 1)] =
                                (uint16_t)(4 * loc);
                        }
                        ++m;
                    }
                }
            }
    if (FILL) {
        for (int32_t q = m; q < width; ++q) col[base + (int64_t)q * kWave] = self;
        for (int32_t q = m; q < (width + 1) / 2 * 2; ++q)
            colh[2 * (basew + (int64_t)(q >> 1) * kWave) + (q & 1)] =
                (uint16_t)(4 * (self - bi.slot0));
    } else {
        cnt[self] = m;
    }
}

// Neighbour rows in one search, one wave per cell.  The wave takes the
// cell's own atoms (cell-order positions k0..k0+na-1 of its system, na <= 64)
// and, for every distinct cell of the 3x3x3 stencil in the fixed order, its
// candidates T = 64 / na at a time: lane L pairs own atom L mod na with
// candidate L / na of the chunk, so the lanes of one candidate read the same
// position.  Atom i's lanes are i, i + na, ...; its accepted candidates keep
// the row order of the thread-per-atom search (stencil cell, then cell order),
// and a lane's place in the row is the atom's running length plus the
// accepted lanes of the same atom below it (a popcount of the ballot).  Every
// lane of an atom carries its running length, so no shared memory is used.
// Rows go to a temporary table in cell order, wcap entries per atom: the
// global cell-order index of the neighbour and its offset in the brick's halo
// list (-1 for a neighbour of the atom's own brick, whose tile place follows
// the count order).  cnt[slot] receives the full count; a row longer than
// wcap raises *overflow and the caller falls back to the thread-per-atom fill.
__global__ __launch_bounds__(256) void k_cell_rows(
    int32_t ncell, int64_t caller_off, const int32_t *__restrict__ pos_slot /*all systems*/,
    const double *__restrict__ cx, const double *__restrict__ cy,
    const double *__restrict__ cz /*this system, cell order*/,
    const int32_t *__restrict__ start, const int32_t *__restrict__ rank_of_cell,
    const int32_t *__restrict__ cell_of_rank, const int32_t *__restrict__ brick_of_rank,
    const BrickInfo *__restrict__ bricks, const int32_t *__restrict__ shell, Grid g, double rc2,
    int32_t wcap, int32_t *__restrict__ cnt, int32_t *__restrict__ tq,
    int16_t *__restrict__ th, unsigned *__restrict__ overflow) {
    // the cell, its atoms and its stencil are wave-uniform: scalar registers and loads
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int32_t r = blockIdx.x * (blockDim.x / kWave) + wave;   // cell rank in this system
    if (r >= ncell) return;
    const int32_t k0 = start[r], na = start[r + 1] - k0;
    if (na == 0 || na > kWave) return;
    const int32_t il = lane % na, tl = lane / na;   // the lane's atom and candidate slot
    const int32_t T = kWave / na;                    // candidates per chunk
    uint64_t pat = 0;                                // lanes 0, na, 2 na, ... of atom 0
    for (int32_t t = 0; t < T; ++t) pat |= 1ull << (t * na);
    const uint64_t mine = pat << il;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    const int32_t k = k0 + il;
    const double xk = cx[k], yk = cy[k], zk = cz[k];
    const int32_t cell0 = cell_of_rank[r];
    const int32_t ic[3] = {cell0 / (g.nc[1] * g.nc[2]), (cell0 / g.nc[2]) % g.nc[1], cell0 % g.nc[2]};
    int32_t sx[3], sy[3], sz[3], ox[3], oy[3], oz[3];
    const int mx = axis_cells(ic[0], g.nc[0], g.periodic[0], sx, ox);
    const int my = axis_cells(ic[1], g.nc[1], g.periodic[1], sy, oy);
    const int mz = axis_cells(ic[2], g.nc[2], g.periodic[2], sz, oz);
    const BrickInfo bi = bricks[brick_of_rank[r]];
    const int64_t row = (caller_off + k) * (int64_t)wcap;
    // the stencil cells in row order t = (a my + b) mz + e: lane t looks up
    // cell t's rank, atom range and halo offset, so the wave waits for one
    // round of these loads instead of one dependent chain per stencil cell
    const int32_t nst = mx * my * mz;
    int32_t q0_l = 0, ms_l = 0, hc_l = 0;
    if (lane < nst) {
        const int a = lane / (my * mz), b = (lane / mz) % my, e = lane % mz;
        const int32_t xa = a == 0 ? sx[0] : (a == 1 ? sx[1] : sx[2]);
        const int32_t yb = b == 0 ? sy[0] : (b == 1 ? sy[1] : sy[2]);
        const int32_t ze = e == 0 ? sz[0] : (e == 1 ? sz[1] : sz[2]);
        const int32_t oa = a == 0 ? ox[0] : (a == 1 ? ox[1] : ox[2]);
        const int32_t ob = b == 0 ? oy[0] : (b == 1 ? oy[1] : oy[2]);
        const int32_t oe = e == 0 ? oz[0] : (e == 1 ? oz[1] : oz[2]);
        const int32_t rk = rank_of_cell[(xa * g.nc[1] + yb) * g.nc[2] + ze];
        const int32_t p0c = ic[0] - bi.o[0] + oa + 1;
        const int32_t p1c = ic[1] - bi.o[1] + ob + 1;
        const int32_t p2c = ic[2] - bi.o[2] + oe + 1;
        hc_l = shell[bi.shell_off + (p0c * bi.sh[1] + p1c) * bi.sh[2] + p2c];
        q0_l = start[rk];
        ms_l = start[rk + 1] - q0_l;
    }
    int32_t len = 0;
    // the first chunk of candidate positions of the next stencil cell is
    // requested before the current cell is searched
    double nx = 0.0, ny = 0.0, nz = 0.0;
    auto first_chunk = [&](int32_t t, double &px, double &py, double &pz) {
        const int32_t q0 = __builtin_amdgcn_readlane(q0_l, t);
        const int32_t ms = __builtin_amdgcn_readlane(ms_l, t);
        if (tl < T && tl < ms) {
            px = cx[q0 + tl];
            py = cy[q0 + tl];
            pz = cz[q0 + tl];
        }
    };
    if (nst > 0) first_chunk(0, nx, ny, nz);
    for (int32_t t = 0; t < nst; ++t) {
        const int32_t q0 = __builtin_amdgcn_readlane(q0_l, t);
        const int32_t ms = __builtin_amdgcn_readlane(ms_l, t);
        const int32_t hcell = __builtin_amdgcn_readlane(hc_l, t);
        const double fx = nx, fy = ny, fz = nz;
        if (t + 1 < nst) first_chunk(t + 1, nx, ny, nz);
        for (int32_t c0 = 0; c0 < ms; c0 += T) {
            const int32_t jq = c0 + tl;
            const int32_t q = q0 + jq;
            bool acc = false;
            if (tl < T && jq < ms && q != k) {
                const double px = c0 == 0 ? fx : cx[q];
                const double py = c0 == 0 ? fy : cy[q];
                const double pz = c0 == 0 ? fz : cz[q];
                const double dx = min_image(px - xk, g.len[0], g.periodic[0]);
                const double dy = min_image(py - yk, g.len[1], g.periodic[1]);
                const double dz = min_image(pz - zk, g.len[2], g.periodic[2]);
                acc = dx * dx + dy * dy + dz * dz <= rc2;
            }
            const uint64_t mask = __ballot(acc);
            if (acc) {
                const int32_t m = len + __popcll(mask & mine & below);
                if (m < wcap) {
                    tq[row + m] = (int32_t)(caller_off + q);
                    th[row + m] = (int16_t)(hcell == -1 ? -1 : hcell + jq);
                }
            }
            len += __popcll(mask & mine);
        }
    }
    if (tl == 0) {
        cnt[pos_slot[caller_off + k]] = len;
        if (len > wcap) atomicOr(overflow, 1u);
    }
}

// sum and largest value of the per-slot neighbour counts (padding slots hold 0)
__global__ __launch_bounds__(256) void k_count_stats(const int32_t *__restrict__ cnt, int64_t n,
                                                     unsigned long long *__restrict__ sum,
                                                     int32_t *__restrict__ mx) {
    __shared__ unsigned long long bs[256];
    __shared__ int32_t bm[256];
    unsigned long long a = 0;
    int32_t m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = cnt[i];
        a += (unsigned long long)v;
        m = max(m, v);
    }
    bs[threadIdx.x] = a;
    bm[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            bs[threadIdx.x] += bs[threadIdx.x + w];
            bm[threadIdx.x] = max(bm[threadIdx.x], bm[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicAdd(sum, bs[0]);
        atomicMax(mx, bm[0]);
    }
}

// slot -> global cell-order index (the inverse of pos_slot)
__global__ void k_cell_index(const int32_t *pos_slot, int64_t n_tot, int32_t *kof) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tot) kof[pos_slot[t]] = (int32_t)t;
}

// Both neighbour tables from the temporary rows, one thread per slot, so the
// writes of a slice's lanes are coalesced: col the global slot, col16 the LDS
// byte offset (own brick: the neighbour's slot after the count order; halo:
// after the brick's own slots).  Entries past the count point at the slot.
__global__ void k_rows_fill(int32_t n_int, const int32_t *__restrict__ perm,
                            const int32_t *__restrict__ kof, const int32_t *__restrict__ cnt,
                            const SliceInfo *__restrict__ slices, const BrickInfo *__restrict__ bricks,
                            const int32_t *__restrict__ pos_slot, const int32_t *__restrict__ tq,
                            const int16_t *__restrict__ th, int32_t wcap, int32_t *__restrict__ col,
                            uint16_t *__restrict__ colh) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_int || perm[s] < 0) return;
    const SliceInfo si = slices[s / kWave];
    const BrickInfo &bi = bricks[si.brick];
    const int64_t base = (int64_t)si.col_base64 * kWave + (s & (kWave - 1));
    const int64_t basew = (int64_t)si.colw_base64 * kWave + (s & (kWave - 1));
    const int32_t width = si.width, slot0 = bi.slot0, own_pad = bi.n_own_pad;
    const int32_t m_n = min(cnt[s], width);
    const int64_t row = (int64_t)kof[s] * wcap;
#pragma unroll 4
    for (int32_t m = 0; m < m_n; ++m) {
        const int32_t j = pos_slot[tq[row + m]];
        const int32_t h = th[row + m];
        col[base + (int64_t)m * kWave] = j;
        colh[2 * (basew + (int64_t)(m >> 1) * kWave) + (m & 1)] =
            (uint16_t)(4 * (h < 0 ? j - slot0 : own_pad + h));
    }
    for (int32_t m = m_n; m < width; ++m) col[base + (int64_t)m * kWave] = s;
    for (int32_t m = m_n; m < (width + 1) / 2 * 2; ++m)
        colh[2 * (basew + (int64_t)(m >> 1) * kWave) + (m & 1)] = (uint16_t)(4 * (s - slot0));
}

// Within each brick, order the atoms by neighbour count (descending, ties in
// cell order) so the 64 lanes of a slice carry rows of nearly equal length;
// the brick kernel reads its tile from LDS, so the order inside a brick costs
// no locality.  One workgroup per non-empty brick; writes new_slot[old slot].
__global__ void k_brick_rank(const BrickInfo *bricks, const int32_t *list, const int32_t *cnt,
                             int32_t *new_slot) {
    extern __shared__ int32_t lc[];
    __shared__ int32_t hist[256];
    const BrickInfo bi = bricks[list[blockIdx.x]];
    for (int32_t t = threadIdx.x; t < 256; t += blockDim.x) hist[t] = 0;
    for (int32_t t = threadIdx.x; t < bi.n_own; t += blockDim.x)
        lc[t] = 255 - min(cnt[bi.slot0 + t], 255);
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int32_t t = 0; t < bi.n_own; ++t) ++hist[lc[t]];
        int32_t acc = 0;
        for (int b = 0; b < 256; ++b) {
            const int32_t v = hist[b];
            hist[b] = acc;
            acc += v;
        }
        for (int32_t t = 0; t < bi.n_own; ++t) lc[t] = hist[lc[t]]++;
    }
    __syncthreads();
    for (int32_t t = threadIdx.x; t < bi.n_own; t += blockDim.x)
        new_slot[bi.slot0 + t] = bi.slot0 + lc[t];
}

__global__ void k_iota(int32_t *p, int32_t n) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) p[s] = s;
}

__global__ void k_scatter_i32(const int32_t *src, const int32_t *to, int32_t n, int32_t *dst) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[to[s]] = src[s];
}

__global__ void k_scatter_f64(const double *src, const int32_t *to, int32_t n, double *dst) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) dst[to[s]] = src[s];
}

__global__ void k_inverse(const int32_t *perm, int32_t n, int32_t *inv) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n && perm[s] >= 0) inv[perm[s]] = s;
}

__global__ void k_remap(int32_t *p, int64_t n, const int32_t *to) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = to[p[i]];
}

__global__ void k_slice_width(const int32_t *cnt, const int32_t *perm, int32_t n_slices,
                              int32_t *width, int32_t *nvalid) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slices) return;
    int32_t w = 0, v = 0;
    for (int l = 0; l < kWave; ++l) {
        int32_t slot = s * kWave + l;
        if (perm[slot] >= 0) {
            w = max(w, cnt[slot]);
            ++v;
        }
    }
    width[s] = w;
    nvalid[s] = v;
}

// padding slots still run the neighbour loop of their slice: every entry of
// their rows points at the slot itself (pair term zero, always in bounds)
__global__ void k_pad_rows(const int32_t *perm, const SliceInfo *slices, const BrickInfo *bricks,
                           int32_t n_int, int32_t *col, uint16_t *colh) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_int || perm[s] >= 0) return;
    const SliceInfo si = slices[s / kWave];
    const int64_t base = (int64_t)si.col_base64 * kWave + (s & (kWave - 1));
    const int64_t basew = (int64_t)si.colw_base64 * kWave + (s & (kWave - 1));
    const int32_t loc = s - bricks[si.brick].slot0;
    for (int32_t q = 0; q < si.width; ++q) col[base + (int64_t)q * kWave] = s;
    for (int32_t q = 0; q < (si.width + 1) / 2 * 2; ++q)
        colh[2 * (basew + (int64_t)(q >> 1) * kWave) + (q & 1)] = (uint16_t)(4 * loc);
}

// halo list of every brick: the slots of the atoms of its halo cells
__global__ void k_halo_expand(const HaloCell *hc, int64_t n_hc, const BrickInfo *bricks,
                              const int32_t *start_all, const int32_t *pos_slot_all,
                              int32_t *halo) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_hc) return;
    const HaloCell h = hc[e];
    const BrickInfo &b = bricks[h.brick];
    const int32_t q0 = start_all[h.start_index], q1 = start_all[h.start_index + 1];
    for (int32_t q = q0; q < q1; ++q) halo[b.halo_off + h.offset + (q - q0)] = pos_slot_all[h.pos_base + q];
}

// estimated work of every listed brick for the XCD split of the brick
// launches, in tenths of a vector instruction per wave: per slice 11 per row
// entry (the pair term, its FP64 sum and the offset) and 140 for the update
// and the ledgers; 0.1 per staged slot; 400 for the workgroup
__global__ void k_brick_work(const BrickInfo *bricks, const int32_t *list, int32_t n_list,
                             const SliceInfo *slices, int32_t *work) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n_list) return;
    const BrickInfo bi = bricks[list[q]];
    int32_t w = 4000 + bi.n_own_pad + bi.n_halo;
    for (int32_t k = 0; k < bi.n_own_pad / kWave; ++k) w += 110 * slices[bi.slice0 + k].width + 1400;
    work[q] = w;
}

// the padding of every halo list: entries n_halo .. to the next multiple of 4
// repeat entry n_halo - 1
__global__ void k_halo_pad(const BrickInfo *bricks, int32_t n_bricks, int32_t *halo) {
    const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_bricks) return;
    const BrickInfo bi = bricks[b];
    if (bi.n_halo <= 0) return;
    const int32_t last = halo[bi.halo_off + bi.n_halo - 1];
    for (int32_t k = bi.n_halo; k < halo_padded(bi.n_halo); ++k) halo[bi.halo_off + k] = last;
}

__global__ void k_field_in(int32_t atom_off, int32_t n_pad, const int32_t *perm, int64_t caller_off,
                           const double *src, int32_t field, int32_t precision, double *T64,
                           float *Thi, int16_t *Tlo, double *Tl64, float *Tl32, double *srcw64,
                           float *srcw32) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    int32_t slot = atom_off + k;
    int32_t g = perm[slot];
    double v = (g >= 0) ? src[g - caller_off] : 0.0;
    if (field == L2T_FIELD_TE) {
        if (precision == L2T_FP64) {
            T64[slot] = v;
        } else {
            const float hi = (float)v;
            Thi[slot] = hi;
            Tlo[slot] = state_lo(v, hi);
        }
    } else if (field == L2T_FIELD_TL) {
        if (precision == L2T_FP64) {
            Tl64[slot] = copysign(v, signbit(Tl64[slot]) ? -1.0 : 1.0);
        } else {
            Tl32[slot] = copysignf((float)v, signbit(Tl32[slot]) ? -1.0f : 1.0f);
        }
    } else if (field == L2T_FIELD_GATE) {
        bool gated = (g >= 0) && v != 0.0;
        if (precision == L2T_FP64) {
            Tl64[slot] = gated ? -fabs(Tl64[slot]) : fabs(Tl64[slot]);
        } else {
            Tl32[slot] = gated ? -fabsf(Tl32[slot]) : fabsf(Tl32[slot]);
        }
    } else if (field == L2T_FIELD_FIXED) {
        // the sign bit of the source weight marks an atom that holds its T_e
        bool fixed = (g >= 0) && v != 0.0;
        if (precision == L2T_FP64) {
            srcw64[slot] = fixed ? -fabs(srcw64[slot]) : fabs(srcw64[slot]);
        } else {
            srcw32[slot] = fixed ? -fabsf(srcw32[slot]) : fabsf(srcw32[slot]);
        }
    }
}

__global__ void k_field_out(int32_t atom_off, int32_t n_pad, const int32_t *perm, int64_t caller_off,
                            int32_t field, int32_t precision, const double *T64, const float *Thi,
                            const int16_t *Tlo, const double *Tl64, const float *Tl32,
                            const int32_t *cnt, const double *eatom, const double *srcw64,
                            const float *srcw32, double *dst) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    int32_t slot = atom_off + k;
    int32_t g = perm[slot];
    if (g < 0) return;
    double v = 0.0;
    if (field == L2T_FIELD_TE) {
        v = (precision == L2T_FP64) ? T64[slot] : state_value(Thi[slot], Tlo[slot]);
    } else if (field == L2T_FIELD_TL) {
        v = (precision == L2T_FP64) ? fabs(Tl64[slot]) : (double)fabsf(Tl32[slot]);
    } else if (field == L2T_FIELD_GATE) {
        bool s = (precision == L2T_FP64) ? signbit(Tl64[slot]) : signbit(Tl32[slot]);
        v = s ? 1.0 : 0.0;
    } else if (field == L2T_FIELD_NBRS) {
        v = (double)cnt[slot];
    } else if (field == L2T_FIELD_ELAT) {
        v = eatom[slot];
    } else if (field == L2T_FIELD_FIXED) {
        bool s = (precision == L2T_FP64) ? signbit(srcw64[slot]) : signbit(srcw32[slot]);
        v = s ? 1.0 : 0.0;
    }
    dst[g - caller_off] = v;
}

// kSliceHeld of every slice of a system from the sign bits of its source weights
__global__ void k_slice_held(SliceInfo *slices, int32_t slice0, int32_t n_slices,
                             int32_t precision, const double *srcw64, const float *srcw32) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t q = blockIdx.x * (blockDim.x / kWave) + wave;
    if (q >= n_slices) return;
    const int32_t sl = slice0 + q;
    const int32_t slot = sl * kWave + lane;
    const bool held = lane < slices[sl].n_valid &&
                      ((precision == L2T_FP64) ? signbit(srcw64[slot]) : signbit(srcw32[slot]));
    const bool any = __any(held);
    if (lane == 0) slices[sl].flags = any ? (slices[sl].flags | kSliceHeld)
                                          : (slices[sl].flags & ~kSliceHeld);
}

__global__ void k_range_count(const double *v, int64_t n, double lo, double hi, unsigned *bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = v[i];
    if (!(x >= lo && x <= hi)) atomicAdd(bad, 1u);
}

// ---- Eq. 4 lattice temperature -----------------------------------------------
// gather velocities and masses of one system into internal order
__global__ void k_gather_vm(int32_t atom_off, int32_t n_pad, const int32_t *perm, int64_t caller_off,
                            int32_t n, const double *v, const double *m, double *out /*[4][n_pad]*/) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    int32_t g = perm[atom_off + k];
    if (g < 0) {
        out[k] = out[n_pad + k] = out[2 * n_pad + k] = out[3 * n_pad + k] = 0.0;
        return;
    }
    int64_t i = g - caller_off;
    out[k] = v[i];
    out[n_pad + k] = v[n + i];
    out[2 * n_pad + k] = v[2 * n + i];
    out[3 * n_pad + k] = m[i];
}

// system-wide momentum and mass (one workgroup, fixed reduction order)
__global__ void k_momentum(const double *vm, int32_t n_pad, double *out /*[4]*/) {
    __shared__ double red[4][256];
    const int t = threadIdx.x;
    double a[4] = {0, 0, 0, 0};
    for (int32_t k = t; k < n_pad; k += blockDim.x) {
        double m = vm[3 * n_pad + k];
        a[0] += m * vm[k];
        a[1] += m * vm[n_pad + k];
        a[2] += m * vm[2 * n_pad + k];
        a[3] += m;
    }
    for (int q = 0; q < 4; ++q) red[q][t] = a[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w)
            for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int q = 0; q < 4; ++q) out[q] = red[q][0];
}

// T_i^lat = sum_{j in {i} U N(i)} 1/2 m_j |v_j - v_com|^2 / (3/2 k_B N_j); the
// coupling of atom i is gated off where 1/2 m_i |v_i - v_com|^2 < ke_eps.  The
// gate is stored in the sign bit of T^lat.  With the local centre of mass
// (the Eq. 4 form) one pass over the neighbours accumulates, for the
// velocities u_j = v_j - v_i shifted by the atom's own, M = sum m_j,
// P = sum m_j u_j and Q = sum m_j |u_j|^2: then v_i - v_com = -P/M and
// sum 1/2 m_j |v_j - v_com|^2 = 1/2 (Q - |P|^2/M).  The shift keeps the
// subtraction at the scale of the thermal spread (a common drift cancels
// in u exactly), as in the shifted-data form of a variance.
__global__ void k_lattice_temp(int32_t atom_off, int32_t n_pad, const int32_t *perm,
                               const SliceInfo *slices, const int32_t *col, const double *vm,
                               const double *gmom, int32_t global_com, double ke_eps,
                               int32_t precision, double *Tl64, float *Tl32) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    int32_t slot = atom_off + k;
    if (perm[slot] < 0) return;
    const double *vx = vm, *vy = vm + n_pad, *vz = vm + 2 * n_pad, *ms = vm + 3 * n_pad;
    const SliceInfo si = slices[slot / kWave];
    const int64_t base = (int64_t)si.col_base64 * kWave + (slot & (kWave - 1));
    double Ki, KE;
    int32_t nj = 1;
    if (global_com) {
        const double vc[3] = {gmom[0] / gmom[3], gmom[1] / gmom[3], gmom[2] / gmom[3]};
        const double ux = vx[k] - vc[0], uy = vy[k] - vc[1], uz = vz[k] - vc[2];
        Ki = 0.5 * ms[k] * (ux * ux + uy * uy + uz * uz) * kMvv2e;
        KE = Ki;
        for (int32_t q = 0; q < si.width; ++q) {
            const int32_t j = col[base + (int64_t)q * kWave];
            if (j == slot) continue;
            const int32_t l = j - atom_off;
            const double wx = vx[l] - vc[0], wy = vy[l] - vc[1], wz = vz[l] - vc[2];
            KE += 0.5 * ms[l] * (wx * wx + wy * wy + wz * wz) * kMvv2e;
            ++nj;
        }
    } else {
        const double xi = vx[k], yi = vy[k], zi = vz[k];
        double M = ms[k], P[3] = {0.0, 0.0, 0.0}, Q = 0.0;
        auto add = [&](int32_t j, double m, double wx, double wy, double wz) {
            if (j == slot) return;   // row padding
            const double ux = wx - xi, uy = wy - yi, uz = wz - zi;
            M += m;
            P[0] += m * ux;
            P[1] += m * uy;
            P[2] += m * uz;
            Q += m * (ux * ux + uy * uy + uz * uz);
            ++nj;
        };
        // neighbours 8 at a time: the chunk's references, then their
        // velocities and masses, are requested before any is added; the sums
        // take the terms in row order either way
        constexpr int kChunk = 8;
        int32_t q = 0;
        for (; q + kChunk <= si.width; q += kChunk) {
            int32_t j[kChunk];
            double m[kChunk], wx[kChunk], wy[kChunk], wz[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) j[u] = col[base + (int64_t)(q + u) * kWave];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) {
                const int32_t l = j[u] - atom_off;
                m[u] = ms[l];
                wx[u] = vx[l];
                wy[u] = vy[l];
                wz[u] = vz[l];
            }
#pragma unroll
            for (int u = 0; u < kChunk; ++u) add(j[u], m[u], wx[u], wy[u], wz[u]);
        }
        for (; q < si.width; ++q) {
            const int32_t j = col[base + (int64_t)q * kWave];
            const int32_t l = j - atom_off;
            add(j, ms[l], vx[l], vy[l], vz[l]);
        }
        const double P2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
        // v_i - v_com = -P / M
        Ki = 0.5 * ms[k] * (P2 / (M * M)) * kMvv2e;
        KE = 0.5 * fmax(Q - P2 / M, 0.0) * kMvv2e;
    }
    double T = KE / (1.5 * kBoltzmann * (double)nj);
    bool gated = Ki < ke_eps;
    if (precision == L2T_FP64) {
        Tl64[slot] = gated ? -T : T;
        if (gated && T == 0.0) Tl64[slot] = -0.0;
    } else {
        float f = (float)T;
        Tl32[slot] = gated ? -f : f;
        if (gated && f == 0.0f) Tl32[slot] = -0.0f;
    }
}

// depth weight of the Eq. 10 source: exp(-(x_i - x_0)/l_p)
__global__ void k_source_weights(int32_t atom_off, int32_t n_pad, const int32_t *perm,
                                 const double *qx, double x0, double lp, double *w64, float *w32) {
    int32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_pad) return;
    int32_t slot = atom_off + k;
    double w = (perm[slot] >= 0) ? exp(-(qx[slot] - x0) / lp) : 0.0;
    // keep the sign bit: it marks atoms that hold their T_e
    if (w64) w64[slot] = copysign(w, w64[slot]);
    if (w32) w32[slot] = copysignf((float)w, w32[slot]);
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// Largest LDS tile (own slots + halo atoms) of one workgroup, in floats: 64 KB
// less 256 bytes, which the FP32C brick kernel keeps beside the tile for its
// per-wave temperature range.
constexpr int32_t kTileCapFloats = 16384 - 64;

namespace {

struct SysLayout {
    int32_t b[3] = {1, 1, 1}, nb[3] = {1, 1, 1};
    int32_t nbrick = 0, brick0 = 0;
    int64_t rank_off = 0;                 // into the rank maps (sum of ncell)
    std::vector<int32_t> brick_cell0;   // first rank of every brick (+ the total)
};

// rank of cell (x, y, z) in brick order (the formula of k_rank_maps)
inline int32_t rank_of(const SysLayout &L, const int32_t nc[3], int32_t x, int32_t y, int32_t z) {
    const int32_t X = x / L.b[0], Y = y / L.b[1], Z = z / L.b[2];
    const int32_t e1 = std::min(L.b[1], nc[1] - Y * L.b[1]);
    const int32_t e2 = std::min(L.b[2], nc[2] - Z * L.b[2]);
    const int32_t bidx = (X * L.nb[1] + Y) * L.nb[2] + Z;
    return L.brick_cell0[bidx] + ((x - X * L.b[0]) * e1 + (y - Y * L.b[1])) * e2 +
           (z - Z * L.b[2]);
}

// Brick edge (cells), one for all systems of the context; along an axis with
// fewer cells than the edge a brick spans the whole axis.  A brick's own
// slots are padded to whole 64-lane slices and its tile adds the one-cell
// halo (clipped to the system's extent, where the halo wraps onto the brick
// itself).  The tile at each system's mean density, with room for
// fluctuations, must fit the LDS cap; among the edges that fit, take the one
// with the least estimated time: rounds of resident workgroups over all bricks
// of all systems (one brick per workgroup; a CU holds as many tiles as its
// 160 KB of LDS and its 8 workgroups of 4 waves allow) times the work of the
// largest brick (its padded slots, plus the halo staging counted at 0.3 of a
// slot).  Edges within 0.1 % of the least time are told apart by the padded
// slots of all bricks together (a few small systems fit in one round at any
// edge, and one-cell bricks would pad every cell to a whole slice).  Edges
// grow until every axis of every system fits in one brick.
int32_t brick_edge(const l2t_ctx *c, int32_t limit) {
    int32_t best = 1;
    double best_cost = 1e300, best_total = 1e300;
    for (int32_t b = 1; b <= limit; ++b) {
        double tile_max = 0.0, work_max = 0.0, nbrick = 0.0, total = 0.0;
        bool grows = false;
        for (const SystemState &st : c->sys) {
            const double dens =
                (double)st.desc.n_atoms / (double)std::max<int64_t>(1, st.ncell);
            double own = 1.0, with_halo = 1.0, nb = 1.0;
            for (int d = 0; d < 3; ++d) {
                const int32_t e = std::min(b, st.nc[d]);
                own *= e;
                with_halo *= std::min(e + 2, st.nc[d]);
                nb *= std::ceil((double)st.nc[d] / e);
                grows |= st.nc[d] > b;
            }
            const double slots = std::ceil(dens * own / kWave) * kWave;
            const double halo = dens * (with_halo - own);
            tile_max = std::max(tile_max, 1.1 * dens * with_halo + kWave);
            work_max = std::max(work_max, slots + 0.3 * halo);
            nbrick += nb;
            total += nb * slots;
        }
        if (tile_max > kTileCapFloats) break;
        const double per_cu = std::max(1.0, std::min(8.0, std::floor(163840.0 / (4.0 * tile_max))));
        const double rounds = std::ceil(nbrick / (per_cu * std::max(1, c->n_cu)));
        const double cost = rounds * work_max;
        if (cost < best_cost * 0.999 || (cost <= best_cost * 1.001 && total < best_total)) {
            best_cost = std::min(best_cost, cost);
            best_total = total;
            best = b;
        }
        if (!grows) break;
    }
    return best;
}

}  // namespace

// cut the brick list into 8 contiguous ranges of about equal estimated work
// and write the launch list (range x at x G/8, -1 after its last brick).
// Splitting by count instead left the XCDs of the 256-slab batch unequal
// (64.1 G atom-substeps/s; 65.7 by work, 66.8 with no XCD ranges at all,
// which costs the 4M-atom system 5 % through its L2 reuse).
int xcd_split(l2t_ctx *c, const std::vector<int32_t> &list, const std::vector<int32_t> &work) {
    const int32_t n = (int32_t)list.size();
    int64_t total = 0;
    for (int32_t w : work) total += w;
    int32_t cut[9];
    cut[0] = 0;
    int64_t acc = 0;
    int32_t q = 0;
    for (int x = 1; x < 8; ++x) {
        const int64_t target = total * x / 8;
        // advance while taking the next brick brings the sum closer to the target
        while (q < n && std::llabs(acc + work[q] - target) <= std::llabs(acc - target)) acc += work[q++];
        cut[x] = q;
    }
    cut[8] = n;
    int32_t per = 0;
    for (int x = 0; x < 8; ++x) per = std::max(per, cut[x + 1] - cut[x]);
    per = std::max(per, 1);
    const int32_t G = 8 * per;
    c->h_xcd_list.assign((size_t)2 * G, -1);
    // inside its range an XCD takes the bricks largest first, so the last
    // workgroups of the launch are small ones (measured on the 4M-atom system,
    // whose bricks are 6 or 7 cells a side: 49.3-50.5 -> 48.4-49.4 us).  The
    // order is by 5 % classes of work, in list order inside a class, which
    // keeps bricks of one size in their spatial order for the L2 (47.7 ->
    // 47.6 us against an order by exact work)
    auto size_class = [&](int32_t k) {
        return (int)std::floor(std::log((double)std::max(work[k], 1)) / std::log(1.05));
    };
    std::vector<int32_t> idx;
    for (int x = 0; x < 8; ++x) {
        idx.clear();
        for (int32_t k = cut[x]; k < cut[x + 1]; ++k) idx.push_back(k);
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int32_t a, int32_t b) { return size_class(a) > size_class(b); });
        for (size_t k = 0; k < idx.size(); ++k) c->h_xcd_list[(size_t)x * per + k] = list[idx[k]];
    }
    // the reversed list: every range backwards (its holes first)
    for (int x = 0; x < 8; ++x)
        for (int32_t k = 0; k < per; ++k)
            c->h_xcd_list[(size_t)G + (size_t)x * per + k] =
                c->h_xcd_list[(size_t)x * per + (per - 1 - k)];
    if ((size_t)2 * G > c->cap_xl) {
        L2T_HIP(c, hipStreamSynchronize(c->stream));
        dev_free(c, c->xcd_list);
        c->xcd_list = nullptr;
        c->cap_xl = 0;
        void *m = nullptr;
        const hipError_t e = dev_malloc(c, &m, sizeof(int32_t) * (size_t)2 * G);
        if (e != hipSuccess) return hip_fail(c, e, "XCD launch list allocation");
        c->xcd_list = static_cast<int32_t *>(m);
        c->cap_xl = (size_t)2 * G;
    }
    L2T_HIP(c, hipMemcpyAsync(c->xcd_list, c->h_xcd_list.data(), sizeof(int32_t) * (size_t)2 * G,
                              hipMemcpyHostToDevice, c->stream));
    c->n_xcd_list = G;
    return L2T_OK;
}

int build_neighbors_once(l2t_ctx *c, double r_cut, int32_t edge_limit, bool forced,
                         bool *tile_overflow) {
    const int S = (int)c->sys.size();
    const hipStream_t st_ = c->stream;
    *tile_overflow = false;
    // ---- cell grids and brick order (host) -------------------------------------
    std::vector<SysLayout> lay(S);
    std::vector<int64_t> cstart_off(S);
    int64_t cells_total = 0, ranks_total = 0;
    int32_t nbricks = 0;
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        st.ncell = 1;
        for (int d = 0; d < 3; ++d) {
            if (st.desc.periodic[d] && st.desc.box_len[d] < 2.0 * r_cut)
                return fail(c, L2T_EINVAL, "system " + std::to_string(s) +
                                               ": periodic box length below 2 r_cut");
            double k = std::floor(st.desc.box_len[d] / r_cut);
            st.nc[d] = (int32_t)std::max(1.0, std::min(k, 1.0e6));
            st.ncell *= st.nc[d];
        }
        if (st.ncell > (int64_t)1 << 28) return fail(c, L2T_EINVAL, "cell grid too large");
    }
    const int32_t be = c->tune.brick_edge > 0 ? std::min(c->tune.brick_edge, edge_limit)
                       : forced                 ? edge_limit
                                                : brick_edge(c, edge_limit);
    c->brick_edge_used = be;
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        SysLayout &L = lay[s];
        L.nbrick = 1;
        for (int d = 0; d < 3; ++d) {
            L.b[d] = std::min(be, st.nc[d]);
            L.nb[d] = (st.nc[d] + L.b[d] - 1) / L.b[d];
            L.nbrick *= L.nb[d];
        }
        L.brick0 = nbricks;
        nbricks += L.nbrick;
        L.rank_off = ranks_total;
        ranks_total += st.ncell;
        cstart_off[s] = cells_total;
        st.cell_off = cells_total;
        cells_total += st.ncell + 1;
        L.brick_cell0.assign(L.nbrick + 1, 0);
        int32_t r = 0, bidx = 0;
        for (int32_t X = 0; X < L.nb[0]; ++X)
            for (int32_t Y = 0; Y < L.nb[1]; ++Y)
                for (int32_t Z = 0; Z < L.nb[2]; ++Z, ++bidx) {
                    L.brick_cell0[bidx] = r;
                    r += std::min(L.b[0], st.nc[0] - X * L.b[0]) *
                         std::min(L.b[1], st.nc[1] - Y * L.b[1]) *
                         std::min(L.b[2], st.nc[2] - Z * L.b[2]);
                }
        L.brick_cell0[L.nbrick] = r;
    }
    // first ranks of every brick, for the device rank maps (system s at brick0 + s)
    std::vector<int32_t> h_bc0((size_t)nbricks + S);
    for (int s = 0; s < S; ++s)
        std::copy(lay[s].brick_cell0.begin(), lay[s].brick_cell0.end(),
                  h_bc0.begin() + lay[s].brick0 + s);
    // grow-only temporaries owned by the context (kept for the next build)
    int32_t *d_rank = tmp_of<int32_t>(c, 0, ranks_total);
    int32_t *d_cell = tmp_of<int32_t>(c, 1, ranks_total);
    int32_t *d_brick = tmp_of<int32_t>(c, 2, ranks_total);
    int32_t *d_count = tmp_of<int32_t>(c, 3, cells_total);
    int32_t *d_start = tmp_of<int32_t>(c, 4, cells_total);
    if (!d_rank || !d_cell || !d_brick || !d_count || !d_start)
        return fail(c, L2T_ENOMEM, "neighbour build scratch allocation failed");
    // the brick starts go through d_count, which binning clears and reuses after
    // the rank maps are written (cells_total >= nbricks + S)
    L2T_HIP(c, hipMemcpyAsync(d_count, h_bc0.data(), sizeof(int32_t) * h_bc0.size(),
                              hipMemcpyHostToDevice, st_));
    for (int s = 0; s < S; ++s) {
        const SystemState &st = c->sys[s];
        const SysLayout &L = lay[s];
        hipLaunchKernelGGL(k_rank_maps, dim3(nblk(st.ncell, 256)), dim3(256), 0, st_,
                           (int64_t)st.ncell, st.nc[1], st.nc[2], L.b[0], L.b[1], L.b[2], L.nb[1],
                           L.nb[2], d_count + L.brick0 + s, L.brick0, d_rank + L.rank_off,
                           d_cell + L.rank_off, d_brick + L.rank_off);
    }
    L2T_HIP(c, hipGetLastError());
    L2T_HIP(c, hipMemsetAsync(c->derr, 0, sizeof(unsigned), st_));
    // ---- binning in brick order (device) -------------------------------------------
    std::vector<Grid> grids(S);
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        Grid &g = grids[s];
        for (int d = 0; d < 3; ++d) {
            g.nc[d] = st.nc[d];
            g.periodic[d] = st.desc.periodic[d];
            g.lo[d] = st.desc.box_lo[d];
            g.len[d] = st.desc.box_len[d];
        }
        const int32_t n = st.desc.n_atoms;
        const double *px = c->pos + st.caller_off, *py = px + c->n_tot, *pz = py + c->n_tot;
        int32_t *count = d_count + cstart_off[s];
        int32_t *start = d_start + cstart_off[s];
        int32_t *cell_of = c->cell_of + st.caller_off;
        int32_t *sorted = c->sorted_local + st.caller_off;
        const int32_t *rank_of_cell = d_rank + lay[s].rank_off;
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk(st.ncell, 256)), dim3(256), 0, st_, count,
                           st.ncell, 0);
        hipLaunchKernelGGL(k_bin, dim3(nblk(n, 256)), dim3(256), 0, st_, px, py, pz, n, g,
                           rank_of_cell, cell_of, count, c->derr);
        {
            const unsigned nt = nblk(st.ncell, kScanTile);
            int32_t *bsum = tmp_of<int32_t>(c, 11, 2 * (int64_t)nt + 1);
            if (!bsum) return fail(c, L2T_ENOMEM, "scan scratch allocation failed");
            hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kScanThreads), 0, st_, count,
                               (int64_t)st.ncell, bsum);
            hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st_, bsum, bsum + nt,
                               (int64_t)nt);
            hipLaunchKernelGGL(k_tile_scan, dim3(nt), dim3(kScanThreads), 0, st_, count,
                               (int64_t)st.ncell, bsum + nt, start);
        }
        hipLaunchKernelGGL(k_fill_i32, dim3(nblk(st.ncell, 256)), dim3(256), 0, st_, count,
                           st.ncell, 0);
        hipLaunchKernelGGL(k_scatter, dim3(nblk(n, 256)), dim3(256), 0, st_, cell_of, n, start,
                           count, sorted);
        hipLaunchKernelGGL(k_sort_cells, dim3(nblk(st.ncell, 256)), dim3(256), 0, st_, start,
                           st.ncell, sorted);
    }
    L2T_HIP(c, hipGetLastError());
    std::vector<int32_t> h_start(cells_total);
    L2T_HIP(c, hipMemcpyAsync(h_start.data(), d_start, sizeof(int32_t) * cells_total,
                              hipMemcpyDeviceToHost, st_));
    unsigned herr = 0;
    L2T_HIP(c, hipMemcpyAsync(&herr, c->derr, sizeof(unsigned), hipMemcpyDeviceToHost, st_));
    L2T_HIP(c, hipStreamSynchronize(st_));
    if (herr & kErrBox) return fail(c, L2T_EINVAL, "an atom lies outside the box on a free axis");
    // ---- slot layout, halo tables (host) -------------------------------------------
    // slots and shell offsets in brick order (sequential, cheap); then every
    // brick's shell table and halo cell list (independent, split over host
    // threads); then halo offsets in brick order
    std::vector<BrickInfo> hb(nbricks);
    std::vector<int32_t> h_atom0(nbricks), h_list;
    std::vector<int32_t> h_shell;
    std::vector<HaloCell> h_halo;
    int32_t slot = 0;
    int64_t halo_total = 0, shell_total = 0;
    int32_t tile_max = 0;
    std::vector<int32_t> sys_of_brick(nbricks);
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        const SysLayout &L = lay[s];
        const int32_t *start = h_start.data() + cstart_off[s];
        st.atom_off = slot;
        st.list0 = (int32_t)h_list.size();
        for (int32_t b = 0; b < L.nbrick; ++b) {
            const int32_t gb = L.brick0 + b;
            BrickInfo &bi = hb[gb];
            sys_of_brick[gb] = s;
            const int32_t X = b / (L.nb[1] * L.nb[2]), Y = (b / L.nb[2]) % L.nb[1], Z = b % L.nb[2];
            bi.o[0] = X * L.b[0];
            bi.o[1] = Y * L.b[1];
            bi.o[2] = Z * L.b[2];
            for (int d = 0; d < 3; ++d) bi.sh[d] = std::min(L.b[d], st.nc[d] - bi.o[d]) + 2;
            const int32_t a0 = start[L.brick_cell0[b]], a1 = start[L.brick_cell0[b + 1]];
            h_atom0[gb] = a0;
            bi.sys = s;
            bi.slot0 = slot;
            bi.n_own = a1 - a0;
            bi.n_own_pad = (bi.n_own + kWave - 1) / kWave * kWave;
            bi.slice0 = slot / kWave;
            bi.n_halo = 0;
            bi.halo_off = 0;
            bi.shell_off = (int32_t)shell_total;
            slot += bi.n_own_pad;
            if (bi.n_own == 0) continue;
            h_list.push_back(gb);
            shell_total += (int64_t)bi.sh[0] * bi.sh[1] * bi.sh[2];
        }
        st.n_pad = slot - st.atom_off;
        st.slice0 = st.atom_off / kWave;
        st.n_slices = st.n_pad / kWave;
        st.n_list = (int32_t)h_list.size() - st.list0;
    }
    if (shell_total > INT32_MAX) return fail(c, L2T_ENOMEM, "shell tables too large");
    h_shell.assign((size_t)shell_total, 0);
    const int32_t n_list = (int32_t)h_list.size();
    const int n_thr = (int)std::max<int64_t>(
        1, std::min<int64_t>({16, (int64_t)std::thread::hardware_concurrency(), n_list / 32}));
    std::vector<std::vector<HaloCell>> part(n_thr);
    auto tables = [&](int t) {
        const int32_t q0 = (int32_t)((int64_t)n_list * t / n_thr);
        const int32_t q1 = (int32_t)((int64_t)n_list * (t + 1) / n_thr);
        std::vector<int32_t> cv[3], seen;
        std::vector<char> ok[3], own[3];
        for (int32_t q = q0; q < q1; ++q) {
            const int32_t gb = h_list[q];
            BrickInfo &bi = hb[gb];
            const int s = sys_of_brick[gb];
            const SystemState &st = c->sys[s];
            const SysLayout &L = lay[s];
            const int32_t *start = h_start.data() + cstart_off[s];
            // per axis: wrapped cell coordinate, inside the grid, inside the brick
            bool wraps = false;
            for (int d = 0; d < 3; ++d) {
                const int32_t e = bi.sh[d] - 2;
                cv[d].resize(bi.sh[d]);
                ok[d].resize(bi.sh[d]);
                own[d].resize(bi.sh[d]);
                for (int32_t p = 0; p < bi.sh[d]; ++p) {
                    int32_t v = bi.o[d] + p - 1;
                    bool in = true;
                    if (st.desc.periodic[d])
                        v = (v % st.nc[d] + st.nc[d]) % st.nc[d];
                    else if (v < 0 || v >= st.nc[d])
                        in = false;
                    cv[d][p] = v;
                    ok[d][p] = in;
                    own[d][p] = v >= bi.o[d] && v < bi.o[d] + e;
                }
                // a periodic axis shorter than the shell maps two shell cells onto one
                wraps |= st.desc.periodic[d] && st.nc[d] < bi.sh[d];
            }
            seen.clear();
            int32_t *shl = h_shell.data() + bi.shell_off;
            for (int32_t p0 = 0; p0 < bi.sh[0]; ++p0)
                for (int32_t p1 = 0; p1 < bi.sh[1]; ++p1)
                    for (int32_t p2 = 0; p2 < bi.sh[2]; ++p2) {
                        int32_t &out = shl[(p0 * bi.sh[1] + p1) * bi.sh[2] + p2];
                        if (!(ok[0][p0] && ok[1][p1] && ok[2][p2])) {
                            out = -2;
                            continue;
                        }
                        if (own[0][p0] && own[1][p1] && own[2][p2]) {
                            out = -1;
                            continue;
                        }
                        const int32_t cell = (cv[0][p0] * st.nc[1] + cv[1][p1]) * st.nc[2] + cv[2][p2];
                        if (wraps) {   // the cell may already be in this brick's halo
                            int32_t hit = -1;
                            for (size_t k = 0; k < seen.size(); k += 2)
                                if (seen[k] == cell) {
                                    hit = seen[k + 1];
                                    break;
                                }
                            if (hit >= 0) {
                                out = hit;
                                continue;
                            }
                            seen.push_back(cell);
                            seen.push_back(bi.n_halo);
                        }
                        const int32_t rk = rank_of(L, st.nc, cv[0][p0], cv[1][p1], cv[2][p2]);
                        HaloCell h;
                        h.brick = gb;
                        h.start_index = (int32_t)(cstart_off[s] + rk);
                        h.offset = bi.n_halo;
                        h.pos_base = (int32_t)st.caller_off;
                        part[t].push_back(h);
                        out = bi.n_halo;
                        bi.n_halo += start[rk + 1] - start[rk];
                    }
        }
    };
    if (n_thr == 1) {
        tables(0);
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < n_thr; ++t) pool.emplace_back(tables, t);
        for (auto &th : pool) th.join();
    }
    size_t n_cells_halo = 0;
    for (const auto &v : part) n_cells_halo += v.size();
    h_halo.reserve(n_cells_halo);
    for (const auto &v : part) h_halo.insert(h_halo.end(), v.begin(), v.end());
    // every list starts on a 16-byte boundary and is padded to whole quads (the
    // padding repeats the list's last entry), so the brick kernels stage it four
    // slots at a time; the tile holds the padded list
    for (BrickInfo &bi : hb) {   // empty bricks keep n_halo = 0 and the running offset
        bi.halo_off = (int32_t)std::min<int64_t>(halo_total, INT32_MAX);
        halo_total += halo_padded(bi.n_halo);
        if (bi.n_own > 0) tile_max = std::max(tile_max, bi.n_own_pad + halo_padded(bi.n_halo));
    }
    if (tile_max > kTileCapFloats) {
        *tile_overflow = true;
        return L2T_OK;
    }
    if (halo_total > INT32_MAX) return fail(c, L2T_ENOMEM, "halo lists too large");
    int rc = alloc_internal(c, slot, nbricks, (int32_t)h_list.size(), (int64_t)h_shell.size(),
                            halo_total);
    if (rc != L2T_OK) return rc;
    c->tile_max = tile_max;
    L2T_HIP(c, hipMemcpyAsync(c->bricks, hb.data(), sizeof(BrickInfo) * hb.size(),
                              hipMemcpyHostToDevice, st_));
    if (!h_list.empty())
        L2T_HIP(c, hipMemcpyAsync(c->brick_list, h_list.data(), sizeof(int32_t) * h_list.size(),
                                  hipMemcpyHostToDevice, st_));
    if (!h_shell.empty())
        L2T_HIP(c, hipMemcpyAsync(c->shell, h_shell.data(), sizeof(int32_t) * h_shell.size(),
                                  hipMemcpyHostToDevice, st_));
    int32_t *d_atom0 = tmp_of<int32_t>(c, 5, nbricks);
    HaloCell *d_halo = tmp_of<HaloCell>(c, 6, (int64_t)h_halo.size());
    if (!d_atom0 || !d_halo) return fail(c, L2T_ENOMEM, "brick table allocation failed");
    L2T_HIP(c, hipMemcpyAsync(d_atom0, h_atom0.data(), sizeof(int32_t) * nbricks,
                              hipMemcpyHostToDevice, st_));
    if (!h_halo.empty())
        L2T_HIP(c, hipMemcpyAsync(d_halo, h_halo.data(), sizeof(HaloCell) * h_halo.size(),
                                  hipMemcpyHostToDevice, st_));
    // ---- slots, counts (device) ----------------------------------------------------
    const double rc2 = r_cut * r_cut;
    const int64_t NI = c->n_int;
    double *qx = c->pos_int, *qy = c->pos_int + NI, *qz = c->pos_int + 2 * NI;
    // wrapped positions in cell order (all systems, caller offsets)
    double *cpos = tmp_of<double>(c, 12, 3 * c->n_tot);
    if (!cpos) return fail(c, L2T_ENOMEM, "neighbour build scratch allocation failed");
    double *csx = cpos, *csy = cpos + c->n_tot, *csz = cpos + 2 * c->n_tot;
    // one search pass (wave per cell, rows into a temporary table) when no cell
    // holds more atoms than a wave has lanes; else the thread-per-atom count and fill
    int32_t occ_max = 0;
    for (int s = 0; s < S; ++s) {
        const int32_t *start = h_start.data() + cstart_off[s];
        for (int64_t r = 0; r < c->sys[s].ncell; ++r)
            occ_max = std::max(occ_max, start[r + 1] - start[r]);
    }
    const bool rows_path = occ_max > 0 && occ_max <= kWave;
    // temporary row width: the widest row of the previous build plus a margin
    const int32_t wcap =
        c->max_nbrs > 0 ? std::min<int32_t>(96, (c->max_nbrs + 8 + 7) / 8 * 8) : 48;
    int32_t *tq = nullptr, *kof = nullptr;
    int16_t *th = nullptr;
    if (rows_path) {
        tq = tmp_of<int32_t>(c, 13, c->n_tot * (int64_t)wcap);
        th = tmp_of<int16_t>(c, 14, c->n_tot * (int64_t)wcap);
        kof = tmp_of<int32_t>(c, 15, c->n_int + 1);   // + the overflow flag
        if (!tq || !th || !kof)
            return fail(c, L2T_ENOMEM, "neighbour build scratch allocation failed");
        L2T_HIP(c, hipMemsetAsync(kof + c->n_int, 0, sizeof(int32_t), st_));
    }
    unsigned *row_overflow = rows_path ? reinterpret_cast<unsigned *>(kof + c->n_int) : nullptr;
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        const int32_t n = st.desc.n_atoms;
        const double *px = c->pos + st.caller_off, *py = px + c->n_tot, *pz = py + c->n_tot;
        const int64_t ro = lay[s].rank_off;
        hipLaunchKernelGGL(k_init_slots, dim3(nblk(st.n_pad, 256)), dim3(256), 0, st_,
                           st.atom_off, st.n_pad, c->perm, c->cell_int, qx, qy, qz, c->cnt);
        hipLaunchKernelGGL(k_assign, dim3(nblk(n, 256)), dim3(256), 0, st_,
                           c->sorted_local + st.caller_off, n, st.atom_off, st.caller_off, px, py,
                           pz, c->cell_of + st.caller_off, d_brick + ro, c->bricks, d_atom0,
                           grids[s], c->perm, c->inv, c->cell_int, c->pos_slot + st.caller_off,
                           qx, qy, qz, csx + st.caller_off, csy + st.caller_off,
                           csz + st.caller_off);
        if (rows_path) {
            const int wpb = 4;
            hipLaunchKernelGGL(k_cell_rows, dim3(nblk(st.ncell, wpb)), dim3(wpb * kWave), 0, st_,
                               (int32_t)st.ncell,
                               st.caller_off, c->pos_slot, csx + st.caller_off,
                               csy + st.caller_off, csz + st.caller_off,
                               d_start + cstart_off[s], d_rank + ro, d_cell + ro, d_brick + ro,
                               c->bricks, c->shell, grids[s], rc2, wcap, c->cnt, tq, th,
                               row_overflow);
        } else {
            hipLaunchKernelGGL(k_neighbors<false>, dim3(nblk(n, 128)), dim3(128), 0, st_, n,
                               c->pos_slot + st.caller_off, csx + st.caller_off,
                               csy + st.caller_off, csz + st.caller_off, c->cell_int,
                               d_start + cstart_off[s], d_rank + ro, d_cell + ro,
                               d_brick + ro, c->bricks, c->shell, grids[s], rc2, c->cnt, nullptr,
                               nullptr, nullptr);
        }
    }
    L2T_HIP(c, hipGetLastError());
    // ---- count order inside every brick --------------------------------------------
    int32_t own_max_all = 0;
    for (int32_t gb : h_list) own_max_all = std::max(own_max_all, hb[gb].n_own);
    if (c->n_brick_list > 0 && own_max_all <= 12288) {   // counts staged in 48 KB of LDS
        const int64_t NIi = c->n_int;
        int32_t *to = tmp_of<int32_t>(c, 7, NIi);
        int32_t *ti = tmp_of<int32_t>(c, 8, 3 * NIi);
        double *td = tmp_of<double>(c, 9, 3 * NIi);
        if (!to || !ti || !td)
            return fail(c, L2T_ENOMEM, "neighbour build scratch allocation failed");
        int32_t own_max = 0;
        for (int32_t gb : h_list) own_max = std::max(own_max, hb[gb].n_own);
        const dim3 gi(nblk(NIi, 256)), bi(256);
        hipLaunchKernelGGL(k_iota, gi, bi, 0, st_, to, c->n_int);
        hipLaunchKernelGGL(k_brick_rank, dim3(c->n_brick_list), dim3(256),
                           sizeof(int32_t) * (size_t)own_max, st_, c->bricks, c->brick_list,
                           c->cnt, to);
        L2T_HIP(c, hipMemcpyAsync(ti, c->perm, sizeof(int32_t) * NIi, hipMemcpyDeviceToDevice,
                                  st_));
        L2T_HIP(c, hipMemcpyAsync(ti + NIi, c->cell_int, sizeof(int32_t) * NIi,
                                  hipMemcpyDeviceToDevice, st_));
        L2T_HIP(c, hipMemcpyAsync(ti + 2 * NIi, c->cnt, sizeof(int32_t) * NIi,
                                  hipMemcpyDeviceToDevice, st_));
        L2T_HIP(c, hipMemcpyAsync(td, c->pos_int, sizeof(double) * 3 * NIi,
                                  hipMemcpyDeviceToDevice, st_));
        hipLaunchKernelGGL(k_scatter_i32, gi, bi, 0, st_, ti, to, c->n_int, c->perm);
        hipLaunchKernelGGL(k_scatter_i32, gi, bi, 0, st_, ti + NIi, to, c->n_int, c->cell_int);
        hipLaunchKernelGGL(k_scatter_i32, gi, bi, 0, st_, ti + 2 * NIi, to, c->n_int, c->cnt);
        for (int d = 0; d < 3; ++d)
            hipLaunchKernelGGL(k_scatter_f64, gi, bi, 0, st_, td + d * NIi, to, c->n_int,
                               c->pos_int + d * NIi);
        hipLaunchKernelGGL(k_inverse, gi, bi, 0, st_, c->perm, c->n_int, c->inv);
        hipLaunchKernelGGL(k_remap, dim3(nblk(c->n_tot, 256)), dim3(256), 0, st_, c->pos_slot,
                           c->n_tot, to);
        L2T_HIP(c, hipGetLastError());
        L2T_HIP(c, hipStreamSynchronize(st_));
    }
    // ---- slice widths -> column offsets (host scan) -------------------------------
    // slice widths and valid lanes, then (8-byte aligned) the count statistics
    const int64_t stat_at = (2 * (int64_t)c->n_slices + 1) / 2 * 2;
    int32_t *dw = tmp_of<int32_t>(c, 10, stat_at + 4);
    if (!dw) return fail(c, L2T_ENOMEM, "slice width allocation failed");
    hipLaunchKernelGGL(k_slice_width, dim3(nblk(c->n_slices, 256)), dim3(256), 0, st_, c->cnt,
                       c->perm, c->n_slices, dw, dw + c->n_slices);
    L2T_HIP(c, hipGetLastError());
    std::vector<int32_t> hw(2 * (size_t)c->n_slices);
    if (!hw.empty())
        L2T_HIP(c, hipMemcpyAsync(hw.data(), dw, sizeof(int32_t) * hw.size(),
                                  hipMemcpyDeviceToHost, st_));
    unsigned h_overflow = 0;
    if (rows_path)
        L2T_HIP(c, hipMemcpyAsync(&h_overflow, row_overflow, sizeof(unsigned),
                                  hipMemcpyDeviceToHost, st_));
    L2T_HIP(c, hipStreamSynchronize(st_));
    std::vector<SliceInfo> hs(c->n_slices);
    int64_t total64 = 0, totalw64 = 0;
    for (int s = 0; s < S; ++s) {
        SystemState &st = c->sys[s];
        st.max_nbrs = 0;
        const SysLayout &L = lay[s];
        for (int32_t b = 0; b < L.nbrick; ++b) {
            const BrickInfo &bi = hb[L.brick0 + b];
            for (int32_t q = 0; q < bi.n_own_pad / kWave; ++q) {
                const int32_t sl = bi.slice0 + q;
                hs[sl].sys = s;
                hs[sl].brick = L.brick0 + b;
                hs[sl].width = hw[sl];
                hs[sl].n_valid = hw[c->n_slices + sl];
                if (total64 > INT32_MAX) return fail(c, L2T_ENOMEM, "neighbour table too large");
                hs[sl].col_base64 = (int32_t)total64;
                hs[sl].colw_base64 = (int32_t)totalw64;
                total64 += hw[sl];
                totalw64 += (hw[sl] + 1) / 2;
                st.max_nbrs = std::max(st.max_nbrs, hw[sl]);
            }
        }
    }
    int64_t col_len = std::max<int64_t>(total64 * kWave, 1);
    if (col_len > c->col_len) {
        dev_free(c, c->col);
        c->col = nullptr;
        c->col_len = 0;
        if (dev_malloc(c, (void **)&c->col, sizeof(int32_t) * col_len) != hipSuccess)
            return fail(c, L2T_ENOMEM, "neighbour table allocation failed");
        c->col_len = col_len;
    }
    int64_t colw_len = std::max<int64_t>(totalw64 * kWave, 1);
    if (colw_len > c->colw_len) {
        dev_free(c, c->colw);
        c->colw = nullptr;
        c->colw_len = 0;
        if (dev_malloc(c, (void **)&c->colw, sizeof(uint32_t) * colw_len) != hipSuccess)
            return fail(c, L2T_ENOMEM, "neighbour table allocation failed");
        c->colw_len = colw_len;
    }
    c->col_used = total64 * kWave;
    if (!hs.empty())
        L2T_HIP(c, hipMemcpyAsync(c->slices, hs.data(), sizeof(SliceInfo) * hs.size(),
                                  hipMemcpyHostToDevice, st_));
    // ---- tables and halo lists (device) ----------------------------------------------
    if (rows_path && h_overflow == 0) {
        hipLaunchKernelGGL(k_cell_index, dim3(nblk(c->n_tot, 256)), dim3(256), 0, st_,
                           c->pos_slot, c->n_tot, kof);
        hipLaunchKernelGGL(k_rows_fill, dim3(nblk(c->n_int, 256)), dim3(256), 0, st_, c->n_int,
                           c->perm, kof, c->cnt, c->slices, c->bricks, c->pos_slot, tq, th, wcap,
                           c->col, (uint16_t *)c->colw);
    } else {
        for (int s = 0; s < S; ++s) {
            SystemState &st = c->sys[s];
            const int32_t n = st.desc.n_atoms;
            const int64_t ro = lay[s].rank_off;
            hipLaunchKernelGGL(k_neighbors<true>, dim3(nblk(n, 128)), dim3(128), 0, st_, n,
                               c->pos_slot + st.caller_off, csx + st.caller_off,
                               csy + st.caller_off, csz + st.caller_off, c->cell_int,
                               d_start + cstart_off[s], d_rank + ro, d_cell + ro,
                               d_brick + ro, c->bricks, c->shell, grids[s], rc2, c->cnt,
                               c->slices, c->col, (uint16_t *)c->colw);
        }
    }
    hipLaunchKernelGGL(k_pad_rows, dim3(nblk(c->n_int, 256)), dim3(256), 0, st_, c->perm,
                       c->slices, c->bricks, c->n_int, c->col, (uint16_t *)c->colw);
    if (!h_halo.empty())
        hipLaunchKernelGGL(k_halo_expand, dim3(nblk((int64_t)h_halo.size(), 256)), dim3(256), 0,
                           st_, d_halo, (int64_t)h_halo.size(), c->bricks, d_start,
                           c->pos_slot, c->halo);
    if (!h_halo.empty())
        hipLaunchKernelGGL(k_halo_pad, dim3(nblk(nbricks, 256)), dim3(256), 0, st_, c->bricks,
                           nbricks, c->halo);
    L2T_HIP(c, hipGetLastError());
    // ---- statistics ----------------------------------------------------------------------
    unsigned long long *dsum = reinterpret_cast<unsigned long long *>(dw + stat_at);
    int32_t *dmax = dw + stat_at + 2;
    L2T_HIP(c, hipMemsetAsync(dw + stat_at, 0, 4 * sizeof(int32_t), st_));
    hipLaunchKernelGGL(k_count_stats, dim3(std::max<unsigned>(1, std::min<unsigned>(1024, nblk(c->n_int, 256)))),
                       dim3(256), 0, st_, c->cnt, (int64_t)c->n_int, dsum, dmax);
    L2T_HIP(c, hipGetLastError());
    std::vector<int32_t> h_work(h_list.size());
    if (!h_list.empty()) {
        int32_t *d_work = tmp_of<int32_t>(c, 16, (int64_t)h_list.size());
        if (!d_work) return fail(c, L2T_ENOMEM, "brick work allocation failed");
        hipLaunchKernelGGL(k_brick_work, dim3(nblk((int64_t)h_list.size(), 256)), dim3(256), 0,
                           st_, c->bricks, c->brick_list, (int32_t)h_list.size(), c->slices,
                           d_work);
        L2T_HIP(c, hipMemcpyAsync(h_work.data(), d_work, sizeof(int32_t) * h_list.size(),
                                  hipMemcpyDeviceToHost, st_));
    }
    int32_t hstat[4] = {0, 0, 0, 0};
    L2T_HIP(c, hipMemcpyAsync(hstat, dw + stat_at, sizeof hstat, hipMemcpyDeviceToHost, st_));
    L2T_HIP(c, hipStreamSynchronize(st_));
    if (!h_list.empty()) {
        const int xrc = xcd_split(c, h_list, h_work);
        if (xrc != L2T_OK) return xrc;
    } else {
        c->n_xcd_list = 0;
    }
    unsigned long long usum = 0;
    std::memcpy(&usum, hstat, sizeof usum);
    const int64_t sum = (int64_t)usum;
    const int32_t mx = hstat[2];
    c->max_nbrs = mx;
    c->mean_nbrs = c->n_tot > 0 ? (double)sum / (double)c->n_tot : 0.0;
    c->mean_width = c->n_tot > 0 ? (double)total64 * kWave / (double)c->n_tot : 0.0;
    c->r_cut = r_cut;
    return L2T_OK;
}

namespace {

// one layout at brick edge `force` (0: the edge model's choice)
int build_layout(l2t_ctx *c, double r_cut, int32_t force) {
    int32_t limit = force > 0 ? force : kMaxBrickEdge;
    c->brick_edge_used = 0;
    for (int attempt = 0; attempt < 12; ++attempt) {
        bool overflow = false;
        int rc = build_neighbors_once(c, r_cut, limit, force > 0, &overflow);
        if (rc != L2T_OK) return rc;
        if (!overflow) return L2T_OK;
        // a tile overflowed its LDS cap: retry below the edge that was used
        const int32_t used = c->brick_edge_used;
        c->brick_edge_used = 0;
        if (used <= 1) break;
        limit = used / 2;
    }
    return fail(c, L2T_EINVAL, "atom density too high for the LDS tile of one cell and its halo");
}

// measured brick edges, per problem shape (cut-off and every system's atom
// count, box and boundaries), for the life of the process; contexts on
// different host threads share it under a lock
std::mutex &edge_mutex() {
    static std::mutex m;
    return m;
}
// the measured brick edge and sweep order (1 fixed, 2 alternating) of a shape
// what the build measured for a problem shape: brick edge, sweep order and
// table-load policy
struct LayoutChoice {
    int32_t edge = 0;
    int sweep = 1, table = 1;
};
std::map<std::string, LayoutChoice> &edge_cache() {
    static std::map<std::string, LayoutChoice> m;
    return m;
}
bool edge_lookup(const std::string &key, LayoutChoice *out) {
    std::lock_guard<std::mutex> g(edge_mutex());
    auto it = edge_cache().find(key);
    if (it == edge_cache().end()) return false;
    *out = it->second;
    return true;
}
void edge_store(const std::string &key, const LayoutChoice &ch) {
    std::lock_guard<std::mutex> g(edge_mutex());
    edge_cache()[key] = ch;
}

std::string edge_key(const l2t_ctx *c, double r_cut) {
    std::string k;
    char buf[192];
    std::snprintf(buf, sizeof buf, "rc=%a cu=%d", r_cut, c->n_cu);
    k += buf;
    for (const SystemState &st : c->sys) {
        std::snprintf(buf, sizeof buf, "|%d %a %a %a %d%d%d", st.desc.n_atoms, st.desc.box_len[0],
                      st.desc.box_len[1], st.desc.box_len[2], st.desc.periodic[0],
                      st.desc.periodic[1], st.desc.periodic[2]);
        k += buf;
    }
    return k;
}

}  // namespace

// The brick edge of an FP32C context with at least as many bricks as the GPU
// has CUs is measured, not only modelled: the model's edge and its two
// neighbours are built and each runs a short probe of the brick kernel
// (brick_probe), and a neighbour replaces the model's edge when it is more
// than 1 % faster; on the chosen layout the sweep order (L2T_OPT_SWEEP) and
// the table-load policy (L2T_OPT_TABLE_STREAM) are timed the same way.  The
// choices are kept per problem shape, so later builds of the same shape build
// once.  Smaller layouts, FP64 contexts, a pinned edge or launch form and a
// disabled autotuner keep the model's edge, the fixed order and cached loads.
int build_neighbors(l2t_ctx *c, double r_cut) {
    Tuning &t = c->tune;
    // an explicit sweep order or table policy applies as set; otherwise the
    // fixed order and cached table loads unless the others measure faster below
    t.sweep_used = t.sweep == 2 ? 2 : 1;
    t.table_used = t.table == 2 ? 2 : 1;
    const bool may_tune = c->precision == L2T_FP32C && t.autotune && !t.pinned &&
                          t.brick_edge == 0;
    const std::string key = may_tune ? edge_key(c, r_cut) : std::string();
    LayoutChoice cached;
    if (may_tune && edge_lookup(key, &cached)) {
        const int rc = build_layout(c, r_cut, cached.edge);
        if (rc == L2T_OK && t.sweep == 0) t.sweep_used = cached.sweep;
        if (rc == L2T_OK && t.table == 0) t.table_used = cached.table;
        return rc;
    }
    int rc = build_layout(c, r_cut, 0);
    if (rc != L2T_OK || !may_tune) return rc;
    const int32_t e0 = c->brick_edge_used;
    if (c->n_brick_list < std::max(1, c->n_cu)) {
        edge_store(key, LayoutChoice{e0, 1, 1});
        return L2T_OK;
    }
    // an edge above e0 changes the layout only where some axis is longer than e0
    bool grows = false;
    for (const SystemState &st : c->sys)
        for (int d = 0; d < 3; ++d) grows |= st.nc[d] > e0;
    constexpr int32_t kProbe = 12;
    float best_ms = 0.0f;
    rc = brick_probe(c, kProbe, false, false, &best_ms);
    if (rc == L2T_ENOMEM) {
        // no room for the stand-in state: keep the model's edge
        c->last_error.clear();
        edge_store(key, LayoutChoice{e0, 1, 1});
        return L2T_OK;
    }
    if (rc != L2T_OK) return rc;
    int32_t best = e0, built = e0;
    for (const int32_t e : {e0 - 1, e0 + 1}) {
        if (e < 1 || (e > e0 && !grows)) continue;
        rc = build_layout(c, r_cut, e);
        if (rc != L2T_OK) return rc;
        built = c->brick_edge_used;
        if (built != e) continue;   // its tiles overflowed: a smaller edge was built
        float ms = 0.0f;
        rc = brick_probe(c, kProbe, false, false, &ms);
        if (rc == L2T_ENOMEM) {   // a larger layout's stand-in did not fit: skip it
            c->last_error.clear();
            continue;
        }
        if (rc != L2T_OK) return rc;
        if (ms < 0.99f * best_ms) {
            best_ms = ms;
            best = e;
        }
    }
    if (built != best) {
        rc = build_layout(c, r_cut, best);
        if (rc != L2T_OK) return rc;
    }
    // on the chosen layout, the sweep order and then the table policy: the
    // alternating order and the non-temporal table loads each replace the
    // default when they are more than 1 % faster
    LayoutChoice ch{best, 1, 1};
    bool alt = t.sweep == 2;
    if (t.sweep == 0) {
        float fixed_ms = 0.0f, alt_ms = 0.0f;
        rc = brick_probe(c, kProbe, false, t.table == 2, &fixed_ms);
        if (rc == L2T_OK) rc = brick_probe(c, kProbe, true, t.table == 2, &alt_ms);
        if (rc == L2T_ENOMEM) {
            c->last_error.clear();
        } else if (rc != L2T_OK) {
            return rc;
        } else if (alt_ms < 0.99f * fixed_ms) {
            ch.sweep = 2;
            alt = true;
        }
        t.sweep_used = ch.sweep;
    }
    if (t.table == 0) {
        float cached_ms = 0.0f, stream_ms = 0.0f;
        rc = brick_probe(c, kProbe, alt, false, &cached_ms);
        if (rc == L2T_OK) rc = brick_probe(c, kProbe, alt, true, &stream_ms);
        if (rc == L2T_ENOMEM) {
            c->last_error.clear();
        } else if (rc != L2T_OK) {
            return rc;
        } else if (stream_ms < 0.99f * cached_ms) {
            ch.table = 2;
        }
        t.table_used = ch.table;
    }
    edge_store(key, ch);
    return L2T_OK;
}

int permute_in(l2t_ctx *c, int32_t sys, const double *src_dev, int32_t field) {
    const SystemState &st = c->sys[sys];
    hipLaunchKernelGGL(k_field_in, dim3(nblk(st.n_pad, 256)), dim3(256), 0, c->stream, st.atom_off,
                       st.n_pad, c->perm, st.caller_off, src_dev, field, c->precision,
                       c->T64[c->cur], c->Thi[c->cur], c->Tlo, c->Tl64, c->Tl32, c->srcw64,
                       c->srcw32);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int mark_held_slices(l2t_ctx *c, int32_t sys) {
    const SystemState &st = c->sys[sys];
    hipLaunchKernelGGL(k_slice_held, dim3(nblk(st.n_slices, 4)), dim3(256), 0, c->stream, c->slices,
                       st.slice0, st.n_slices, c->precision, c->srcw64, c->srcw32);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int permute_out(l2t_ctx *c, int32_t sys, int32_t field, double *dst_dev) {
    const SystemState &st = c->sys[sys];
    hipLaunchKernelGGL(k_field_out, dim3(nblk(st.n_pad, 256)), dim3(256), 0, c->stream,
                       st.atom_off, st.n_pad, c->perm, st.caller_off, field, c->precision,
                       c->T64[c->cur], c->Thi[c->cur], c->Tlo, c->Tl64, c->Tl32, c->cnt, c->eatom,
                       c->srcw64, c->srcw32, dst_dev);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int check_field_range(l2t_ctx *c, const double *src_dev, int64_t n, double lo, double hi,
                      bool *ok) {
    unsigned *bad = c->derr + 1;
    L2T_HIP(c, hipMemsetAsync(bad, 0, sizeof(unsigned), c->stream));
    hipLaunchKernelGGL(k_range_count, dim3(nblk(n, 256)), dim3(256), 0, c->stream, src_dev, n, lo,
                       hi, bad);
    unsigned h = 0;
    L2T_HIP(c, hipMemcpyAsync(&h, bad, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    *ok = (h == 0);
    return L2T_OK;
}

namespace {

// Eq. 4 for system sys with the velocities and masses gathered into internal
// order in vm ([4][n_pad] doubles followed by the 4 doubles of the system's
// momentum and mass); synchronises.
int lattice_temperature_into(l2t_ctx *c, int32_t sys, const double *v_dev, const double *m_dev,
                             int32_t global_com, double *vm) {
    const SystemState &st = c->sys[sys];
    double *gm = vm + 4 * (size_t)st.n_pad;
    hipLaunchKernelGGL(k_gather_vm, dim3(nblk(st.n_pad, 256)), dim3(256), 0, c->stream,
                       st.atom_off, st.n_pad, c->perm, st.caller_off, st.desc.n_atoms, v_dev, m_dev,
                       vm);
    if (global_com)
        hipLaunchKernelGGL(k_momentum, dim3(1), dim3(256), 0, c->stream, vm, st.n_pad, gm);
    hipLaunchKernelGGL(k_lattice_temp, dim3(nblk(st.n_pad, 128)), dim3(128), 0, c->stream,
                       st.atom_off, st.n_pad, c->perm, c->slices, c->col, vm, gm, global_com,
                       st.params.ke_eps, c->precision, c->Tl64, c->Tl32);
    L2T_HIP(c, hipGetLastError());
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    return L2T_OK;
}

// Staging of the allocation-free Eq. 4 entry point: one array per GPU, held
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it names a stand-in, not device memory); it passes the
// device address hipGetSymbolAddress returned for the current device.
constexpr size_t kStaticScratchDoubles = kStaticScratchBytes / sizeof(double);
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
double *g_static_ptr[kMaxDevices] = {};
hipError_t g_static_err[kMaxDevices] = {};
bool g_static_done[kMaxDevices] = {};

}  // namespace

int lattice_temperature(l2t_ctx *c, int32_t sys, const double *v_dev, const double *m_dev,
                        int32_t global_com) {
    const SystemState &st = c->sys[sys];
    size_t need = sizeof(double) * (4 * (size_t)st.n_pad + 4);
    if (ensure_scratch(c, need) != L2T_OK) return L2T_ENOMEM;
    return lattice_temperature_into(c, sys, v_dev, m_dev, global_com, (double *)c->scratch);
}

int static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return L2T_EINVAL;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_done[device]) {
        // called with `device` current (l2t_create), once per device
        void *p = nullptr;
        g_static_err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_static_ptr[device] = g_static_err[device] == hipSuccess ? (double *)p : nullptr;
        g_static_done[device] = true;
    }
    return g_static_ptr[device] ? L2T_OK : L2T_EHIP;
}

int lattice_temperature_static(l2t_ctx *c, int32_t sys, const double *v_dev, const double *m_dev,
                               int32_t global_com) {
    const SystemState &st = c->sys[sys];
    if (4 * (size_t)st.n_pad + 4 > kStaticScratchDoubles)
        return fail(c, L2T_EINVAL, "system larger than the static staging array");
    double *vm = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (c->device >= 0 && c->device < kMaxDevices) vm = g_static_ptr[c->device];
    }
    if (!vm) return fail(c, L2T_EHIP, "no device address for the static staging array");
    return lattice_temperature_into(c, sys, v_dev, m_dev, global_com, vm);
}

int source_weights(l2t_ctx *c, int32_t sys) {
    const SystemState &st = c->sys[sys];
    if (!st.params.laser_on) return L2T_OK;
    hipLaunchKernelGGL(k_source_weights, dim3(nblk(st.n_pad, 256)), dim3(256), 0, c->stream,
                       st.atom_off, st.n_pad, c->perm, c->pos_int, st.params.laser_x0,
                       st.params.laser_lp, c->precision == L2T_FP64 ? c->srcw64 : nullptr,
                       c->precision == L2T_FP32C ? c->srcw32 : nullptr);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int neighbors_to_host(l2t_ctx *c, int32_t sys, int64_t *row_ptr, int32_t *col, int64_t cap) {
    const SystemState &st = c->sys[sys];
    const int32_t n = st.desc.n_atoms;
    std::vector<SliceInfo> hs(st.n_slices);
    std::vector<int32_t> perm(st.n_pad), cnt(st.n_pad), inv(n);
    L2T_HIP(c, hipMemcpyAsync(hs.data(), c->slices + st.slice0, sizeof(SliceInfo) * hs.size(),
                              hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipMemcpyAsync(perm.data(), c->perm + st.atom_off, sizeof(int32_t) * st.n_pad,
                              hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipMemcpyAsync(cnt.data(), c->cnt + st.atom_off, sizeof(int32_t) * st.n_pad,
                              hipMemcpyDeviceToHost, c->stream));
    int64_t c0 = (int64_t)hs.empty() ? 0 : (int64_t)hs[0].col_base64 * kWave;
    int64_t c1 = c0;
    for (const SliceInfo &si : hs) c1 = std::max<int64_t>(c1, ((int64_t)si.col_base64 + si.width) * kWave);
    std::vector<int32_t> hcol(std::max<int64_t>(c1 - c0, 1));
    if (c1 > c0)
        L2T_HIP(c, hipMemcpyAsync(hcol.data(), c->col + c0, sizeof(int32_t) * (c1 - c0),
                                  hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    // row lengths in caller order
    for (int32_t k = 0; k < st.n_pad; ++k)
        if (perm[k] >= 0) inv[perm[k] - st.caller_off] = k;
    row_ptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[inv[i]];
    if (!col) return L2T_OK;
    if (row_ptr[n] > cap) return fail(c, L2T_EINVAL, "col capacity below the neighbour count");
    for (int32_t i = 0; i < n; ++i) {
        int32_t k = inv[i];
        const SliceInfo &si = hs[k / kWave];
        int64_t base = (int64_t)si.col_base64 * kWave - c0 + (k % kWave);
        int32_t *dst = col + row_ptr[i];
        for (int32_t q = 0; q < cnt[k]; ++q) {
            int32_t j = hcol[base + (int64_t)q * kWave];
            dst[q] = (int32_t)(perm[j - st.atom_off] - st.caller_off);
        }
        std::sort(dst, dst + cnt[k]);
    }
    return L2T_OK;
}

}  // namespace l2t
