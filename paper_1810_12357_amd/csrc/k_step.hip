// Sub-step kernels of the master equation (Eq. 2) with electron-phonon
// coupling and the laser source (Eq. 10), forward Euler (Section 2.1), plus the
// per-system FP64 energy / ledger reductions.
//
// Layout: one wavefront owns one slice of 64 consecutive cell-sorted atoms;
// lane l of the wave owns atom 64*slice + l.  Neighbour indices of a slice are
// column-major (entry k of all 64 lanes is one coalesced 256-byte read) and
// short rows are padded with the atom's own index, whose pair term is zero.
//
//  * FP64 plain: literal two-exponential pair term, one launch per sub-step.
//  * FP32C: cancellation-free product form of the pair term evaluated in
//    FP32 from the hi part of the neighbour temperatures, per-atom sum of the
//    terms in FP64 (one conversion and one FP64 add per term, two vector
//    instructions where a Kahan step takes four), state kept as the FP32 hi
//    that neighbours read and a 16-bit low part (state_fp32c.h) whose sum with
//    the increment is formed in FP64 and split again; ledgers in FP64.  One launch per sub-step (global gathers or LDS brick tiles), or
//    a persistent launch that runs all sub-steps with a grid barrier between
//    them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "l2t_internal.h"
#include "step_device.h"

namespace l2t {
namespace {

using namespace dev;

// ---- kernels ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_step_fp64(const SliceInfo *slices, int32_t slice0,
                                                   int32_t n_slices, const int32_t *col,
                                                   const double *T, double *Tn, const double *Tl,
                                                   double *Tl_out, const double *srcw,
                                                   const DevParams *P,
                                                   const int64_t *dstep, int32_t rel,
                                                   double *ledger, double *eatom, unsigned *err) {
    // the wave index is uniform: slice record, row width and loop bounds sit in
    // scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int32_t q = blockIdx.x * (blockDim.x / kWave) + wave;
    if (q >= n_slices) return;
    const int32_t sl = slice0 + q;
    const SliceInfo si = slices[sl];
    const DevParams &p = P[si.sys];
    slice_step_fp64(si, sl, lane, p, col, T, Tn, Tl, Tl_out, srcw, dstep[si.sys] + rel, ledger,
                    eatom, err);
}

__global__ __launch_bounds__(256) void k_step_fp32c(const SliceInfo *slices, int32_t slice0,
                                                    int32_t n_slices, const int32_t *col,
                                                    const float *Thi, float *Thi_n, int16_t *Tlo,
                                                    const float *Tl, const float *srcw,
                                                    const DevParams *P, const int64_t *dstep,
                                                    int32_t rel, double *ledger, double *eatom,
                                                    unsigned *err) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t q = blockIdx.x * (blockDim.x / kWave) + wave;
    if (q >= n_slices) return;
    const int32_t sl = slice0 + q;
    const SliceInfo si = slices[sl];
    const DevParams &p = P[si.sys];
    slice_step_fp32c(si, sl, lane, p, col, Thi, Thi_n, Tlo, Tl, srcw, dstep[si.sys] + rel, ledger,
                     eatom, err);
}

// LDS-tile FP32C sub-step: one workgroup per brick stages the FP32 hi
// temperatures of the brick's own slots and of its halo atoms in LDS, then its
// waves run the brick's slices reading neighbours from the tile through the
// uint16 table.  Workgroup b runs on XCD b mod 8 and takes entry
// (b mod 8) * (G/8) + b/8 of the launch list: with the XCD launch list each
// XCD sweeps one contiguous range of bricks (its L2 serves the halo loads),
// the ranges carry equal estimated work, and entries past a range are holes
// (-1) whose workgroups return at once.
// LO_IN: read the low part from lo_in and write the new one to Tlo (two
// buffers, as the adjoint's recomputation keeps every state of a segment);
// otherwise the low part is updated in place and lo_in is unused.  POLICY:
// cache policy of the table loads (kTableCached, kTableStream).
template <bool LO_IN, int POLICY>
__global__ __launch_bounds__(kBrickBlockMax) __attribute__((amdgpu_waves_per_eu(8))) void k_brick_fp32c(
    const BrickInfo *__restrict__ bricks, const int32_t *__restrict__ list, int32_t n_list,
    const SliceInfo *__restrict__ slices, const uint32_t *__restrict__ colw,
    const int32_t *__restrict__ halo, const float *__restrict__ Thi, float *__restrict__ Thi_n,
    const int16_t *__restrict__ lo_in, int16_t *__restrict__ Tlo, const float *__restrict__ Tl,
    const float *__restrict__ srcw, const DevParams *__restrict__ P,
    const int64_t *__restrict__ dstep, int32_t rel, double *__restrict__ ledger,
    double *__restrict__ eatom, unsigned *__restrict__ err) {
    extern __shared__ __align__(16) float tile[];
    __shared__ float wlo[kBrickBlockMax / kWave], whi[kBrickBlockMax / kWave];
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned logical = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    if ((int32_t)logical >= n_list) return;
    const int32_t gb = list[logical];
    if (gb < 0) return;   // a hole of the XCD launch list
    const BrickInfo bi = bricks[gb];
    // stage the tile four slots at a time, keeping the range of the staged
    // temperatures (padding slots aside): the brick's own slots are contiguous
    // and 64-aligned (real atoms first), and its halo list is 16-byte aligned
    // and padded to a multiple of 4 with copies of its last entry, which leave
    // the range unchanged.  Two quads per thread and pass keep 8 loads in
    // flight; the second is clamped to the last quad, so a thread past the end
    // stages that quad again (the same values to the same place).
    const int32_t B = blockDim.x;
    const char *tb_in = reinterpret_cast<const char *>(Thi);
    auto hi_at = [&](int32_t slot) {   // 32-bit unsigned byte offset: one address op
        return *reinterpret_cast<const float *>(tb_in + (uint32_t)slot * 4u);
    };
    float tmin = INFINITY, tmax = -INFINITY;
    auto range4 = [&](const float4 &v) {
        tmin = fminf(tmin, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
        tmax = fmaxf(tmax, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
    };
    auto range_own = [&](float4 v, int32_t q) {
        const int32_t i = 4 * q;
        if (i + 4 > bi.n_own) {      // the quad of the last real slot, or padding only
            if (i >= bi.n_own) return;
            if (i + 1 >= bi.n_own) v.y = v.x;
            if (i + 2 >= bi.n_own) v.z = v.x;
            v.w = v.x;
        }
        range4(v);
    };
    {
        const int32_t nq = bi.n_own_pad >> 2;
        const float4 *src = reinterpret_cast<const float4 *>(Thi + bi.slot0);
        float4 *dst = reinterpret_cast<float4 *>(tile);
        for (int32_t q0 = threadIdx.x; q0 < nq; q0 += 2 * B) {
            const int32_t q1 = min(q0 + B, nq - 1);
            const float4 a = src[q0];
            const float4 c = src[q1];
            dst[q0] = a;
            dst[q1] = c;
            range_own(a, q0);
            range_own(c, q1);
        }
        const int32_t nh = halo_padded(bi.n_halo) >> 2;
        const int4 *hl = reinterpret_cast<const int4 *>(halo + bi.halo_off);
        float4 *ht = reinterpret_cast<float4 *>(tile + bi.n_own_pad);
        for (int32_t q0 = threadIdx.x; q0 < nh; q0 += 2 * B) {
            const int32_t q1 = min(q0 + B, nh - 1);
            const int4 ia = hl[q0];
            const int4 ic = hl[q1];
            const float4 a = make_float4(hi_at(ia.x), hi_at(ia.y), hi_at(ia.z), hi_at(ia.w));
            const float4 c = make_float4(hi_at(ic.x), hi_at(ic.y), hi_at(ic.z), hi_at(ic.w));
            ht[q0] = a;
            ht[q1] = c;
            range4(a);
            range4(c);
        }
    }
    // wave index, slice records and row widths are wave-uniform (scalar registers)
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    tmin = wave_min_f32(tmin);
    tmax = wave_max_f32(tmax);
    if (lane == 0) {
        wlo[wave] = tmin;
        whi[wave] = tmax;
    }
    __syncthreads();
    const int32_t ns = bi.n_own_pad / kWave;
    if (wave >= ns) return;
    // every slice of a brick belongs to the brick's system
    const DevParams &p = P[bi.sys];
    const float qpulse = source_factor32(p, dstep[bi.sys] + rel);
    // every row of the brick pairs two staged temperatures, so the FP32
    // difference of any pair is at most the rounded span of the tile, and
    // its square at most the span's (rounding is monotone): a span whose
    // square lies within the lowest tier of the pair term puts every pair
    // of the brick on that tier
    float bmin = wlo[0], bmax = whi[0];
    for (int k = 1; k < nw; ++k) {
        bmin = fminf(bmin, wlo[k]);
        bmax = fmaxf(bmax, whi[k]);
    }
    const float span = bmax - bmin;
    const bool one_tier = __builtin_amdgcn_readfirstlane((int)(span * span <= p.f_w_tiny)) != 0;
    // ledger terms summed per lane over the wave's slices, reduced once per wave
    // into the row of the wave's first slice (all rows of a system are summed)
    LedgerTerms acc{0.0f, 0.0f, 0.0f};
    for (int32_t q = wave; q < ns; q += nw) {
        const int32_t sl = bi.slice0 + q;
        const int32_t w = __builtin_amdgcn_readfirstlane(slices[sl].width);
        const int32_t nv = __builtin_amdgcn_readfirstlane(slices[sl].n_valid);
        const int32_t base = __builtin_amdgcn_readfirstlane(slices[sl].colw_base64);
        const int32_t held = __builtin_amdgcn_readfirstlane(slices[sl].flags) & kSliceHeld;
        const int32_t slot = sl * kWave + lane;
        const int16_t lo = LO_IN ? lo_in[slot] : Tlo[slot];
        const float tl = Tl[slot];
        const float sw = (p.laser_on | held) ? srcw[slot] : 0.0f;
        const float Ti = tile[q * kWave + lane];
        const uint32_t *row = colw + (int64_t)base * kWave;
        const LedgerTerms t =
            one_tier ? slice_core_brick<false, POLICY>(w, slot, lane < nv, p, Ti, lo, tl, sw, row,
                                                       lane, tile, Thi_n, Tlo, eatom, qpulse, err)
                     : slice_core_brick<true, POLICY>(w, slot, lane < nv, p, Ti, lo, tl, sw, row,
                                                      lane, tile, Thi_n, Tlo, eatom, qpulse, err);
        acc.e2l += t.e2l;
        acc.src += t.src;
        acc.lt += t.lt;
    }
    ledger_add(ledger, bi.slice0 + wave, lane, acc, p.dt);
}

// the brick kernel with the table-load policy in effect (1 cached, 2 streamed)
template <bool LO_IN>
decltype(&k_brick_fp32c<LO_IN, kTableCached>) brick_kernel(int table) {
    return table == 2 ? &k_brick_fp32c<LO_IN, kTableStream> : &k_brick_fp32c<LO_IN, kTableCached>;
}

// LDS-tile FP64 sub-step (the plain form of Eq. 2 with the brick layout):
// one workgroup per brick stages the FP64 temperatures of the brick's own
// slots and of its halo atoms in LDS, then its waves run the brick's slices
// through the uint16 table, whose entries are byte offsets into a 4-byte
// tile (halved for this 8-byte one).  The rows hold the same neighbours in
// the same order as the int32 table and the per-lane arithmetic is the same
// template, so states and per-slice ledger rows are bitwise those of
// k_step_fp64.  Systems in the lattice mode are not launched here.
__global__ __launch_bounds__(kBrickBlockMax) void k_brick_fp64(
    const BrickInfo *__restrict__ bricks, const int32_t *__restrict__ list, int32_t n_list,
    const SliceInfo *__restrict__ slices, const uint32_t *__restrict__ colw,
    const int32_t *__restrict__ halo, const double *__restrict__ T, double *__restrict__ Tn,
    const double *__restrict__ Tl, const double *__restrict__ srcw,
    const DevParams *__restrict__ P, const int64_t *__restrict__ dstep, int32_t rel,
    double *__restrict__ ledger, double *__restrict__ eatom, unsigned *__restrict__ err) {
    extern __shared__ double tile64[];
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned logical = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    if ((int32_t)logical >= n_list) return;
    const int32_t gb = list[logical];
    if (gb < 0) return;   // a hole of the XCD launch list
    const BrickInfo bi = bricks[gb];
    constexpr int U = 4;
    const int32_t B = blockDim.x;
    for (int32_t t0 = threadIdx.x; t0 < bi.n_own_pad; t0 += U * B) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t t = t0 + u * B;
            v[u] = (t < bi.n_own_pad) ? T[bi.slot0 + t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + u * B < bi.n_own_pad) tile64[t0 + u * B] = v[u];
    }
    const int32_t *hl = halo + bi.halo_off;
    double *ht = tile64 + bi.n_own_pad;
    for (int32_t t0 = threadIdx.x; t0 < bi.n_halo; t0 += U * B) {
        int32_t id[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t t = t0 + u * B;
            id[u] = (t < bi.n_halo) ? hl[t] : bi.slot0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = T[id[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + u * B < bi.n_halo) ht[t0 + u * B] = v[u];
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    const int32_t ns = bi.n_own_pad / kWave;
    if (wave >= ns) return;
    const DevParams &p = P[bi.sys];
    const int64_t step = dstep[bi.sys] + rel;
    const char *tb = reinterpret_cast<const char *>(tile64);
    for (int32_t q = wave; q < ns; q += nw) {
        const int32_t sl = bi.slice0 + q;
        const SliceInfo si = slices[sl];
        const int32_t slot = sl * kWave + lane;
        const bool valid = lane < si.n_valid;
        const double sw = (p.laser_on | (si.flags & kSliceHeld)) ? srcw[slot] : 0.0;
        const uint32_t *rw = colw + (int64_t)si.colw_base64 * kWave + lane;
        const Fp64Lane r = lane_step_fp64_refs<false>(
            si, valid, p,
            [&](int32_t k) { return (rw[(int64_t)(k >> 1) * kWave] >> (16 * (k & 1))) & 0xffffu; },
            tile64[q * kWave + lane], Tl[slot], sw,
            [&](uint32_t off) { return *reinterpret_cast<const double *>(tb + 2 * off); },
            [&](uint32_t) { return 0.0; }, step, err);
        if (eatom && valid) eatom[slot] += r.e2l;
        Tn[slot] = r.Tnew;
        const double e2l = wave_sum(r.e2l), qv = wave_sum(r.q), lt = wave_sum(r.lt);
        if (lane == 0) {
            ledger[3 * (int64_t)sl + 0] += e2l;
            ledger[3 * (int64_t)sl + 1] += qv;
            ledger[3 * (int64_t)sl + 2] += lt;
        }
    }
}

// Grid-wide barrier for the persistent kernel.  bar[0] counts arrivals over
// the whole launch (barrier k completes at k * nblocks arrivals); bar[1] is an
// abort word raised when a block spins past the limit, so every block leaves
// instead of waiting forever.  Release / acquire at agent scope make the
// sub-step's writes visible across the XCDs.
__device__ inline bool grid_barrier(unsigned *bar, unsigned nblocks, unsigned k, unsigned *err) {
    __syncthreads();
    __shared__ int abort_flag;
    if (threadIdx.x == 0) {
        __threadfence();
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = k * nblocks;
        int ab = 0;
        unsigned long long spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                ab = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1ull << 25)) {
                atomicOr(err, kErrBarrier);
                __hip_atomic_store(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ab = 1;
                break;
            }
        }
        __threadfence();
        abort_flag = ab;
    }
    __syncthreads();
    return abort_flag == 0;
}

// Persistent FP32C launch: every workgroup owns a fixed contiguous range of
// slices, runs n_steps sub-steps over it, and meets the others at a grid
// barrier after each sub-step.  Workgroup b runs on XCD b mod 8; it takes
// logical range (b mod 8) * (G/8) + b/8 so that each XCD sweeps one
// contiguous eighth of the atoms and its L2 serves the neighbour gathers.
__global__ __launch_bounds__(256) void k_persistent_fp32c(
    const SliceInfo *slices, int32_t n_slices, const int32_t *col, float *Thi0, float *Thi1,
    int16_t *Tlo, const float *Tl, const float *srcw, const DevParams *P, const int64_t *dstep,
    int32_t n_steps, double *ledger, double *eatom, unsigned *err, unsigned *bar) {
    const unsigned G = gridDim.x;
    const unsigned b = blockIdx.x;
    const unsigned logical = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    const int32_t per = (n_slices + (int32_t)G - 1) / (int32_t)G;
    const int32_t s_lo = min(n_slices, (int32_t)logical * per);
    const int32_t s_hi = min(n_slices, s_lo + per);
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    for (int32_t st = 0; st < n_steps; ++st) {
        const float *Tin = (st & 1) ? Thi1 : Thi0;
        float *Tout = (st & 1) ? Thi0 : Thi1;
        for (int32_t sl = s_lo + wave; sl < s_hi; sl += nw) {
            const SliceInfo si = slices[sl];
            slice_step_fp32c(si, sl, lane, P[si.sys], col, Tin, Tout, Tlo, Tl, srcw,
                             dstep[si.sys] + st, ledger, eatom, err);
        }
        if (!grid_barrier(bar, G, (unsigned)st + 1u, err)) return;
    }
}

// Mean-field parameters (Section 2), first level: one workgroup of 4 waves per
// chunk of a system's slices; lanes accumulate T_e and |T^lat| of the valid
// atoms of slices wave, wave + 4, ..., then a fixed-order reduction.
__global__ __launch_bounds__(256) void k_mf_chunks(const MfChunk *chunks, int32_t chunk0,
                                                   const SliceInfo *slices, int32_t precision,
                                                   const double *T64, const float *Thi,
                                                   const int16_t *Tlo, const double *Tl64,
                                                   const float *Tl32, double *part) {
    const MfChunk ch = chunks[chunk0 + blockIdx.x];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double t = 0.0, l = 0.0;
    for (int32_t sl = ch.slice_begin + wave; sl < ch.slice_end; sl += 4) {
        if (lane < slices[sl].n_valid) {
            const int32_t slot = sl * kWave + lane;
            t += (precision == L2T_FP64) ? T64[slot] : state_value(Thi[slot], Tlo[slot]);
            l += (precision == L2T_FP64) ? fabs(Tl64[slot]) : (double)fabsf(Tl32[slot]);
        }
    }
    t = wave_sum(t);
    l = wave_sum(l);
    __shared__ double sh[2][4];
    if (lane == 0) {
        sh[0][wave] = t;
        sh[1][wave] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[2 * (int64_t)(chunk0 + blockIdx.x)] = ((sh[0][0] + sh[0][1]) + sh[0][2]) + sh[0][3];
        part[2 * (int64_t)(chunk0 + blockIdx.x) + 1] = ((sh[1][0] + sh[1][1]) + sh[1][2]) + sh[1][3];
    }
}

// Second level, one workgroup of 256 per system: fixed-order sum of the chunk
// partials, then c = lambda mean(T_e) and K = k_coef / mean(T^lat) into the
// parameter table.
__global__ __launch_bounds__(256) void k_mf_apply(DevParams *P, int32_t sys0, const double *part,
                                                  unsigned *err) {
    DevParams &p = P[sys0 + blockIdx.x];
    if (!p.mean_field) return;
    __shared__ double sh[2][256];
    double t = 0.0, l = 0.0;
    for (int32_t k = threadIdx.x; k < p.mf_nchunk; k += blockDim.x) {
        t += part[2 * (int64_t)(p.mf_chunk0 + k)];
        l += part[2 * (int64_t)(p.mf_chunk0 + k) + 1];
    }
    sh[0][threadIdx.x] = t;
    sh[1][threadIdx.x] = l;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double Te = sh[0][0] / (double)p.n_atoms, Tl = sh[1][0] / (double)p.n_atoms;
        if (!(Tl > 0.0)) {
            atomicOr(err, kErrMeanField);
            return;
        }
        const double cv = p.mf_lambda * Te, K = p.mf_kcoef / Tl;
        p.ce_model = L2T_CE_CONST;
        p.ce_const = cv;
        p.f_ce_const = (float)cv;
        p.K = K;
        p.A = p.span * K;
        p.f_A = (float)p.A;
        p.f_K = (float)K;
    }
}

__global__ void k_zero_u32(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

__global__ void k_bump(int64_t *dstep, int32_t s0, int32_t s1, int32_t n) {
    int32_t s = s0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (s < s1) dstep[s] += n;
}

__global__ void k_fill_f32(float *p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_f64(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_copy_range_f64(const double *a, double *b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}
__global__ void k_copy_range_f32(const float *a, float *b, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// per-slice E_e, sum T, max T, min T (one wave per slice)
__global__ void k_slice_energy(const SliceInfo *slices, int32_t slice0, int32_t n_slices,
                               int32_t precision, const double *T64, const float *Thi,
                               const int16_t *Tlo, const DevParams *P, double *red) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t q = blockIdx.x * (blockDim.x / kWave) + wave;
    if (q >= n_slices) return;
    const int32_t sl = slice0 + q;
    const SliceInfo si = slices[sl];
    const DevParams &p = P[si.sys];
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    double T = 0.0;
    if (valid) T = (precision == L2T_FP64) ? T64[slot] : state_value(Thi[slot], Tlo[slot]);
    double e = valid ? energy_of(p, T) : 0.0;
    double s = valid ? T : 0.0;
    double mx = valid ? T : -INFINITY, mn = valid ? T : INFINITY;
    e = wave_sum(e);
    s = wave_sum(s);
    mx = wave_max(mx);
    mn = wave_min(mn);
    if (lane == 0) {
        red[4 * (int64_t)sl + 0] = e;
        red[4 * (int64_t)sl + 1] = s;
        red[4 * (int64_t)sl + 2] = mx;
        red[4 * (int64_t)sl + 3] = mn;
    }
}

// per-system sums over its slices in a fixed order (one workgroup)
__global__ void k_system_reduce(int32_t slice0, int32_t n_slices, const double *red,
                                const double *ledger, double *out) {
    __shared__ double acc[7][256];
    const int t = threadIdx.x;
    double a[7] = {0, 0, 0, 0, 0, -INFINITY, INFINITY};
    for (int32_t q = t; q < n_slices; q += blockDim.x) {
        const int64_t sl = slice0 + q;
        a[0] += red[4 * sl + 0];
        a[1] += red[4 * sl + 1];
        a[2] += ledger[3 * sl + 0];
        a[3] += ledger[3 * sl + 1];
        a[4] += ledger[3 * sl + 2];
        a[5] = fmax(a[5], red[4 * sl + 2]);
        a[6] = fmin(a[6], red[4 * sl + 3]);
    }
    for (int k = 0; k < 7; ++k) acc[k][t] = a[k];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) {
            for (int k = 0; k < 5; ++k) acc[k][t] += acc[k][t + w];
            acc[5][t] = fmax(acc[5][t], acc[5][t + w]);
            acc[6][t] = fmin(acc[6][t], acc[6][t + w]);
        }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < 7; ++k) out[k] = acc[k][0];
}

__global__ void k_pair(const float *ti, const float *tj, float *out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = pair32(ti[i], tj[i], PairK{0.5f, 0.0f, 1.0f, -1.0f / 3.0f, kUTiny});
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// kernel parameter block of one system (its parameters, layout and modes)
DevParams dev_params_of(const SystemState &st) {
    const l2t_params &q = st.params;
    DevParams p{};
    p.T_min = q.T_min;
    p.span = q.T_max - q.T_min;
    p.inv_span = 1.0 / p.span;
    p.K = q.K;
    p.A = p.span * q.K;
    p.dt = q.dt;
    p.g = q.g;
    p.ce_const = q.ce_const;
    p.gamma = q.gamma;
    p.ce_cap = q.ce_cap;
    p.ce_model = q.ce_model;
    p.laser_on = q.laser_on;
    p.lp = q.laser_lp;
    p.t0 = q.laser_t0;
    p.sigma = q.laser_sigma;
    p.inv_sigma = q.laser_on ? 1.0 / q.laser_sigma : 0.0;
    p.x0 = q.laser_x0;
    p.i0 = q.laser_on ? q.laser_fluence * q.v_atom /
                            (q.laser_lp * std::sqrt(2.0 * M_PI) * q.laser_sigma)
                      : 0.0;
    p.atom_off = st.atom_off;
    p.n_pad = st.n_pad;
    p.slice0 = st.slice0;
    p.n_slices = st.n_slices;
    p.f_inv_span = (float)p.inv_span;
    p.f_half_inv_span = (float)(0.5 * p.inv_span);
    p.f_m_off = (float)(-q.T_min * p.inv_span);
    p.f_A = (float)p.A;
    p.f_K = (float)q.K;
    p.f_dt = (float)q.dt;
    p.f_g = (float)q.g;
    p.f_ce_const = (float)q.ce_const;
    p.f_gamma = (float)q.gamma;
    p.f_ce_cap = (float)q.ce_cap;
    p.f_T_min = (float)q.T_min;
    p.f_T_max = (float)q.T_max;
    p.f_i0 = (float)p.i0;
    p.f_inv2 = (float)(p.inv_span * p.inv_span);
    p.f_c_tiny = (float)(-p.inv_span * p.inv_span / 3.0);
    p.f_w_tiny = (float)((double)dev::kUTiny * p.span * p.span);
    p.has_fixed = st.has_fixed ? 1 : 0;
    p.mean_field = st.mf.on ? 1 : 0;
    p.n_atoms = st.desc.n_atoms;
    p.mf_lambda = st.mf.lambda;
    p.mf_kcoef = st.mf.k_coef;
    p.lat_fd = st.lf.on ? 1 : 0;
    p.K_lat = st.lf.K_lat;
    p.g_over_clat = st.lf.on ? q.g / st.lf.c_lat : 0.0;
    return p;
}

int upload_params(l2t_ctx *c) {
    const int S = (int)c->sys.size();
    c->hparams.assign(S, DevParams{});
    for (int s = 0; s < S; ++s) c->hparams[s] = dev_params_of(c->sys[s]);
    // mean-field chunk table: every system in the mode, in order, its slices in
    // chunks of kMfChunk
    std::vector<MfChunk> &chunks = c->h_mf_chunks;
    chunks.clear();
    for (int s = 0; s < S; ++s) {
        DevParams &p = c->hparams[s];
        const SystemState &st = c->sys[s];
        p.mf_chunk0 = (int32_t)chunks.size();
        if (st.mf.on)
            for (int32_t b = 0; b < st.n_slices; b += kMfChunk)
                chunks.push_back(MfChunk{s, st.slice0 + b, st.slice0 + std::min(st.n_slices, b + kMfChunk), 0});
        p.mf_nchunk = (int32_t)chunks.size() - p.mf_chunk0;
    }
    c->n_mf_chunks = (int32_t)chunks.size();
    if (c->n_mf_chunks > c->mf_chunks_cap) {
        drop_graphs(c);   // captured refreshes hold the old table
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, c->mf_chunks);
        c->mf_chunks = nullptr;
        c->mf_chunks_cap = 0;
        if (dev_malloc(c, (void **)&c->mf_chunks, sizeof(MfChunk) * chunks.size()) != hipSuccess)
            return fail(c, L2T_ENOMEM, "mean-field chunk table allocation failed");
        c->mf_chunks_cap = c->n_mf_chunks;
    }
    if (!chunks.empty())
        L2T_HIP(c, hipMemcpyAsync(c->mf_chunks, chunks.data(), sizeof(MfChunk) * chunks.size(),
                                  hipMemcpyHostToDevice, c->stream));
    L2T_HIP(c, hipMemcpyAsync(c->dparams, c->hparams.data(), sizeof(DevParams) * S,
                              hipMemcpyHostToDevice, c->stream));
    return L2T_OK;
}

int bump_steps(l2t_ctx *c, int32_t sys, int32_t n) {
    int32_t s0 = sys < 0 ? 0 : sys, s1 = sys < 0 ? (int32_t)c->sys.size() : sys + 1;
    hipLaunchKernelGGL(k_bump, dim3(nblk(s1 - s0, 256)), dim3(256), 0, c->stream, c->dstep, s0, s1,
                       n);
    L2T_HIP(c, hipGetLastError());
    for (int32_t s = s0; s < s1; ++s) c->sys[s].step += n;
    return L2T_OK;
}

int reset_ledger(l2t_ctx *c, int32_t sys) {
    const SystemState &st = c->sys[sys];
    hipLaunchKernelGGL(k_zero_f64, dim3(nblk(3 * (int64_t)st.n_slices, 256)), dim3(256), 0,
                       c->stream, c->ledger + 3 * (int64_t)st.slice0, 3 * (int64_t)st.n_slices);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

// One system (sys >= 0) or all systems (sys < 0), one launch per sub-step.
int mean_field_refresh(l2t_ctx *c, int32_t sys) {
    const int32_t s0 = sys < 0 ? 0 : sys, s1 = sys < 0 ? (int32_t)c->sys.size() : sys + 1;
    bool any = false;
    for (int32_t s = s0; s < s1; ++s) any |= c->sys[s].mf.on != 0;
    if (!any) return L2T_OK;
    // the chunks of systems s0..s1-1 are contiguous in the table
    const int32_t ch0 = c->hparams[s0].mf_chunk0;
    const int32_t ch1 = c->hparams[s1 - 1].mf_chunk0 + c->hparams[s1 - 1].mf_nchunk;
    if (ch1 > ch0)
        hipLaunchKernelGGL(k_mf_chunks, dim3(ch1 - ch0), dim3(256), 0, c->stream, c->mf_chunks, ch0,
                           c->slices, c->precision, c->T64[c->cur], c->Thi[c->cur], c->Tlo,
                           c->Tl64, c->Tl32, c->slice_red);
    hipLaunchKernelGGL(k_mf_apply, dim3(s1 - s0), dim3(256), 0, c->stream, c->dparams, s0,
                       c->slice_red, c->derr);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int zero_atom_ledger(l2t_ctx *c, int32_t sys) {
    const int64_t off = sys < 0 ? 0 : c->sys[sys].atom_off;
    const int64_t len = sys < 0 ? c->n_int : c->sys[sys].n_pad;
    if (len > 0)
        hipLaunchKernelGGL(k_zero_f64, dim3(nblk(len, 256)), dim3(256), 0, c->stream,
                           c->eatom + off, len);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

// All n sub-steps of one small system in one workgroup (FP64): the system's
// T and T^lat live in LDS, double-buffered, and a sub-step ends with a
// workgroup barrier, so no state goes through HBM between sub-steps.  One
// thread per slot (blockDim covers the largest system); neighbours are the
// global slots of the table minus the system's first slot.  The per-lane
// arithmetic is that of the per-sub-step kernel and the ledger rows and
// per-atom records receive the same additions in the same order, so the
// results are bitwise equal to n launches of k_step_fp64.
namespace {

__global__ __launch_bounds__(kResidentMaxSlots) void k_resident_fp64(
    const ResidentSys *__restrict__ rsys, const SliceInfo *__restrict__ slices,
    const int32_t *__restrict__ col, const double *T_in, double *T_even, double *T_odd,
    const double *Tl_in, double *Tl_even, double *Tl_odd, const double *__restrict__ srcw,
    const DevParams *__restrict__ P, const int64_t *__restrict__ dstep, int32_t n,
    double *__restrict__ ledger, double *__restrict__ eatom, unsigned *__restrict__ err) {
    extern __shared__ double sh[];
    const ResidentSys r = rsys[blockIdx.x];
    const int32_t np = blockDim.x;        // LDS stride: T[2][np], T^lat[2][np]
    const int32_t t = threadIdx.x;
    const bool mine = t < r.n_pad;        // whole waves: n_pad is a multiple of 64
    const int lane = t % kWave;
    const int32_t slot = r.slot0 + t;
    const int32_t sl = r.slice0 + t / kWave;
    SliceInfo si{};
    double sw = 0.0, ea = 0.0, l0 = 0.0, l1 = 0.0, l2 = 0.0;
    const DevParams &p = P[r.sys];
    if (mine) {
        si = slices[sl];
        sh[t] = T_in[slot];
        sh[2 * np + t] = Tl_in[slot];
        if (p.laser_on | (si.flags & kSliceHeld)) sw = srcw[slot];
        if (eatom) ea = eatom[slot];
        if (lane == 0) {
            l0 = ledger[3 * (int64_t)sl + 0];
            l1 = ledger[3 * (int64_t)sl + 1];
            l2 = ledger[3 * (int64_t)sl + 2];
        }
    }
    __syncthreads();
    const int64_t step0 = dstep[r.sys];
    const bool valid = mine && lane < si.n_valid;
    for (int32_t k = 0; k < n; ++k) {
        const double *Tc = sh + (k & 1) * np, *Lc = sh + (2 + (k & 1)) * np;
        double *Tn = sh + ((k & 1) ^ 1) * np, *Ln = sh + (2 + ((k & 1) ^ 1)) * np;
        if (mine) {
            const Fp64Lane o = lane_step_fp64(
                si, lane, valid, p, col, Tc[t], Lc[t], sw,
                [&](int32_t j) { return Tc[j - r.slot0]; },
                [&](int32_t j) { return Lc[j - r.slot0]; }, step0 + k, err);
            Tn[t] = o.Tnew;
            Ln[t] = o.tl_new;
            if (eatom && valid) ea += o.e2l;
            const double e2l = wave_sum(o.e2l), q = wave_sum(o.q), lt = wave_sum(o.lt);
            l0 += e2l;
            l1 += q;
            l2 += lt;
        }
        __syncthreads();
    }
    if (!mine) return;
    // the final state goes where n launches would leave it: the output buffer
    // of the last sub-step
    (n & 1 ? T_odd : T_even)[slot] = sh[(n & 1) * np + t];
    (n & 1 ? Tl_odd : Tl_even)[slot] = sh[(2 + (n & 1)) * np + t];
    if (eatom) eatom[slot] = ea;
    if (lane == 0) {
        ledger[3 * (int64_t)sl + 0] = l0;
        ledger[3 * (int64_t)sl + 1] = l1;
        ledger[3 * (int64_t)sl + 2] = l2;
    }
}

}  // namespace

// Batched FP64 advance with every system resident in one workgroup, when
// all systems fit (L2T_OPT_RESIDENT_MAX); L2T_ENOTIMPL otherwise, and the
// caller takes the per-sub-step launches.
static int resident_fp64(l2t_ctx *c, int32_t n, bool lat, double *eatom) {
    const int lim = c->tune.resident_max == 0 ? kResidentMaxSlots
                                              : std::min(c->tune.resident_max, kResidentMaxSlots);
    if (lim <= 0 || c->sys.empty()) return L2T_ENOTIMPL;
    int32_t np = 0;
    for (const auto &st : c->sys) {
        if (st.n_pad > lim) return L2T_ENOTIMPL;
        np = std::max(np, st.n_pad);
    }
    if (np <= 0) return L2T_ENOTIMPL;
    if (!c->res_valid) {
        c->h_res.resize(c->sys.size());
        for (size_t s = 0; s < c->sys.size(); ++s)
            c->h_res[s] = ResidentSys{(int32_t)s, c->sys[s].atom_off, c->sys[s].n_pad,
                                      c->sys[s].slice0};
        if (c->h_res.size() > c->res_cap) {
            dev_free(c, c->res);
            c->res = nullptr;
            c->res_cap = 0;
            if (dev_malloc(c, (void **)&c->res, sizeof(ResidentSys) * c->h_res.size()) != hipSuccess)
                return fail(c, L2T_ENOMEM, "resident system table allocation failed");
            c->res_cap = c->h_res.size();
        }
        L2T_HIP(c, hipMemcpyAsync(c->res, c->h_res.data(), sizeof(ResidentSys) * c->h_res.size(),
                                  hipMemcpyHostToDevice, c->stream));
        c->res_valid = true;
    }
    const int cur = c->cur;
    // without the lattice mode T^lat stays in its buffer
    double *tl_odd = lat ? c->Tl64b : c->Tl64;
    hipLaunchKernelGGL(k_resident_fp64, dim3((unsigned)c->sys.size()), dim3(np),
                       4 * sizeof(double) * (size_t)np, c->stream, c->res, c->slices, c->col,
                       c->T64[cur], c->T64[cur], c->T64[cur ^ 1], c->Tl64, c->Tl64, tl_odd,
                       c->srcw64, c->dparams, c->dstep, n, c->ledger, eatom, c->derr);
    L2T_HIP(c, hipGetLastError());
    if (n & 1) {
        c->cur ^= 1;
        if (lat) std::swap(c->Tl64, c->Tl64b);
    }
    return bump_steps(c, -1, n);
}

int advance_plain(l2t_ctx *c, int32_t sys, int32_t n) {
    const int32_t s0 = sys < 0 ? 0 : c->sys[sys].slice0;
    const int32_t ns = sys < 0 ? c->n_slices : c->sys[sys].n_slices;
    const int wpb = 4;
    const dim3 grid(nblk(ns, wpb)), block(wpb * kWave);
    double *eatom = atom_ledger_ptr(c);
    int rc0 = mean_field_refresh(c, sys);
    if (rc0 != L2T_OK) return rc0;
    // two-temperature lattice: T^lat alternates between the two buffers
    bool lat = false;
    if (c->precision == L2T_FP64)
        for (int32_t s = (sys < 0 ? 0 : sys); s < (sys < 0 ? (int32_t)c->sys.size() : sys + 1); ++s)
            lat |= c->sys[s].lf.on != 0;
    if (sys < 0 && c->precision == L2T_FP64) {
        int rc = resident_fp64(c, n, lat, eatom);
        if (rc != L2T_ENOTIMPL) return rc;
    }
    // FP64 sub-steps through LDS brick tiles (the kernel choice) when the
    // launch covers at least one brick per CU, no system is in the lattice
    // mode and an 8-byte tile fits 64 KB of LDS; otherwise the global-gather
    // k_step_fp64, whose one wave per slice spreads a small system over more
    // CUs (one brick is one workgroup).  Both give bitwise-equal states.
    // all systems: the XCD launch list; one system: its range of the brick list
    const int32_t *b_list0 = sys < 0 ? c->xcd_list : c->brick_list + c->sys[sys].list0;
    const int32_t b_n = sys < 0 ? c->n_xcd_list : c->sys[sys].n_list;
    const int32_t b_bricks = sys < 0 ? c->n_brick_list : c->sys[sys].n_list;
    const bool brick64 = c->precision == L2T_FP64 && c->tune.kernel == kKernelBrick && !lat &&
                         b_bricks >= std::max(1, c->n_cu) &&
                         (size_t)c->tile_max * sizeof(double) <= 65536;
    const unsigned b_grid = (unsigned)((b_n + 7) / 8 * 8);
    const size_t b_lds = sizeof(double) * (size_t)c->tile_max;
    // one FP64 sub-step from state buffer cu (relative step q within the call)
    auto step64 = [&](int cu, int32_t q, const double *tl_in, double *tl_out) {
        if (brick64) {
            const int32_t *b_list = sys < 0 ? xcd_list_for(c, q) : b_list0;
            if (b_n > 0)
                hipLaunchKernelGGL(k_brick_fp64, dim3(b_grid), dim3(kBrickBlockMax), b_lds,
                                   c->stream, c->bricks, b_list, b_n, c->slices, c->colw, c->halo,
                                   c->T64[cu], c->T64[cu ^ 1], c->Tl64, c->srcw64, c->dparams,
                                   c->dstep, q, c->ledger, eatom, c->derr);
        } else {
            hipLaunchKernelGGL(k_step_fp64, grid, block, 0, c->stream, c->slices, s0, ns, c->col,
                               c->T64[cu], c->T64[cu ^ 1], tl_in, tl_out, c->srcw64, c->dparams,
                               c->dstep, q, c->ledger, eatom, c->derr);
        }
    };
    if (sys < 0 && c->precision == L2T_FP64 && c->tune.graph != 0) {
        // all systems: replays of captured chunks, as in the FP32C advance.
        // A chunk is keyed by its length, the state buffer it starts from,
        // the lattice mode and which lattice buffer holds T^lat.
        for (int32_t left = n; left > 0;) {
            const int32_t k = std::min(left, kGraphChunk);
            const int mode = (1 << 16) | (c->cur << 8) | ((int)lat << 9) |
                             ((int)(c->Tl64 > c->Tl64b) << 10) | (eatom ? 1 << 12 : 0) |
                             (brick64 ? 1 << 13 : 0);
            GraphKey key{k, mode, 0};
            auto it = c->graphs.find(key);
            if (it == c->graphs.end()) {
                if (!c->cap_stream)
                    L2T_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                hipGraph_t g = nullptr;
                hipStream_t user = c->stream;
                L2T_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
                c->stream = c->cap_stream;
                double *tlb[2] = {c->Tl64, c->Tl64b};
                for (int32_t q = 0; q < k; ++q)
                    step64(c->cur ^ (q & 1), q, lat ? tlb[q & 1] : c->Tl64,
                           lat ? tlb[(q & 1) ^ 1] : nullptr);
                hipLaunchKernelGGL(k_bump, dim3(nblk((int64_t)c->sys.size(), 256)), dim3(256), 0,
                                   c->stream, c->dstep, 0, (int32_t)c->sys.size(), k);
                const hipError_t el = hipGetLastError();
                c->stream = user;
                hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
                if (el != hipSuccess || e != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return hip_fail(c, el != hipSuccess ? el : e, "plain advance capture");
                }
                hipGraphExec_t ge = nullptr;
                e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
                it = c->graphs.emplace(key, ge).first;
            }
            L2T_HIP(c, hipGraphLaunch(it->second, c->stream));
            if (k & 1) {
                c->cur ^= 1;
                if (lat) std::swap(c->Tl64, c->Tl64b);
            }
            left -= k;
        }
        for (auto &st : c->sys) st.step += n;
        return L2T_OK;
    }
    double *tl_buf[2] = {c->Tl64, c->Tl64b};
    int cur = c->cur;
    for (int32_t k = 0; k < n; ++k) {
        if (c->precision == L2T_FP64) {
            step64(cur, k, lat ? tl_buf[k & 1] : c->Tl64, lat ? tl_buf[(k & 1) ^ 1] : nullptr);
        } else {
            hipLaunchKernelGGL(k_step_fp32c, grid, block, 0, c->stream, c->slices, s0, ns, c->col,
                               c->Thi[cur], c->Thi[cur ^ 1], c->Tlo, c->Tl32, c->srcw32,
                               c->dparams, c->dstep, k, c->ledger, eatom, c->derr);
        }
        cur ^= 1;
    }
    L2T_HIP(c, hipGetLastError());
    if (lat && (n & 1)) {
        if (sys < 0) {
            std::swap(c->Tl64, c->Tl64b);   // every slot was carried over
        } else {
            const SystemState &st = c->sys[sys];
            hipLaunchKernelGGL(k_copy_range_f64, dim3(nblk(st.n_pad, 256)), dim3(256), 0,
                               c->stream, c->Tl64b + st.atom_off, c->Tl64 + st.atom_off,
                               (int64_t)st.n_pad);
            L2T_HIP(c, hipGetLastError());
        }
    }
    if (n & 1) {
        if (sys < 0) {
            c->cur ^= 1;
        } else {
            // keep every system's state in the same buffer: copy this one back
            const SystemState &st = c->sys[sys];
            if (c->precision == L2T_FP64)
                hipLaunchKernelGGL(k_copy_range_f64, dim3(nblk(st.n_pad, 256)), dim3(256), 0,
                                   c->stream, c->T64[c->cur ^ 1] + st.atom_off,
                                   c->T64[c->cur] + st.atom_off, (int64_t)st.n_pad);
            else
                hipLaunchKernelGGL(k_copy_range_f32, dim3(nblk(st.n_pad, 256)), dim3(256), 0,
                                   c->stream, c->Thi[c->cur ^ 1] + st.atom_off,
                                   c->Thi[c->cur] + st.atom_off, (int64_t)st.n_pad);
            L2T_HIP(c, hipGetLastError());
        }
    }
    return bump_steps(c, sys, n);
}

// Largest co-resident grid of the persistent kernel at this block size.
static int persistent_grid(l2t_ctx *c, int block) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent_fp32c, block, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int slices_per_block_min = std::max(1, block / kWave);
    int want = (c->n_slices + slices_per_block_min - 1) / slices_per_block_min;
    int g = std::min(per_cu * c->n_cu, want);
    if (g >= 8) g -= g % 8;
    return std::max(1, g);
}

// FP32C, all systems, n sub-steps starting at the current state.
int fp32c_launch(l2t_ctx *c, int32_t n, int kernel, int persistent, int block, double *eatom) {
    int cur = c->cur;
    if (kernel == kKernelBrick) {
        // the XCD launch list: G workgroups, a multiple of 8
        const int32_t nl = c->n_xcd_list;
        const unsigned grid = (unsigned)nl;
        const size_t lds = sizeof(float) * (size_t)c->tile_max;
        const auto kern = brick_kernel<false>(c->tune.table_used);
        for (int32_t k = 0; k < n && nl > 0; ++k) {
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, c->stream,
                               c->bricks, xcd_list_for(c, k), nl, c->slices, c->colw, c->halo,
                               c->Thi[cur], c->Thi[cur ^ 1], nullptr, c->Tlo, c->Tl32, c->srcw32,
                               c->dparams, c->dstep, k, c->ledger, eatom, c->derr);
            cur ^= 1;
        }
    } else if (persistent) {
        block = std::min(block, kSlicedBlockMax);
        const int grid = persistent_grid(c, block);
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, c->stream, c->dbar, 2);
        hipLaunchKernelGGL(k_persistent_fp32c, dim3(grid), dim3(block), 0, c->stream, c->slices,
                           c->n_slices, c->col, c->Thi[cur], c->Thi[cur ^ 1], c->Tlo, c->Tl32,
                           c->srcw32, c->dparams, c->dstep, n, c->ledger, eatom, c->derr, c->dbar);
    } else {
        block = std::min(block, kSlicedBlockMax);
        const int wpb = block / kWave;
        const dim3 g(nblk(c->n_slices, wpb)), b(block);
        for (int32_t k = 0; k < n; ++k) {
            hipLaunchKernelGGL(k_step_fp32c, g, b, 0, c->stream, c->slices, 0, c->n_slices, c->col,
                               c->Thi[cur], c->Thi[cur ^ 1], c->Tlo, c->Tl32, c->srcw32,
                               c->dparams, c->dstep, k, c->ledger, eatom, c->derr);
            cur ^= 1;
        }
    }
    L2T_HIP(c, hipGetLastError());
    hipLaunchKernelGGL(k_bump, dim3(nblk((int64_t)c->sys.size(), 256)), dim3(256), 0, c->stream,
                       c->dstep, 0, (int32_t)c->sys.size(), n);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

// Time n sub-steps of the brick kernel on the current layout from a uniform
// stand-in state held in scratch memory (1,000 K, no coupling, no source), so
// the brick edge can be measured before any field of the new layout is
// written.  The context's state, ledger, step counters and error word are not
// touched.  alternate: the sweep order that reverses the launch list on odd
// sub-steps; stream: non-temporal table loads.  *ms receives the faster of
// two timed runs.
int brick_probe(l2t_ctx *c, int32_t n, bool alternate, bool stream, float *ms) {
    *ms = 0.0f;
    const size_t NI = (size_t)c->n_int, NS = (size_t)c->n_slices, S = c->sys.size();
    if (c->n_brick_list == 0 || NI == 0 || n < 1) return L2T_OK;
    const size_t fb = sizeof(float) * NI;
    const size_t bytes = 4 * fb + sizeof(DevParams) * S + sizeof(double) * 3 * NS +
                         sizeof(int64_t) * S + sizeof(unsigned) + 8 * 256;
    if (ensure_scratch(c, bytes) != L2T_OK) return L2T_ENOMEM;
    char *q = (char *)c->scratch;
    auto take = [&](size_t b) {
        char *r = q;
        q += (b + 255) / 256 * 256;
        return r;
    };
    float *Ta = (float *)take(fb), *Tb = (float *)take(fb), *zf = (float *)take(fb);
    int16_t *zl = reinterpret_cast<int16_t *>(zf);   // q = 0 (the 0.0f fill clears its bits)
    float *tl = (float *)take(fb);
    DevParams *P = (DevParams *)take(sizeof(DevParams) * S);
    double *led = (double *)take(sizeof(double) * 3 * NS);
    int64_t *stp = (int64_t *)take(sizeof(int64_t) * S);
    unsigned *perr = (unsigned *)take(sizeof(unsigned));
    std::vector<DevParams> hp(S);
    for (size_t s = 0; s < S; ++s) {
        SystemState st = c->sys[s];
        st.params = l2t_params{};
        st.params.T_min = 0.0;
        st.params.T_max = 2.0e4;
        st.params.K = 1.0;
        st.params.dt = 0.05;
        st.params.ce_model = L2T_CE_CONST;
        st.params.ce_const = 1.0e-4;
        st.has_fixed = false;
        st.mf.on = 0;
        st.lf.on = 0;
        hp[s] = dev_params_of(st);
    }
    const hipStream_t s_ = c->stream;
    L2T_HIP(c, hipMemcpyAsync(P, hp.data(), sizeof(DevParams) * S, hipMemcpyHostToDevice, s_));
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk((int64_t)NI, 256)), dim3(256), 0, s_, Ta, (int64_t)NI,
                       1000.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk((int64_t)NI, 256)), dim3(256), 0, s_, zf, (int64_t)NI,
                       0.0f);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblk((int64_t)NI, 256)), dim3(256), 0, s_, tl, (int64_t)NI,
                       1000.0f);
    hipLaunchKernelGGL(k_zero_f64, dim3(nblk((int64_t)(3 * NS), 256)), dim3(256), 0, s_, led,
                       (int64_t)(3 * NS));
    L2T_HIP(c, hipMemsetAsync(stp, 0, sizeof(int64_t) * S, s_));
    L2T_HIP(c, hipMemsetAsync(perr, 0, sizeof(unsigned), s_));
    L2T_HIP(c, hipGetLastError());
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    L2T_HIP(c, hipEventCreate(&ev.e0));
    L2T_HIP(c, hipEventCreate(&ev.e1));
    hipEvent_t e0 = ev.e0, e1 = ev.e1;
    const unsigned grid = (unsigned)c->n_xcd_list;
    const size_t lds = sizeof(float) * (size_t)c->tile_max;
    float best = 1e30f;
    hipError_t e = hipSuccess;
    const auto kern = brick_kernel<false>(stream ? 2 : 1);
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
        (void)hipEventRecord(e0, s_);
        // T^lat and the source weight both read the constant 1,000 K buffer
        // (a positive weight marks no atom as held); the low part is updated in place
        for (int32_t k = 0; k < n; ++k)
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kBrickBlockMax), lds, s_,
                               c->bricks,
                               c->xcd_list + ((alternate && (k & 1)) ? c->n_xcd_list : 0),
                               c->n_xcd_list, c->slices, c->colw,
                               c->halo, (k & 1) ? Tb : Ta, (k & 1) ? Ta : Tb, nullptr, zl, tl, tl,
                               P, stp, k, led, nullptr, perr);
        (void)hipEventRecord(e1, s_);
        e = hipEventSynchronize(e1);
        float t = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e == hipSuccess) best = std::min(best, t);
    }
    if (e != hipSuccess) return hip_fail(c, e, "brick probe");
    L2T_HIP(c, hipGetLastError());
    *ms = best;
    return L2T_OK;
}

// one FP32C sub-step of all systems in the LDS-brick form on explicit state
// buffers, the low part read from lo_in and written to Tlo (the adjoint's
// recomputation between checkpoints)
int brick_step_fp32c(l2t_ctx *c, int block, const float *Thi, float *Thi_n, const int16_t *lo_in,
                     int16_t *Tlo, const int64_t *dstep, int32_t rel, double *ledger) {
    const int32_t nl = c->n_xcd_list;
    if (nl <= 0) return L2T_OK;
    const unsigned grid = (unsigned)nl;
    const size_t lds = sizeof(float) * (size_t)c->tile_max;
    const auto kern = brick_kernel<true>(c->tune.table_used);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, c->stream, c->bricks,
                       xcd_list_for(c, rel), nl, c->slices, c->colw, c->halo, Thi, Thi_n, lo_in, Tlo,
                       c->Tl32, c->srcw32, c->dparams, dstep, rel, ledger, nullptr, c->derr);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

void drop_graphs(l2t_ctx *c) {
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// capture k FP32C sub-steps of all systems (from buffer `cur`, the step
// counters advanced at the end) into an executable hipGraph.  The capture runs
// on a private stream: the caller's may be the legacy null stream, which
// cannot be captured; the graph is replayed on the caller's.
int capture_fp32c(l2t_ctx *c, int32_t k, int kernel, int persistent, int block, double *eatom,
                  hipGraphExec_t *out) {
    if (!c->cap_stream)
        L2T_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipStream_t user = c->stream;
    L2T_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    c->stream = c->cap_stream;
    int rc = fp32c_launch(c, k, kernel, persistent, block, eatom);
    c->stream = user;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc != L2T_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    *out = ge;
    return L2T_OK;
}

// FP32C advance of all systems with the tuned configuration.  The mean-field
// parameters are refreshed from the state at the start of the advance.  The
// sub-steps are then launched one by one, or run as replays of captured
// hipGraphs of kGraphChunk sub-steps plus one graph for the remainder, each
// captured once per (length, buffer parity, configuration); which of the two
// is the option's, or the autotuner's, timed on its probe.  Every captured
// chunk ends by advancing the device step counters, so a replay does not
// depend on where in the advance it runs, and a new neighbour table costs one
// short capture rather than one node per sub-step of the whole advance.
int advance_fp32c(l2t_ctx *c, int32_t n) {
    const Tuning &t = c->tune;
    int rc = mean_field_refresh(c, -1);
    if (rc != L2T_OK) return rc;
    double *eatom = atom_ledger_ptr(c);
    if (!t.graph_used) {
        rc = fp32c_launch(c, n, t.kernel, t.persistent, t.block, eatom);
        if (rc != L2T_OK) return rc;
        if (n & 1) c->cur ^= 1;
    } else {
        for (int32_t left = n; left > 0;) {
            const int32_t k = std::min(left, kGraphChunk);
            GraphKey key{k, (c->cur << 8) | (t.persistent << 4) | t.kernel | (eatom ? 1 << 12 : 0),
                         t.block};
            auto it = c->graphs.find(key);
            if (it == c->graphs.end()) {
                hipGraphExec_t ge = nullptr;
                rc = capture_fp32c(c, k, t.kernel, t.persistent, t.block, eatom, &ge);
                if (rc != L2T_OK) return rc;
                it = c->graphs.emplace(key, ge).first;
            }
            L2T_HIP(c, hipGraphLaunch(it->second, c->stream));
            if (k & 1) c->cur ^= 1;
            left -= k;
        }
    }
    for (auto &st : c->sys) st.step += n;
    return L2T_OK;
}

int energies(l2t_ctx *c, int32_t sys, l2t_energy_report *out) {
    const SystemState &st = c->sys[sys];
    hipLaunchKernelGGL(k_slice_energy, dim3(nblk(st.n_slices, 4)), dim3(256), 0, c->stream,
                       c->slices, st.slice0, st.n_slices, c->precision, c->T64[c->cur],
                       c->Thi[c->cur], c->Tlo, c->dparams, c->slice_red);
    hipLaunchKernelGGL(k_system_reduce, dim3(1), dim3(256), 0, c->stream, st.slice0, st.n_slices,
                       c->slice_red, c->ledger, c->energy_out);
    L2T_HIP(c, hipGetLastError());
    double h[8] = {0};
    L2T_HIP(c, hipMemcpyAsync(h, c->energy_out, sizeof(double) * 7, hipMemcpyDeviceToHost,
                              c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    out->step = st.step;
    out->t = 0.0;
    out->E_e = h[0];
    out->sum_T = h[1];
    out->E_e_to_l = h[2];
    out->E_src = h[3];
    out->T_ledger_acc = h[4];
    out->T_max_atom = h[5];
    out->T_min_atom = h[6];
    return L2T_OK;
}

int pair_fp32(const float *ti, const float *tj, float *out, int64_t n, hipStream_t s) {
    if (n == 0) return L2T_OK;
    hipLaunchKernelGGL(k_pair, dim3(nblk(n, 256)), dim3(256), 0, s, ti, tj, out, n);
    return hipGetLastError() == hipSuccess ? L2T_OK : L2T_EHIP;
}

}  // namespace l2t
