// Device-side building blocks of the sub-step: reductions, heat capacity,
// the FP32 product-form pair term and its derivative, and the per-slice
// FP64 / FP32C sub-step bodies.  Included by the forward kernels and by the
// adjoint, which recomputes forward states with exactly these functions.
#pragma once

#include <hip/hip_runtime.h>

#include "l2t_internal.h"
#include "state_fp32c.h"

namespace l2t {
namespace dev {

// ---- wavefront reductions ----------------------------------------------------
__device__ inline double wave_sum(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double wave_max(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}
__device__ inline double wave_min(double v) {
    for (int o = kWave / 2; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
    return v;
}


// ---- heat capacity models --------------------------------------------------------
__device__ inline double ce64(const DevParams &p, double T) {
    if (p.ce_model == L2T_CE_CONST) return p.ce_const;
    double c = p.gamma * T;
    return (p.ce_model == L2T_CE_CAPPED && c > p.ce_cap) ? p.ce_cap : c;
}
__device__ inline float ce32(const DevParams &p, float T) {
    if (p.ce_model == L2T_CE_CONST) return p.f_ce_const;
    float c = p.f_gamma * T;
    return (p.ce_model == L2T_CE_CAPPED && c > p.f_ce_cap) ? p.f_ce_cap : c;
}
__device__ inline double energy_of(const DevParams &p, double T) {
    if (p.ce_model == L2T_CE_CONST) return p.ce_const * T;
    if (p.ce_model == L2T_CE_LINEAR) return 0.5 * p.gamma * T * T;
    double Ts = p.ce_cap / p.gamma;
    return (T <= Ts) ? 0.5 * p.gamma * T * T : 0.5 * p.gamma * Ts * Ts + p.ce_cap * (T - Ts);
}

// Gaussian time factor of Eq. 10 at the start of sub-step `step`
__device__ inline double pulse64(const DevParams &p, int64_t step) {
    double t = (double)step * p.dt - p.t0;
    return exp(-t * t / (2.0 * p.sigma * p.sigma));
}
__device__ inline float pulse32(const DevParams &p, int64_t step) {
    const float x = (float)(((double)step * p.dt - p.t0) * p.inv_sigma);
    return expf(-0.5f * x * x);
}
// i_0 times the Gaussian time factor of Eq. 10 at sub-step `step` (0 without the
// source): the same for every atom of the system, so taken once per wave
__device__ inline float source_factor32(const DevParams &p, int64_t step) {
    return p.laser_on ? p.f_i0 * pulse32(p, step) : 0.0f;
}

// ---- FP32 pair term -------------------------------------------------------------
// With d = theta_j - theta_i and m = (theta_i + theta_j)/2 the pair term of
// Eq. 2 equals d [cosh d - (2 m (1 - m) + d^2/2) sinh(d)/d].  Writing u = d^2,
// cosh d - (u/2) sinh(d)/d = sum_k (1 - k) u^k / (2k)! =: P(u) and
// sinh(d)/d = sum_k u^k / (2k+1)! =: Q(u), so f = d h with
// h = P(u) - 2 m (1 - m) Q(u).  pair32 returns span * f = dT h in temperature
// units (dT = T_j - T_i is exact for nearby FP32 temperatures).  Three exact
// tiers by the size of u: u <= kUTiny keeps P = 1, Q = 1 + u/6 (dropped terms
// below 3e-9 relative), u <= 1e-2 adds the u^2, u^3 terms, larger u takes the
// series to u^6 (below half an FP32 ulp of h for |d| <= 1).  Everything
// depends on (m, u) only, symmetric in (i, j), so pair32(i, j) = -pair32(j, i)
// holds bitwise.
constexpr float kUTiny = 2.5e-4f;

// third descriptor word of a raw (unswizzled, stride 0) buffer resource on
// gfx9-family chips: 32-bit data format, range checked against num_records
constexpr int kBufferRsrcWord3 = 0x00020000;

struct PairK {
    float hinv;     // 0.5 / span
    float moff;     // -T_min / span
    float inv2;     // 1 / span^2
    float c_tiny;   // -1 / (3 span^2): u/6 scaled by -2, in T^2 units
    float w_tiny;   // kUTiny * span^2
};

__device__ __forceinline__ PairK pair_consts(const DevParams &p) {
    PairK k{p.f_half_inv_span, p.f_m_off, p.f_inv2, p.f_c_tiny, p.f_w_tiny};
    // m = (Ti + Tj) * hinv + moff reads two uniform operands; a VALU instruction
    // reads at most one scalar register, so moff is held in a vector register
    // (otherwise it is copied into one for every pair term)
    asm volatile("" : "+v"(k.moff));
    return k;
}

// Series coefficients of the two upper tiers.  Kept in a device table (read
// into scalar registers) rather than as literals, which the compiler would
// otherwise hoist into vector registers for the whole sub-step loop.
__constant__ float kPairUpper[10] = {
    -1.0f / 360.0f,      -1.0f / 24.0f,       // P, middle tier
    -2.0f / 120.0f,      -2.0f / 6.0f,        // Q2, middle tier
    -5.0f / 479001600.0f, -4.0f / 3628800.0f, -3.0f / 40320.0f,   // P, top tier
    -2.0f / 39916800.0f, -2.0f / 362880.0f, -2.0f / 5040.0f};     // Q2, top tier

// h on the two upper tiers (w = dT^2 > w_tiny), a = 2 m (1 - m) / 2
__device__ __forceinline__ float pair32_h_upper(float a, float w, const PairK &k) {
    const float *c = kPairUpper;
    const float u = w * k.inv2;
    float P, Q2;   // Q2 = -2 Q
    if (u <= 1.0e-2f) {
        P = fmaf(u * u, fmaf(u, c[0], c[1]), 1.0f);
        Q2 = fmaf(u, fmaf(u, c[2], c[3]), -2.0f);
    } else {
        float pp = fmaf(u, c[4], c[5]);
        pp = fmaf(u, pp, c[6]);
        pp = fmaf(u, pp, c[0]);
        pp = fmaf(u, pp, c[1]);
        P = fmaf(u * u, pp, 1.0f);
        float q = fmaf(u, c[7], c[8]);
        q = fmaf(u, q, c[9]);
        q = fmaf(u, q, c[2]);
        q = fmaf(u, q, c[3]);
        Q2 = fmaf(u, q, -2.0f);
    }
    return fmaf(a, Q2, P);
}

// the parts of one pair term every tier shares, and h on the lowest tier
struct PairParts {
    float dT, a, w, h;
};
__device__ __forceinline__ PairParts pair32_parts(float Ti, float Tj, const PairK &k) {
    PairParts r;
    r.dT = Tj - Ti;
    const float m = fmaf(Ti + Tj, k.hinv, k.moff);
    r.a = fmaf(-m, m, m);
    r.w = r.dT * r.dT;
    r.h = fmaf(r.a, fmaf(r.w, k.c_tiny, -2.0f), 1.0f);
    return r;
}

__device__ __forceinline__ float pair32(float Ti, float Tj, const PairK &k) {
    PairParts r = pair32_parts(Ti, Tj, k);
    if (r.w > k.w_tiny) r.h = pair32_h_upper(r.a, r.w, k);
    return r.dT * r.h;
}

// ---- one FP64 plain sub-step --------------------------------------------------------
struct Fp64Lane {
    double Tnew, tl_new, e2l, q, lt;
};

// One lane of the literal Eq. 2 sub-step in FP64.  Ti, tl_i and sw are the
// lane's own T, T^lat and source weight; T_of(j) and Tl_of(j) return the
// step-n values of the neighbour in global slot j (from HBM or from an LDS
// copy of the system).  tl_new is the lattice temperature after the step
// (the Section 3.1 Fourier law when the system carries the lattice mode,
// otherwise tl_i); e2l, q and lt are the lane's ledger terms.
// ref_at(k) returns the lane's k-th neighbour reference (a global slot, or
// the byte offset of an LDS tile entry), T_of and Tl_of the step-n T and
// T^lat it refers to.  LAT = false compiles the lattice mode out (for
// launches that never carry a system in that mode).
template <bool LAT = true, class RefAt, class TOf, class TlOf>
__device__ __forceinline__ Fp64Lane lane_step_fp64_refs(const SliceInfo &si, bool valid,
                                                        const DevParams &p, RefAt ref_at,
                                                        double Ti, double tl_i, double sw,
                                                        TOf T_of, TlOf Tl_of, int64_t step,
                                                        unsigned *err) {
    Fp64Lane r{Ti, tl_i, 0.0, 0.0, 0.0};
    // two-temperature lattice (Section 3.1): the Fourier law over the same
    // neighbours plus the coupling, from the step-n states
    if constexpr (LAT) {
        if (p.lat_fd && valid) {
            const double tli = fabs(tl_i);
            double Lsum = 0.0;
            for (int32_t k = 0; k < si.width; ++k) Lsum += fabs(Tl_of(ref_at(k))) - tli;
            r.tl_new = tli + p.dt * (p.K_lat * Lsum + p.g_over_clat * (Ti - tli));
        }
    }
    const double ti = (Ti - p.T_min) * p.inv_span;
    // the literal pair term of Eq. 2 in theta units; its two exponentials are
    // e and 1/e, so one exponential and one division per pair
    auto pair = [&](double Tj) {
        const double tj = (Tj - p.T_min) * p.inv_span;
        const double e = exp(ti - tj);
        return tj * (1.0 - ti) * e - ti * (1.0 - tj) / e;
    };
    // neighbours in chunks of 8: the chunk's references, then its temperatures,
    // are requested before any term is evaluated, so 8 loads are in flight
    // where the plain loop has one; terms are added in row order either way
    constexpr int kChunk = 8;
    double S = 0.0;
    int32_t k = 0;
    for (; k + kChunk <= si.width; k += kChunk) {
        decltype(ref_at(0)) j[kChunk];
        double Tj[kChunk];
#pragma unroll
        for (int u = 0; u < kChunk; ++u) j[u] = ref_at(k + u);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) Tj[u] = T_of(j[u]);
#pragma unroll
        for (int u = 0; u < kChunk; ++u) S += pair(Tj[u]);
    }
    for (; k < si.width; ++k) S += pair(T_of(ref_at(k)));
    if (valid) {
        const double c = ce64(p, Ti);
        const double coup = (signbit(tl_i) && !p.lat_fd) ? 0.0 : p.g * (Ti - fabs(tl_i));
        double q = 0.0;
        if (p.laser_on) q = p.i0 * fabs(sw) * pulse64(p, step);
        r.e2l = coup * p.dt;
        if (p.has_fixed && signbit(sw)) {
            // held: the exchange it would receive goes to the temperature ledger
            r.lt = p.dt * (p.A * S);
        } else {
            r.Tnew = Ti + p.dt * (p.A * S - coup / c + q / c);
            r.lt = p.dt * (coup - q) / c;
            const double th = (r.Tnew - p.T_min) * p.inv_span;
            if (!(th >= 0.0 && th <= 1.0)) atomicOr(err, kErrRange);
        }
        r.q = q * p.dt;
    }
    return r;
}

// the same lane with its neighbours through the int32 global-slot table
template <class TOf, class TlOf>
__device__ __forceinline__ Fp64Lane lane_step_fp64(const SliceInfo &si, int lane, bool valid,
                                                   const DevParams &p,
                                                   const int32_t *__restrict__ col, double Ti,
                                                   double tl_i, double sw, TOf T_of, TlOf Tl_of,
                                                   int64_t step, unsigned *err) {
    const int32_t *__restrict__ cp = col + (int64_t)si.col_base64 * kWave + lane;
    return lane_step_fp64_refs(
        si, valid, p, [&](int32_t k) { return cp[(int64_t)k * kWave]; }, Ti, tl_i, sw, T_of,
        Tl_of, step, err);
}

// one slice through HBM; Tl_out, when given, receives T^lat after the step
// (carried over for systems without the lattice mode)
__device__ inline void slice_step_fp64(const SliceInfo &si, int32_t sl, int lane,
                                       const DevParams &p, const int32_t *__restrict__ col,
                                       const double *__restrict__ T, double *__restrict__ Tn,
                                       const double *__restrict__ Tl,
                                       double *__restrict__ Tl_out,
                                       const double *__restrict__ srcw, int64_t step,
                                       double *__restrict__ ledger, double *__restrict__ eatom,
                                       unsigned *err) {
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    // the source weight's sign bit marks atoms that hold their T_e
    const double sw = (p.laser_on | (si.flags & kSliceHeld)) ? srcw[slot] : 0.0;
    const Fp64Lane r = lane_step_fp64(
        si, lane, valid, p, col, T[slot], Tl[slot], sw, [&](int32_t j) { return T[j]; },
        [&](int32_t j) { return Tl[j]; }, step, err);
    if (Tl_out) Tl_out[slot] = r.tl_new;
    if (eatom && valid) eatom[slot] += r.e2l;
    Tn[slot] = r.Tnew;
    const double e2l = wave_sum(r.e2l), q = wave_sum(r.q), lt = wave_sum(r.lt);
    if (lane == 0) {
        ledger[3 * (int64_t)sl + 0] += e2l;
        ledger[3 * (int64_t)sl + 1] += q;
        ledger[3 * (int64_t)sl + 2] += lt;
    }
}

// Sum over the 64 lanes with DPP moves (VALU only, no LDS traffic); the
// total lands in lane 63 and is broadcast through readlane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
    v += dpp_f32<0x111, 0xf>(v);   // row_shr:1
    v += dpp_f32<0x112, 0xf>(v);   // row_shr:2
    v += dpp_f32<0x114, 0xf>(v);   // row_shr:4
    v += dpp_f32<0x118, 0xf>(v);   // row_shr:8   -> lane 15 of each row: row sum
    v += dpp_f32<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f32<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3 -> lane 63: total
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Smallest and largest value over the 64 lanes with DPP moves: a lane whose
// DPP source lies outside its row keeps the identity (bound_ctrl off), and
// the result lands in lane 63, broadcast through readlane.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_keep_f32(float old, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL,
                                                      ROW_MASK, 0xf, false));
}
__device__ __forceinline__ float wave_min_f32(float v) {
    const float I = INFINITY;
    v = fminf(v, dpp_keep_f32<0x111, 0xf>(I, v));
    v = fminf(v, dpp_keep_f32<0x112, 0xf>(I, v));
    v = fminf(v, dpp_keep_f32<0x114, 0xf>(I, v));
    v = fminf(v, dpp_keep_f32<0x118, 0xf>(I, v));
    v = fminf(v, dpp_keep_f32<0x142, 0xa>(I, v));
    v = fminf(v, dpp_keep_f32<0x143, 0xc>(I, v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_max_f32(float v) {
    const float I = -INFINITY;
    v = fmaxf(v, dpp_keep_f32<0x111, 0xf>(I, v));
    v = fmaxf(v, dpp_keep_f32<0x112, 0xf>(I, v));
    v = fmaxf(v, dpp_keep_f32<0x114, 0xf>(I, v));
    v = fmaxf(v, dpp_keep_f32<0x118, 0xf>(I, v));
    v = fmaxf(v, dpp_keep_f32<0x142, 0xa>(I, v));
    v = fmaxf(v, dpp_keep_f32<0x143, 0xc>(I, v));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// ---- one FP32C sub-step of one slice ------------------------------------------------
// idx_at(k) loads this lane's k-th neighbour reference, val_of(ref) returns the
// FP32 hi temperature it refers to.  The global-gather and LDS-tile kernels
// differ only in these two, so both produce bit-identical states.  The
// references of the next chunk of 8 are loaded before the current chunk is
// evaluated; terms are added in neighbour order.  The caller loads the
// lane's own low part, T^lat and source weight ahead of the neighbour loop and
// receives the lane's ledger terms (energy to the lattice, source, temperature
// ledger, per unit time) for its wave reduction.
struct LedgerTerms {
    float e2l, src, lt;
};

// coupling, source and state update of one lane, given the neighbour sum
// S = span * sum_j f(theta_i, theta_j) accumulated in FP64.  The state is
// (hi, q) with T = hi + q s(hi) (state_fp32c.h): the increment is added to T
// in FP64 and the sum split back into a rounded hi and its 16-bit remainder q.
__device__ __forceinline__ LedgerTerms finish_fp32c(const DevParams &p, int32_t slot, bool valid,
                                                    float Ti, double S, int16_t lo, float tl,
                                                    float sw, float *__restrict__ Thi_n,
                                                    int16_t *__restrict__ Tlo,
                                                    double *__restrict__ eatom, float qpulse,
                                                    unsigned *err) {
    float hi_new = Ti;
    LedgerTerms r{0.0f, 0.0f, 0.0f};
    if (valid) {
        const float c = ce32(p, Ti);
        // hardware reciprocal (within 1 ulp): it scales only the local terms,
        // whose own size is a small fraction of the state's FP32 resolution
        const float invc = __builtin_amdgcn_rcpf(c);
        const float coup = signbit(tl) ? 0.0f : p.f_g * (Ti - tl);
        float q = 0.0f;
        if (p.laser_on) q = qpulse * fabsf(sw);
        const float loc = (q - coup) * invc;
        if (eatom) eatom[slot] += (double)coup * p.dt;
        if (p.has_fixed && signbit(sw)) {
            // held: the exchange it would receive goes to the temperature ledger
            r = LedgerTerms{coup, q, (float)(p.K * S)};
        } else {
            const double T = state_value(Ti, lo) + p.dt * (p.K * S + (double)loc);
            hi_new = (float)T;
            Tlo[slot] = state_lo(T, hi_new);
            r = LedgerTerms{coup, q, -loc};
            if (!(hi_new >= p.f_T_min && hi_new <= p.f_T_max)) atomicOr(err, kErrRange);
        }
    }
    Thi_n[slot] = hi_new;
    return r;
}

template <class IdxAt, class ValOf>
__device__ __forceinline__ LedgerTerms slice_core_fp32c(const SliceInfo &si, int32_t sl, int lane,
                                                        const DevParams &p, float Ti, int16_t lo,
                                                        float tl, float sw, IdxAt idx_at,
                                                        ValOf val_of, float *__restrict__ Thi_n,
                                                        int16_t *__restrict__ Tlo,
                                                        double *__restrict__ eatom, float qpulse,
                                                        unsigned *err) {
    constexpr int C = 8;
    using Ref = decltype(idx_at(0));
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    const PairK pk = pair_consts(p);
    double S = 0.0;   // span * sum_j f(theta_i, theta_j), in row order
    const int32_t w = si.width;
    Ref cur[C], nxt[C];
#pragma unroll
    for (int u = 0; u < C; ++u) cur[u] = (u < w) ? idx_at(u) : Ref{};
    for (int32_t k0 = 0; k0 < w; k0 += C) {
#pragma unroll
        for (int u = 0; u < C; ++u) nxt[u] = (k0 + C + u < w) ? idx_at(k0 + C + u) : Ref{};
        float Tj[C];
#pragma unroll
        for (int u = 0; u < C; ++u) Tj[u] = (k0 + u < w) ? val_of(cur[u]) : Ti;
#pragma unroll
        for (int u = 0; u < C; ++u)
            if (k0 + u < w) S += (double)pair32(Ti, Tj[u], pk);
#pragma unroll
        for (int u = 0; u < C; ++u) cur[u] = nxt[u];
    }
    return finish_fp32c(p, slot, valid, Ti, S, lo, tl, sw, Thi_n, Tlo, eatom, qpulse, err);
}

// cache policy of the table loads: the default, or the non-temporal hint
// (the table is read once per sub-step)
constexpr int kTableCached = 0, kTableStream = 2;

// LDS-tile form for one slice.  TIERS = false: the caller has shown that every
// pair of the slice lies on the lowest tier of pair32 (it evaluates exactly
// that tier, bitwise what pair32 returns there).  w is the slice's row width and row the first
// word of its packed table (both wave-uniform).  Each word holds the LDS byte
// offsets of two neighbours; a chunk is 4 words = 8 neighbours.  The words of
// chunk c + 2 are requested once those of chunk c have been turned into LDS
// reads, alternating between two buffers.  Same terms in the same order as
// slice_core_fp32c.  POLICY: kTableCached or kTableStream for the row loads.
template <bool TIERS, int POLICY>
__device__ __forceinline__ LedgerTerms slice_core_brick(int32_t w, int32_t slot, bool valid,
                                                        const DevParams &p, float Ti, int16_t lo,
                                                        float tl, float sw,
                                                        const uint32_t *__restrict__ row,
                                                        int lane, const float *tile,
                                                        float *__restrict__ Thi_n,
                                                        int16_t *__restrict__ Tlo,
                                                        double *__restrict__ eatom, float qpulse,
                                                        unsigned *err) {
    const PairK pk = pair_consts(p);
    const char *tb = reinterpret_cast<const char *>(tile);
    const int32_t nwd = (w + 1) >> 1;
    const int32_t nch = (w + 7) >> 3;
    double S = 0.0;
    // The row is read through a buffer resource spanning exactly its nwd word
    // rows: the lane offset is a constant vector register and the word row a
    // scalar offset, so no vector instruction goes into addressing.  Word
    // indices past the row's end are clamped to its last word (a re-read of a
    // line just fetched), so every load is unconditional and inside the row.
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(row), 0, nwd * kWave * (int)sizeof(uint32_t), kBufferRsrcWord3);
    const int32_t lane_off = lane * (int)sizeof(uint32_t);
    auto load = [&](int32_t c, uint32_t (&d)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int32_t wi = min(4 * c + u, nwd - 1);
            d[u] = __builtin_amdgcn_raw_buffer_load_b32(rs, lane_off,
                                                        wi * kWave * (int)sizeof(uint32_t), POLICY);
        }
    };
    auto at = [&](uint32_t off) { return *reinterpret_cast<const float *>(tb + off); };
    auto term = [&](float Tj) {
        if constexpr (TIERS) {
            return pair32(Ti, Tj, pk);
        } else {
            const PairParts r = pair32_parts(Ti, Tj, pk);
            return r.dT * r.h;
        }
    };
    auto terms = [&](const float (&Tj)[8], float (&f)[8]) {
#pragma unroll
        for (int u = 0; u < 8; ++u) f[u] = term(Tj[u]);
    };
    // a full chunk c: LDS reads of its 8 neighbours (the offsets are consumed
    // here), then the request of chunk c + 2 into the same buffer, then the 8
    // pair terms; no per-neighbour condition
    auto full_chunk = [&](int32_t c, uint32_t (&d)[4]) {
        float Tj[8], f[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            Tj[2 * u] = at(d[u] & 0xffffu);
            Tj[2 * u + 1] = at(d[u] >> 16);
        }
        load(c + 2, d);
        terms(Tj, f);
#pragma unroll
        for (int u = 0; u < 8; ++u) S += (double)f[u];
    };
    // the row's last chunk when the width is not a multiple of 8: only its
    // entries inside the row are read and evaluated (wave-uniform conditions)
    auto tail_chunk = [&](int32_t c, const uint32_t (&d)[4]) {
        const int32_t m = w - 8 * c;
        float Tj[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < m) Tj[u] = at((u & 1) ? (d[u >> 1] >> 16) : (d[u >> 1] & 0xffffu));
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (u < m) S += (double)term(Tj[u]);
    };
    if (nch > 0) {
        uint32_t A[4], B[4];
        load(0, A);
        load(1, B);
        const int32_t nfull = w >> 3;
        int32_t c = 0;
        for (; c + 2 <= nfull; c += 2) {
            full_chunk(c, A);
            full_chunk(c + 1, B);
        }
        // chunk c (even) takes buffer A, c + 1 buffer B
        if (c < nfull) {
            full_chunk(c, A);
            if (c + 1 < nch) tail_chunk(c + 1, B);
        } else if (c < nch) {
            tail_chunk(c, A);
        }
    }
    return finish_fp32c(p, slot, valid, Ti, S, lo, tl, sw, Thi_n, Tlo, eatom, qpulse, err);
}

// wave sums of ledger terms, added in FP64 to one ledger row.  A row is
// updated by one wave per sub-step and the sub-steps are ordered launches, so
// the additions happen in a fixed order; the FP64 atomic only spares the wave
// the wait for the old value.
__device__ __forceinline__ void ledger_add(double *__restrict__ ledger, int32_t row_id, int lane,
                                           const LedgerTerms &t, double dt) {
    const double e2l = (double)wave_sum_f32(t.e2l) * dt;
    const double src = (double)wave_sum_f32(t.src) * dt;
    const double lt = (double)wave_sum_f32(t.lt) * dt;
    if (lane == 0) {
        double *row = ledger + 3 * (int64_t)row_id;
        unsafeAtomicAdd(row + 0, e2l);
        unsafeAtomicAdd(row + 1, src);
        unsafeAtomicAdd(row + 2, lt);
    }
}

// global-gather form over the int32 table (one slice)
__device__ __forceinline__ void slice_step_fp32c(const SliceInfo &si, int32_t sl, int lane,
                                                 const DevParams &p,
                                                 const int32_t *__restrict__ col,
                                                 const float *__restrict__ Thi,
                                                 float *__restrict__ Thi_n,
                                                 int16_t *__restrict__ Tlo,
                                                 const float *__restrict__ Tl,
                                                 const float *__restrict__ srcw, int64_t step,
                                                 double *__restrict__ ledger,
                                                 double *__restrict__ eatom, unsigned *err) {
    const int32_t slot = sl * kWave + lane;
    const int32_t *cp = col + (int64_t)si.col_base64 * kWave + lane;
    const float Ti = Thi[slot];
    const int16_t lo = Tlo[slot];
    const float tl = Tl[slot];
    const float sw = (p.laser_on | (si.flags & kSliceHeld)) ? srcw[slot] : 0.0f;
    const LedgerTerms t = slice_core_fp32c(
        si, sl, lane, p, Ti, lo, tl, sw, [&](int32_t k) { return cp[k * kWave]; },
        [&](int32_t j) { return Thi[j]; }, Thi_n, Tlo, eatom, source_factor32(p, step), err);
    ledger_add(ledger, sl, lane, t, p.dt);
}

}  // namespace dev
}  // namespace l2t
