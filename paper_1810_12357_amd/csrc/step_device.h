// Device-side building blocks of the sub-step: reductions, heat capacity,
// the FP32 product-form pair term and its derivative, and the per-slice
// FP64 / FP32C sub-step bodies.  Included by the forward kernels and by the
// adjoint, which recomputes forward states with exactly these functions.
#pragma once

#include <hip/hip_runtime.h>

#include "l2t_internal.h"

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

// Gaussian time factor of Eq. 9 at the start of sub-step `step`
__device__ inline double pulse64(const DevParams &p, int64_t step) {
    double t = (double)step * p.dt - p.t0;
    return exp(-t * t / (2.0 * p.sigma * p.sigma));
}
__device__ inline float pulse32(const DevParams &p, int64_t step) {
    const float x = (float)(((double)step * p.dt - p.t0) * p.inv_sigma);
    return expf(-0.5f * x * x);
}

// ---- FP32 pair term -------------------------------------------------------------
// With d = theta_j - theta_i and m = (theta_i + theta_j)/2 the pair term of
// Eq. 2 equals d [cosh d - (2 m (1 - m) + d^2/2) sinh(d)/d].  Writing u = d^2,
// cosh d - (u/2) sinh(d)/d = sum_k (1 - k) u^k / (2k)! =: P(u) and
// sinh(d)/d = sum_k u^k / (2k+1)! =: Q(u), so f = d (P(u) - 2 m (1 - m) Q(u)).
// Both series are truncated below half an FP32 ulp of h for |d| <= 1; for
// u <= 1e-2 the short forms are used.  h depends on (m, u) only, both
// symmetric in (i, j), so f(i, j) = -f(j, i) holds bitwise.
__device__ __forceinline__ float pair32(float Ti, float Tj, float inv_span, float half_inv_span,
                                        float m_off) {
    const float d = (Tj - Ti) * inv_span;
    const float m = fmaf(Ti + Tj, half_inv_span, m_off);
    const float a = fmaf(-m, m, m);
    const float u = d * d;
    float P, Q2;   // Q2 = -2 Q
    if (u <= 1.0e-2f) {
        P = fmaf(u * u, fmaf(u, -1.0f / 360.0f, -1.0f / 24.0f), 1.0f);
        Q2 = fmaf(u, fmaf(u, -2.0f / 120.0f, -2.0f / 6.0f), -2.0f);
    } else {
        float p = fmaf(u, -5.0f / 479001600.0f, -4.0f / 3628800.0f);
        p = fmaf(u, p, -3.0f / 40320.0f);
        p = fmaf(u, p, -1.0f / 360.0f);
        p = fmaf(u, p, -1.0f / 24.0f);
        P = fmaf(u * u, p, 1.0f);
        float q = fmaf(u, -2.0f / 39916800.0f, -2.0f / 362880.0f);
        q = fmaf(u, q, -2.0f / 5040.0f);
        q = fmaf(u, q, -2.0f / 120.0f);
        q = fmaf(u, q, -2.0f / 6.0f);
        Q2 = fmaf(u, q, -2.0f);
    }
    const float h = fmaf(a, Q2, P);
    return d * h;
}

// ---- one FP64 plain sub-step of one slice ---------------------------------------
__device__ inline void slice_step_fp64(const SliceInfo &si, int32_t sl, int lane,
                                       const DevParams &p, const int32_t *__restrict__ col,
                                       const double *__restrict__ T, double *__restrict__ Tn,
                                       const double *__restrict__ Tl,
                                       const double *__restrict__ srcw, int64_t step,
                                       double *__restrict__ ledger, unsigned *err) {
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    const double Ti = T[slot];
    const double ti = (Ti - p.T_min) * p.inv_span;
    const int64_t base = (int64_t)si.col_base64 * kWave + lane;
    double S = 0.0;
    for (int32_t k = 0; k < si.width; ++k) {
        const int32_t j = col[base + (int64_t)k * kWave];
        const double tj = (T[j] - p.T_min) * p.inv_span;
        S += tj * (1.0 - ti) * exp(ti - tj) - ti * (1.0 - tj) * exp(tj - ti);
    }
    double e2l = 0.0, q = 0.0, lt = 0.0, Tnew = Ti;
    if (valid) {
        const double c = ce64(p, Ti);
        const double tl = Tl[slot];
        const double coup = signbit(tl) ? 0.0 : p.g * (Ti - tl);
        if (p.laser_on) q = p.i0 * srcw[slot] * pulse64(p, step);
        Tnew = Ti + p.dt * (p.A * S - coup / c + q / c);
        e2l = coup * p.dt;
        lt = p.dt * (coup - q) / c;
        q *= p.dt;
        const double th = (Tnew - p.T_min) * p.inv_span;
        if (!(th >= 0.0 && th <= 1.0)) atomicOr(err, kErrRange);
    }
    Tn[slot] = Tnew;
    e2l = wave_sum(e2l);
    q = wave_sum(q);
    lt = wave_sum(lt);
    if (lane == 0) {
        ledger[3 * (int64_t)sl + 0] += e2l;
        ledger[3 * (int64_t)sl + 1] += q;
        ledger[3 * (int64_t)sl + 2] += lt;
    }
}

// ---- one FP32C sub-step of one slice ------------------------------------------------
__device__ __forceinline__ void slice_step_fp32c(const SliceInfo &si, int32_t sl, int lane,
                                                 const DevParams &p,
                                                 const int32_t *__restrict__ col,
                                                 const float *__restrict__ Thi,
                                                 float *__restrict__ Thi_n,
                                                 float *__restrict__ Tlo,
                                                 const float *__restrict__ Tl,
                                                 const float *__restrict__ srcw, int64_t step,
                                                 double *__restrict__ ledger, unsigned *err) {
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    const float Ti = Thi[slot];
    const int32_t *cp = col + (int64_t)si.col_base64 * kWave + lane;
    const float inv = p.f_inv_span, hinv = p.f_half_inv_span, moff = p.f_m_off;
    float S = 0.0f, comp = 0.0f;
    int32_t k = 0;
    const int32_t w = si.width;
    // batches of 4 neighbours: issue the index and temperature loads first
    for (; k + 4 <= w; k += 4) {
        const int32_t j0 = cp[(k + 0) * kWave], j1 = cp[(k + 1) * kWave];
        const int32_t j2 = cp[(k + 2) * kWave], j3 = cp[(k + 3) * kWave];
        const float T0 = Thi[j0], T1 = Thi[j1], T2 = Thi[j2], T3 = Thi[j3];
        const float f[4] = {pair32(Ti, T0, inv, hinv, moff), pair32(Ti, T1, inv, hinv, moff),
                            pair32(Ti, T2, inv, hinv, moff), pair32(Ti, T3, inv, hinv, moff)};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float y = f[q] - comp;
            const float t = S + y;
            comp = (t - S) - y;
            S = t;
        }
    }
    for (; k < w; ++k) {
        const float f = pair32(Ti, Thi[cp[k * kWave]], inv, hinv, moff);
        const float y = f - comp;
        const float t = S + y;
        comp = (t - S) - y;
        S = t;
    }
    float hi_new = Ti;
    double e2l = 0.0, qd = 0.0, lt = 0.0;
    if (valid) {
        const float lo = Tlo[slot];
        const float tl = Tl[slot];
        const float c = ce32(p, Ti);
        const float invc = 1.0f / c;
        const float coup = signbit(tl) ? 0.0f : p.f_g * (Ti - tl);
        float q = 0.0f;
        if (p.laser_on) q = (p.f_i0 * pulse32(p, step)) * srcw[slot];
        const float loc = (q - coup) * invc;
        const float dT = p.f_dt * fmaf(p.f_A, S, loc);
        // (hi, lo) + dT without rounding error: TwoSum then renormalise
        const float s = Ti + dT;
        const float bp = s - Ti;
        const float er = (Ti - (s - bp)) + (dT - bp);
        const float lo2 = lo + er;
        hi_new = s + lo2;
        const float lo_new = lo2 - (hi_new - s);
        Tlo[slot] = lo_new;
        e2l = (double)coup * p.dt;
        qd = (double)q * p.dt;
        lt = -(double)loc * p.dt;
        if (!(hi_new >= p.f_T_min && hi_new <= p.f_T_max)) atomicOr(err, kErrRange);
    }
    Thi_n[slot] = hi_new;
    e2l = wave_sum(e2l);
    qd = wave_sum(qd);
    lt = wave_sum(lt);
    if (lane == 0) {
        ledger[3 * (int64_t)sl + 0] += e2l;
        ledger[3 * (int64_t)sl + 1] += qd;
        ledger[3 * (int64_t)sl + 2] += lt;
    }
}

}  // namespace dev
}  // namespace l2t
