// Discrete adjoint of the FP32C forward-Euler sub-step (derived from Eq. 2).
//
// Forward: T^{n+1} = T^n + dt R(T^n), with
//   R_k = (T_max - T_min) K sum_{j in N(k)} f(theta_k, theta_j)
//         - g_k (T_k - T_k^lat)/c_k + q_k(t_n)/c_k.
// Reverse: lambda^n = lambda^{n+1} + dt J(T^n)^T lambda^{n+1}.  Because the
// neighbour relation is symmetric and f(a, b) = -f(b, a),
//   (J^T lambda)_k = K sum_{j in N(k)} d1f(theta_k, theta_j) (lambda_k - lambda_j)
//                    + lambda_k d/dT_k[-g_k (T_k - T^lat_k)/c_k + q_k/c_k],
// a gather over the forward neighbour table (no atomics), with
//   d1f = -[(1 - 2m(1-m) - d^2/2) cosh d + (1 - 2m) sinh d],
//   d = theta_j - theta_k, m = (theta_k + theta_j)/2.
// Parameter gradients: dL/dK = sum_n dt sum_k lambda_k^{n+1} (T_max - T_min) S_k(T^n)
// (the kernels carry S in temperature units, (T_max - T_min) S),
// dL/dg = sum_n dt sum_k lambda_k^{n+1} (-gate_k (T_k - T^lat_k)/c_k).
//
// States between checkpoints are recomputed with the forward slice function
// itself, so they equal the forward states bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <vector>

#include "l2t_internal.h"
#include "step_device.h"

namespace l2t {
namespace {

using namespace dev;

// f and d1f of one pair from FP32 temperatures.  With d = theta_j - theta_k,
// u = d^2, s = 1 - 2m = 1 - theta_k - theta_j, C(u) = cosh d and
// Q(u) = sinh(d)/d, and since 2m(1-m) = (1 - s^2)/2, e = u - s^2 gives
//   f   = d [C - (u/2 + 2m(1-m)) Q]                 = d [C - (1 + e)/2 Q]
//   d1f = -[(1 - 2m(1-m) - u/2) C + (1 - 2m) d Q]   = -[(1 - e)/2 C + s d Q]
// (f is the pair term of Eq. 2, d1f its derivative in theta_k), so both come
// from one evaluation of C and Q.  f is returned in temperature units
// (span * f), as the forward sums it.  sk = s + T_j/span is the lane's own
// part of s.  C runs to u^5 and Q to u^4: for |d| <= 1 the dropped terms are
// below 3e-9 and 3e-8 (half an FP32 ulp of Q >= 1 is 6e-8).  One
// straight-line form for every pair measured faster than branching to shorter
// series for small u.
__device__ __forceinline__ float adj_sk(float Tk, const PairK &pk, float inv_span) {
    // theta = T/span + moff with moff = -T_min/span, so
    // s + T_j/span = 1 - 2 moff - T_k/span
    return fmaf(Tk, -inv_span, fmaf(-2.0f, pk.moff, 1.0f));
}

__device__ __forceinline__ void pair_adj(float Tk, float Tj, float sk, float inv_span, float &f,
                                         float &d1) {
    const float dT = Tj - Tk;
    const float d = dT * inv_span;
    const float u = d * d;
    const float s = fmaf(Tj, -inv_span, sk);
    const float e = fmaf(-s, s, u);
    float C = fmaf(u, 1.0f / 3628800.0f, 1.0f / 40320.0f);
    C = fmaf(u, C, 1.0f / 720.0f);
    C = fmaf(u, C, 1.0f / 24.0f);
    C = fmaf(u, C, 0.5f);
    C = fmaf(u, C, 1.0f);
    float Q = fmaf(u, 1.0f / 362880.0f, 1.0f / 5040.0f);
    Q = fmaf(u, Q, 1.0f / 120.0f);
    Q = fmaf(u, Q, 1.0f / 6.0f);
    Q = fmaf(u, Q, 1.0f);
    // with h = (1 + e)/2, (1 - e)/2 = 1 - h: f = dT (C - h Q), d1f = -(C - h C + s d Q)
    const float h = fmaf(e, 0.5f, 0.5f);
    f = dT * fmaf(-h, Q, C);
    d1 = -fmaf(s * d, Q, fmaf(-h, C, C));
}

// the terms of two consecutive row entries (2m, 2m + 1) added to the lane's
// FP64 sums S and D: the pair's two f, and its two d1f (lambda_k - lambda_j),
// are summed in FP32 first, so each FP64 sum takes one addition per two
// entries.  Every form calls this on the same entry pairs in the same order.
__device__ __forceinline__ void two_terms(float Tk, float lk, float sk, float inv_span, float Tj0,
                                          float lj0, float Tj1, float lj1, double &S, double &D) {
    float f0, d0, f1, d1;
    pair_adj(Tk, Tj0, sk, inv_span, f0, d0);
    pair_adj(Tk, Tj1, sk, inv_span, f1, d1);
    S += (double)(f0 + f1);
    D += (double)fmaf(d1, lk - lj1, d0 * (lk - lj0));
}

// the term of a row's last entry when the row length is odd
__device__ __forceinline__ void one_term(float Tk, float lk, float sk, float inv_span, float Tj,
                                         float lj, double &S, double &D) {
    float f, d1;
    pair_adj(Tk, Tj, sk, inv_span, f, d1);
    S += (double)f;
    D += (double)(d1 * (lk - lj));
}

struct AdjGrad {
    double k, g;
};

// reverse update of one lane given S = span * sum_j f and D = sum_j d1f
// (lambda_k - lambda_j), accumulated in FP64 in row order, two entries at a
// time.  lambda is the FP32 pair (hi, lo) with hi + lo exact in FP64; the
// increment is added in FP64 and the sum split back, as the forward does with
// T.  Returns this lane's terms of dL/dK and dL/dg.
__device__ __forceinline__ AdjGrad adjoint_finish(const DevParams &p, bool valid, int32_t slot,
                                                  float Tk, float lk, double S, double D,
                                                  const float *__restrict__ Tl,
                                                  const float *__restrict__ srcw,
                                                  float *__restrict__ lam_n,
                                                  float *__restrict__ lam_lo, int64_t step) {
    float l_new = lk;
    AdjGrad r{0.0, 0.0};
    if (valid) {
        const float tl = Tl[slot];
        const bool gated = signbit(tl);
        const float c = ce32(p, Tk);
        float cpr = 0.0f;
        if (p.ce_model == L2T_CE_LINEAR || (p.ce_model == L2T_CE_CAPPED && p.f_gamma * Tk <= p.f_ce_cap))
            cpr = p.f_gamma;
        const float ge = gated ? 0.0f : p.f_g;
        float q = 0.0f;
        if (p.laser_on) q = (p.f_i0 * pulse32(p, step)) * srcw[slot];
        const float invc = 1.0f / c;
        const float dloc = -ge * invc + (ge * (Tk - tl) - q) * cpr * invc * invc;
        const double lfull = (double)lk + (double)lam_lo[slot];
        const double ln = lfull + p.dt * (p.K * D + (double)(lk * dloc));
        l_new = (float)ln;
        lam_lo[slot] = (float)(ln - (double)l_new);
        r.k = lfull * p.dt * S;
        r.g = gated ? 0.0 : -lfull * p.dt * (double)(Tk - tl) * (double)invc;
    }
    lam_n[slot] = l_new;
    return r;
}

// global-gather form: one wave per slice, neighbours through the int32 table
__global__ __launch_bounds__(256) void k_adjoint_step(
    const SliceInfo *__restrict__ slices, int32_t n_slices, const int32_t *__restrict__ col,
    const float *__restrict__ Thi, const float *__restrict__ Tl, const float *__restrict__ srcw,
    const DevParams *__restrict__ P, const int64_t *__restrict__ dstep, int32_t rel,
    const float *__restrict__ lam, float *__restrict__ lam_n, float *__restrict__ lam_lo,
    double *__restrict__ grad /*[n_slices][2]*/) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t sl = blockIdx.x * (blockDim.x / kWave) + wave;
    if (sl >= n_slices) return;
    const SliceInfo si = slices[sl];
    const DevParams &p = P[si.sys];
    const int32_t slot = sl * kWave + lane;
    const float Tk = Thi[slot];
    const float lk = lam[slot];
    const int32_t *cp = col + (int64_t)si.col_base64 * kWave + lane;
    const PairK pk = pair_consts(p);
    const float sk = adj_sk(Tk, pk, p.f_inv_span);
    double S = 0.0, D = 0.0;
    const int32_t full = si.width >> 1;
    for (int32_t m = 0; m < full; ++m) {
        const int32_t j0 = cp[(2 * m) * kWave], j1 = cp[(2 * m + 1) * kWave];
        two_terms(Tk, lk, sk, p.f_inv_span, Thi[j0], lam[j0], Thi[j1], lam[j1], S, D);
    }
    if (si.width & 1) {
        const int32_t j = cp[(si.width - 1) * kWave];
        one_term(Tk, lk, sk, p.f_inv_span, Thi[j], lam[j], S, D);
    }
    const AdjGrad g = adjoint_finish(p, lane < si.n_valid, slot, Tk, lk, S, D, Tl, srcw, lam_n,
                                     lam_lo, dstep[si.sys] + rel);
    const double gK = wave_sum(g.k), gG = wave_sum(g.g);
    if (lane == 0) {
        grad[2 * (int64_t)sl + 0] += gK;
        grad[2 * (int64_t)sl + 1] += gG;
    }
}

// LDS-brick form: one workgroup per brick stages T^n and lambda^{n+1} of the
// brick's slots and of its halo list in two tiles; the slices then read both
// through the uint16 table (the byte offset of atom j in the T tile; lambda_j
// sits LAM floats further, a constant multiple of 64 floats, so the two reads
// of a neighbour are one two-address LDS instruction on one vector address).
// Same terms in the same order as k_adjoint_step, so lambda is bitwise equal;
// the gradient terms are summed per lane over the wave's slices and added
// once per wave to the row of its first slice.
template <int LAM>
__global__ __launch_bounds__(kBrickBlockMax) void k_adjoint_brick(
    const BrickInfo *__restrict__ bricks, const int32_t *__restrict__ list, int32_t n_list,
    const SliceInfo *__restrict__ slices, const uint32_t *__restrict__ colw,
    const int32_t *__restrict__ halo, const float *__restrict__ Thi,
    const float *__restrict__ Tl, const float *__restrict__ srcw, const DevParams *__restrict__ P,
    const int64_t *__restrict__ dstep, int32_t rel, const float *__restrict__ lam,
    float *__restrict__ lam_n, float *__restrict__ lam_lo, double *__restrict__ grad) {
    extern __shared__ __align__(16) float tile[];
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned logical = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    if ((int32_t)logical >= n_list) return;
    const int32_t gb = list[logical];
    if (gb < 0) return;   // a hole of the XCD launch list
    const BrickInfo bi = bricks[gb];
    float *lt = tile + LAM;
    const int32_t B = blockDim.x;
    // both tiles four slots at a time, as the forward brick kernel stages its
    // tile: own slots contiguous and 64-aligned, the halo list 16-byte aligned
    // and padded to a multiple of 4 with copies of its last entry; the second
    // quad of a pass is clamped to the last one (the same values again)
    const char *t_in = reinterpret_cast<const char *>(Thi);
    const char *l_in = reinterpret_cast<const char *>(lam);
    auto at = [](const char *base, int32_t slot) {
        return *reinterpret_cast<const float *>(base + (uint32_t)slot * 4u);
    };
    {
        const int32_t nq = bi.n_own_pad >> 2;
        const float4 *ts = reinterpret_cast<const float4 *>(Thi + bi.slot0);
        const float4 *ls = reinterpret_cast<const float4 *>(lam + bi.slot0);
        float4 *td = reinterpret_cast<float4 *>(tile), *ld = reinterpret_cast<float4 *>(lt);
        for (int32_t q0 = threadIdx.x; q0 < nq; q0 += 2 * B) {
            const int32_t q1 = min(q0 + B, nq - 1);
            const float4 a = ts[q0], c = ts[q1], la = ls[q0], lc = ls[q1];
            td[q0] = a;
            td[q1] = c;
            ld[q0] = la;
            ld[q1] = lc;
        }
        const int32_t nh = halo_padded(bi.n_halo) >> 2;
        const int4 *hl = reinterpret_cast<const int4 *>(halo + bi.halo_off);
        float4 *th = reinterpret_cast<float4 *>(tile + bi.n_own_pad);
        float4 *lh = reinterpret_cast<float4 *>(lt + bi.n_own_pad);
        for (int32_t q0 = threadIdx.x; q0 < nh; q0 += 2 * B) {
            const int32_t q1 = min(q0 + B, nh - 1);
            const int4 ia = hl[q0], ic = hl[q1];
            const float4 a = make_float4(at(t_in, ia.x), at(t_in, ia.y), at(t_in, ia.z), at(t_in, ia.w));
            const float4 c = make_float4(at(t_in, ic.x), at(t_in, ic.y), at(t_in, ic.z), at(t_in, ic.w));
            const float4 la = make_float4(at(l_in, ia.x), at(l_in, ia.y), at(l_in, ia.z), at(l_in, ia.w));
            const float4 lc = make_float4(at(l_in, ic.x), at(l_in, ic.y), at(l_in, ic.z), at(l_in, ic.w));
            th[q0] = a;
            th[q1] = c;
            lh[q0] = la;
            lh[q1] = lc;
        }
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const int lane = threadIdx.x % kWave;
    const int nw = blockDim.x / kWave;
    const int32_t ns = bi.n_own_pad / kWave;
    if (wave >= ns) return;
    const DevParams &p = P[bi.sys];
    const int64_t step = dstep[bi.sys] + rel;
    const PairK pk = pair_consts(p);
    const char *tb = reinterpret_cast<const char *>(tile);
    double gK = 0.0, gG = 0.0;
    for (int32_t q = wave; q < ns; q += nw) {
        const int32_t sl = bi.slice0 + q;
        const int32_t w = __builtin_amdgcn_readfirstlane(slices[sl].width);
        const int32_t nv = __builtin_amdgcn_readfirstlane(slices[sl].n_valid);
        const int32_t base = __builtin_amdgcn_readfirstlane(slices[sl].colw_base64);
        const int32_t slot = sl * kWave + lane;
        const float Tk = tile[q * kWave + lane];
        const float lk = lt[q * kWave + lane];
        const float sk = adj_sk(Tk, pk, p.f_inv_span);
        const uint32_t *row = colw + (int64_t)base * kWave + lane;
        double S = 0.0, D = 0.0;
        auto Tat = [&](uint32_t off) { return *reinterpret_cast<const float *>(tb + off); };
        auto lat = [&](uint32_t off) { return *reinterpret_cast<const float *>(tb + off + 4 * LAM); };
        const int32_t full = w >> 1;
#pragma unroll 2
        for (int32_t k = 0; k < full; ++k) {   // one word: entries 2k and 2k + 1
            const uint32_t wd = row[(int64_t)k * kWave];
            const uint32_t o0 = wd & 0xffffu, o1 = wd >> 16;
            two_terms(Tk, lk, sk, p.f_inv_span, Tat(o0), lat(o0), Tat(o1), lat(o1), S, D);
        }
        if (w & 1) {
            const uint32_t o = row[(int64_t)full * kWave] & 0xffffu;
            one_term(Tk, lk, sk, p.f_inv_span, Tat(o), lat(o), S, D);
        }
        const AdjGrad g = adjoint_finish(p, lane < nv, slot, Tk, lk, S, D, Tl, srcw, lam_n,
                                         lam_lo, step);
        gK += g.k;
        gG += g.g;
    }
    gK = wave_sum(gK);
    gG = wave_sum(gG);
    if (lane == 0) {
        grad[2 * (int64_t)(bi.slice0 + wave) + 0] += gK;
        grad[2 * (int64_t)(bi.slice0 + wave) + 1] += gG;
    }
}

__global__ void k_lambda_in(const int32_t *perm, int32_t n_int, const double *w, float *hi,
                            float *lo) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_int) return;
    int32_t g = perm[s];
    double v = g >= 0 ? w[g] : 0.0;
    float h = (float)v;
    hi[s] = h;
    lo[s] = (float)(v - (double)h);
}

__global__ void k_lambda_out(const int32_t *perm, int32_t n_int, const float *hi, const float *lo,
                             double *out) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_int) return;
    int32_t g = perm[s];
    if (g >= 0) out[g] = (double)hi[s] + (double)lo[s];
}

__global__ void k_grad_reduce(const SliceInfo *slices, int32_t n_slices, const double *grad,
                              int32_t sys, int32_t slice0, int32_t ns, double *out) {
    __shared__ double a[2][256];
    const int t = threadIdx.x;
    double k = 0.0, g = 0.0;
    for (int32_t q = t; q < ns; q += blockDim.x) {
        k += grad[2 * (int64_t)(slice0 + q) + 0];
        g += grad[2 * (int64_t)(slice0 + q) + 1];
    }
    a[0][t] = k;
    a[1][t] = g;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) {
            a[0][t] += a[0][t + w];
            a[1][t] += a[1][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[2 * sys + 0] = a[0][0];
        out[2 * sys + 1] = a[1][0];
    }
    (void)slices;
    (void)n_slices;
}

__global__ void k_forward_step(const SliceInfo *slices, int32_t n_slices, const int32_t *col,
                               const float *Thi, float *Thi_n, int16_t *Tlo, const float *Tl,
                               const float *srcw, const DevParams *P, const int64_t *dstep,
                               int32_t rel, double *ledger, unsigned *err) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t sl = blockIdx.x * (blockDim.x / kWave) + wave;
    if (sl >= n_slices) return;
    const SliceInfo si = slices[sl];
    slice_step_fp32c(si, sl, lane, P[si.sys], col, Thi, Thi_n, Tlo, Tl, srcw,
                     dstep[si.sys] + rel, ledger, nullptr, err);
}

__global__ void k_zero_d(double *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int record_checkpoint(l2t_ctx *c, int64_t k) {
    const size_t NI = (size_t)c->n_int;
    float *dst = (float *)c->rec.buf + (size_t)k * 2 * NI;
    L2T_HIP(c, hipMemcpyAsync(dst, c->Thi[c->cur], sizeof(float) * NI, hipMemcpyDeviceToDevice,
                              c->stream));
    L2T_HIP(c, hipMemcpyAsync(dst + NI, c->Tlo, sizeof(int16_t) * NI, hipMemcpyDeviceToDevice,
                              c->stream));
    return L2T_OK;
}

int adjoint(l2t_ctx *c, const double *w, double *dL_dK, double *dL_dg, double *dL_dT0) {
    const Recording &r = c->rec;
    const size_t NI = (size_t)c->n_int, NS = (size_t)c->n_slices, S = c->sys.size();
    const int32_t C = r.ckpt;
    // scratch: segment states [C][hi, lo], lambda hi x2 + lo, ledger, grads, dstep, outputs
    const size_t seg_f = (size_t)C * 2 * NI;
    const size_t nck = (size_t)r.n_ckpt;
    const size_t bytes = sizeof(float) * (seg_f + 3 * NI) +
                         sizeof(double) * (3 * NS + 2 * NS + 2 * S) +
                         sizeof(int64_t) * S * (1 + nck) + 256;
    if (ensure_scratch(c, bytes) != L2T_OK) return L2T_ENOMEM;
    char *p = (char *)c->scratch;
    float *seg = (float *)p;
    p += sizeof(float) * seg_f;
    float *lam0 = (float *)p;
    p += sizeof(float) * NI;
    float *lam1 = (float *)p;
    p += sizeof(float) * NI;
    float *lamlo = (float *)p;
    p += sizeof(float) * NI;
    double *led = (double *)p;
    p += sizeof(double) * 3 * NS;
    double *grad = (double *)p;
    p += sizeof(double) * 2 * NS;
    double *gout = (double *)p;
    p += sizeof(double) * 2 * S;
    int64_t *dst = (int64_t *)p;
    int64_t *dtab = dst + S;   // step counters at the start of every segment [n_ckpt][S]
    float *lam[2] = {lam0, lam1};
    int lc = 0;
    const hipStream_t s_ = c->stream;
    hipLaunchKernelGGL(k_lambda_in, dim3(nblk(NI, 256)), dim3(256), 0, s_, c->perm, c->n_int, w,
                       lam[0], lamlo);
    hipLaunchKernelGGL(k_zero_d, dim3(nblk(2 * NS, 256)), dim3(256), 0, s_, grad, (int64_t)(2 * NS));
    hipLaunchKernelGGL(k_zero_d, dim3(nblk(3 * NS, 256)), dim3(256), 0, s_, led, (int64_t)(3 * NS));
    const dim3 g(nblk(NS, 4)), b(256);
    // the brick forms when the tuned forward is the brick kernel and both
    // tiles of the reverse step fit in 64 KB of LDS: the lambda tile starts
    // 4096 or 8192 floats after the T tile
    const bool brick = c->tune.kernel == kKernelBrick && c->n_brick_list > 0 &&
                       c->tile_max <= 8192;
    const bool lam_near = c->tile_max <= 4096;
    // the recomputation runs the forward's tuned block; the reverse step always
    // takes the largest: a CU holds as many workgroups as their tiles fit in
    // LDS, so larger workgroups keep more waves resident (adjoint 142 ms at
    // 512 threads against 159 ms at 256 on the 64 x 32,000-atom workload)
    const int bblock = std::min(std::max(c->tune.block, kWave), kBrickBlockMax);
    const int rblock = kBrickBlockMax;
    const unsigned bgrid = (unsigned)c->n_xcd_list;
    const size_t blds = sizeof(float) * ((lam_near ? 4096 : 8192) + (size_t)c->tile_max);
    std::vector<int64_t> htab(nck * S);
    for (size_t k = 0; k < nck; ++k)
        for (size_t q = 0; q < S; ++q) htab[k * S + q] = r.step0[q] + (int64_t)k * C;
    L2T_HIP(c, hipMemcpyAsync(dtab, htab.data(), sizeof(int64_t) * htab.size(),
                              hipMemcpyHostToDevice, s_));
    // the sub-steps of one checkpoint segment: the recomputation of states
    // 1..L-1 from the segment's checkpoint, then L reverse sub-steps from
    // lambda buffer `l0`.  Captured once per (L, l0) for this call and replayed
    // for every segment of that length; the checkpoint copy and the step
    // counters go in before each replay.
    auto segment = [&](int32_t L, int l0) -> int {
        int lc2 = l0;
        for (int32_t m = 0; m + 1 < L; ++m) {
            float *in = seg + (size_t)m * 2 * NI, *out = seg + (size_t)(m + 1) * 2 * NI;
            // each state is [hi: NI floats][q: NI int16 in a region of NI floats]
            int16_t *qin = reinterpret_cast<int16_t *>(in + NI);
            int16_t *qout = reinterpret_cast<int16_t *>(out + NI);
            if (brick) {
                int rc = brick_step_fp32c(c, bblock, in, out, qin, qout, dst, m, led);
                if (rc != L2T_OK) return rc;
            } else {
                L2T_HIP(c, hipMemcpyAsync(qout, qin, sizeof(int16_t) * NI,
                                          hipMemcpyDeviceToDevice, c->stream));
                hipLaunchKernelGGL(k_forward_step, g, b, 0, c->stream, c->slices, c->n_slices,
                                   c->col, in, out, qout, c->Tl32, c->srcw32, c->dparams, dst,
                                   m, led, c->derr);
            }
        }
        for (int32_t m = L - 1; m >= 0; --m) {
            const float *Tst = seg + (size_t)m * 2 * NI;
            if (brick)
                hipLaunchKernelGGL(lam_near ? k_adjoint_brick<4096> : k_adjoint_brick<8192>,
                                   dim3(bgrid), dim3(rblock), blds, c->stream, c->bricks,
                                   xcd_list_for(c, m), c->n_xcd_list, c->slices, c->colw, c->halo,
                                   Tst, c->Tl32, c->srcw32, c->dparams, dst, m, lam[lc2],
                                   lam[lc2 ^ 1], lamlo, grad);
            else
                hipLaunchKernelGGL(k_adjoint_step, g, b, 0, c->stream, c->slices, c->n_slices,
                                   c->col, Tst, c->Tl32, c->srcw32, c->dparams, dst, m, lam[lc2],
                                   lam[lc2 ^ 1], lamlo, grad);
            lc2 ^= 1;
        }
        L2T_HIP(c, hipGetLastError());
        return L2T_OK;
    };
    // executable graphs of this call; on every way out the stream is drained
    // before they are destroyed
    struct Graphs {
        hipStream_t s;
        std::map<std::pair<int32_t, int>, hipGraphExec_t> m;
        ~Graphs() {
            if (m.empty()) return;
            (void)hipStreamSynchronize(s);
            for (auto &kv : m) (void)hipGraphExecDestroy(kv.second);
        }
    } graphs{s_, {}};
    for (int64_t k = r.n_ckpt - 1; k >= 0; --k) {
        const int64_t start = k * C;
        const int32_t L = (int32_t)std::min<int64_t>(C, r.n_steps - start);
        const float *ck = (const float *)r.buf + (size_t)k * 2 * NI;
        L2T_HIP(c, hipMemcpyAsync(seg, ck, sizeof(float) * 2 * NI, hipMemcpyDeviceToDevice, s_));
        L2T_HIP(c, hipMemcpyAsync(dst, dtab + (size_t)k * S, sizeof(int64_t) * S,
                                  hipMemcpyDeviceToDevice, s_));
        if (c->tune.graph == 0) {   // graph replays unless switched off
            int rc = segment(L, lc);
            if (rc != L2T_OK) return rc;
        } else {
            auto it = graphs.m.find({L, lc});
            if (it == graphs.m.end()) {
                if (!c->cap_stream)
                    L2T_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
                hipGraph_t gr = nullptr;
                L2T_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
                c->stream = c->cap_stream;
                int rc = segment(L, lc);
                c->stream = s_;
                hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
                if (rc != L2T_OK || e != hipSuccess) {
                    if (gr) (void)hipGraphDestroy(gr);
                    return rc != L2T_OK ? rc : hip_fail(c, e, "hipStreamEndCapture");
                }
                hipGraphExec_t ge = nullptr;
                e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
                (void)hipGraphDestroy(gr);
                if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
                it = graphs.m.emplace(std::make_pair(L, lc), ge).first;
            }
            L2T_HIP(c, hipGraphLaunch(it->second, s_));
        }
        if (L & 1) lc ^= 1;
    }
    for (size_t q = 0; q < S; ++q) {
        const SystemState &st = c->sys[q];
        hipLaunchKernelGGL(k_grad_reduce, dim3(1), dim3(256), 0, s_, c->slices, c->n_slices, grad,
                           (int32_t)q, st.slice0, st.n_slices, gout);
    }
    if (dL_dT0)
        hipLaunchKernelGGL(k_lambda_out, dim3(nblk(NI, 256)), dim3(256), 0, s_, c->perm, c->n_int,
                           lam[lc], lamlo, dL_dT0);
    L2T_HIP(c, hipGetLastError());
    std::vector<double> h(2 * S);
    L2T_HIP(c, hipMemcpyAsync(h.data(), gout, sizeof(double) * 2 * S, hipMemcpyDeviceToHost, s_));
    L2T_HIP(c, hipStreamSynchronize(s_));
    for (size_t q = 0; q < S; ++q) {
        dL_dK[q] = h[2 * q];
        dL_dg[q] = h[2 * q + 1];
    }
    return L2T_OK;
}

}  // namespace l2t
