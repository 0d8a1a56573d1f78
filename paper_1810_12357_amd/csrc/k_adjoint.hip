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
#include <vector>

#include "l2t_internal.h"
#include "step_device.h"

namespace l2t {
namespace {

using namespace dev;

// f and d1f of one pair from FP32 temperatures (same d, m, u as pair32)
// f is returned in temperature units (span * f), as the forward sums it
__device__ __forceinline__ void pair32_with_d1(float Tk, float Tj, const PairK &pk,
                                               float inv_span, float *f, float *d1) {
    *f = pair32(Tk, Tj, pk);
    const float d = (Tj - Tk) * inv_span;
    const float m = fmaf(Tk + Tj, pk.hinv, pk.moff);
    const float u = d * d;
    // cosh d = sum u^k/(2k)!,  sinh(d)/d = sum u^k/(2k+1)!
    float ch = fmaf(u, 1.0f / 3628800.0f, 1.0f / 40320.0f);
    ch = fmaf(u, ch, 1.0f / 720.0f);
    ch = fmaf(u, ch, 1.0f / 24.0f);
    ch = fmaf(u, ch, 0.5f);
    ch = fmaf(u, ch, 1.0f);
    float sq = fmaf(u, 1.0f / 39916800.0f, 1.0f / 362880.0f);
    sq = fmaf(u, sq, 1.0f / 5040.0f);
    sq = fmaf(u, sq, 1.0f / 120.0f);
    sq = fmaf(u, sq, 1.0f / 6.0f);
    sq = fmaf(u, sq, 1.0f);
    const float cm = fmaf(2.0f * m, m - 1.0f, 1.0f);   // 1 - 2 m (1 - m)
    *d1 = -fmaf(cm - 0.5f * u, ch, (1.0f - 2.0f * m) * (d * sq));
}

__global__ __launch_bounds__(256) void k_adjoint_step(
    const SliceInfo *slices, int32_t n_slices, const int32_t *col, const float *Thi,
    const float *Tl, const float *srcw, const DevParams *P, const int64_t *dstep, int32_t rel,
    const float *lam, float *lam_n, float *lam_lo, double *grad /*[n_slices][2]*/) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int32_t sl = blockIdx.x * (blockDim.x / kWave) + wave;
    if (sl >= n_slices) return;
    const SliceInfo si = slices[sl];
    const DevParams &p = P[si.sys];
    const int32_t slot = sl * kWave + lane;
    const bool valid = lane < si.n_valid;
    const float Tk = Thi[slot];
    const float lk = lam[slot];
    const int32_t *cp = col + (int64_t)si.col_base64 * kWave + lane;
    const PairK pk = pair_consts(p);
    float S = 0.0f, cS = 0.0f, D = 0.0f, cD = 0.0f;
    for (int32_t q = 0; q < si.width; ++q) {
        const int32_t j = cp[q * kWave];
        float f, d1;
        pair32_with_d1(Tk, Thi[j], pk, p.f_inv_span, &f, &d1);
        const float term = d1 * (lk - lam[j]);
        float y = f - cS, t = S + y;
        cS = (t - S) - y;
        S = t;
        y = term - cD;
        t = D + y;
        cD = (t - D) - y;
        D = t;
    }
    float l_new = lk;
    double gK = 0.0, gG = 0.0;
    if (valid) {
        const float tl = Tl[slot];
        const bool gated = signbit(tl);
        const float c = ce32(p, Tk);
        float cpr = 0.0f;
        if (p.ce_model == L2T_CE_LINEAR || (p.ce_model == L2T_CE_CAPPED && p.f_gamma * Tk <= p.f_ce_cap))
            cpr = p.f_gamma;
        const float ge = gated ? 0.0f : p.f_g;
        float q = 0.0f;
        if (p.laser_on) q = (p.f_i0 * pulse32(p, dstep[si.sys] + rel)) * srcw[slot];
        const float invc = 1.0f / c;
        const float dloc = -ge * invc + (ge * (Tk - tl) - q) * cpr * invc * invc;
        const float dl = p.f_dt * fmaf(p.f_K, D, lk * dloc);
        // compensated lambda update, as for the forward state
        const float lo = lam_lo[slot];
        const float s = lk + dl;
        const float bp = s - lk;
        const float er = (lk - (s - bp)) + (dl - bp);
        const float lo2 = lo + er;
        l_new = s + lo2;
        lam_lo[slot] = lo2 - (l_new - s);
        const double lfull = (double)lk + (double)lo;
        gK = lfull * p.dt * (double)S;          // S = span * sum_j f
        gG = gated ? 0.0 : -lfull * p.dt * (double)(Tk - tl) * (double)invc;
    }
    lam_n[slot] = l_new;
    gK = wave_sum(gK);
    gG = wave_sum(gG);
    if (lane == 0) {
        grad[2 * (int64_t)sl + 0] += gK;
        grad[2 * (int64_t)sl + 1] += gG;
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
                               const float *Thi, float *Thi_n, float *Tlo, const float *Tl,
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
    L2T_HIP(c, hipMemcpyAsync(dst + NI, c->Tlo, sizeof(float) * NI, hipMemcpyDeviceToDevice,
                              c->stream));
    return L2T_OK;
}

int adjoint(l2t_ctx *c, const double *w, double *dL_dK, double *dL_dg, double *dL_dT0) {
    const Recording &r = c->rec;
    const size_t NI = (size_t)c->n_int, NS = (size_t)c->n_slices, S = c->sys.size();
    const int32_t C = r.ckpt;
    // scratch: segment states [C][hi, lo], lambda hi x2 + lo, ledger, grads, dstep, outputs
    const size_t seg_f = (size_t)C * 2 * NI;
    const size_t bytes = sizeof(float) * (seg_f + 3 * NI) +
                         sizeof(double) * (3 * NS + 2 * NS + 2 * S) + sizeof(int64_t) * S + 256;
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
    float *lam[2] = {lam0, lam1};
    int lc = 0;
    const hipStream_t s_ = c->stream;
    hipLaunchKernelGGL(k_lambda_in, dim3(nblk(NI, 256)), dim3(256), 0, s_, c->perm, c->n_int, w,
                       lam[0], lamlo);
    hipLaunchKernelGGL(k_zero_d, dim3(nblk(2 * NS, 256)), dim3(256), 0, s_, grad, (int64_t)(2 * NS));
    hipLaunchKernelGGL(k_zero_d, dim3(nblk(3 * NS, 256)), dim3(256), 0, s_, led, (int64_t)(3 * NS));
    const dim3 g(nblk(NS, 4)), b(256);
    std::vector<int64_t> hstep(S);
    for (int64_t k = r.n_ckpt - 1; k >= 0; --k) {
        const int64_t start = k * C;
        const int32_t L = (int32_t)std::min<int64_t>(C, r.n_steps - start);
        const float *ck = (const float *)r.buf + (size_t)k * 2 * NI;
        L2T_HIP(c, hipMemcpyAsync(seg, ck, sizeof(float) * 2 * NI, hipMemcpyDeviceToDevice, s_));
        for (size_t q = 0; q < S; ++q) hstep[q] = r.step0[q] + start;
        L2T_HIP(c, hipMemcpyAsync(dst, hstep.data(), sizeof(int64_t) * S, hipMemcpyHostToDevice, s_));
        for (int32_t m = 0; m + 1 < L; ++m) {
            float *in = seg + (size_t)m * 2 * NI, *out = seg + (size_t)(m + 1) * 2 * NI;
            L2T_HIP(c, hipMemcpyAsync(out + NI, in + NI, sizeof(float) * NI,
                                      hipMemcpyDeviceToDevice, s_));
            hipLaunchKernelGGL(k_forward_step, g, b, 0, s_, c->slices, c->n_slices, c->col, in, out,
                               out + NI, c->Tl32, c->srcw32, c->dparams, dst, m, led, c->derr);
        }
        for (int32_t m = L - 1; m >= 0; --m) {
            const float *Tst = seg + (size_t)m * 2 * NI;
            hipLaunchKernelGGL(k_adjoint_step, g, b, 0, s_, c->slices, c->n_slices, c->col, Tst,
                               c->Tl32, c->srcw32, c->dparams, dst, m, lam[lc], lam[lc ^ 1], lamlo,
                               grad);
            lc ^= 1;
        }
        L2T_HIP(c, hipGetLastError());
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
