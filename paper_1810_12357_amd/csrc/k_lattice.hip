// Lattice side of the two-temperature scheme: the coupling coefficient of
// Eq. 8 for the damping force of Eq. 5, and one explicit velocity step of the
// damped equation of motion (Section 2).
//
// The damping force xi_i m_i v_i does work 2 xi_i K_i per unit time (Eq. 7),
// K_i = 1/2 m_i |v_i|^2.  Setting that equal to the rate P_i at which atom i's
// electrons hand energy to the lattice (Eq. 6) gives xi_i = P_i / (2 K_i)
// (Eq. 8).  P_i is either the instantaneous g (T_i - T_i^lat) or the energy
// the atom handed over during the last advance divided by the MD step it
// spans; atoms under the kinetic-energy gate (remark after Eq. 8) and atoms
// with K_i < epsilon get xi_i = 0.
//
// Both kernels are elementwise and HBM-bound.  They run one thread per atom in
// the caller's order, so the caller's velocity, mass, force and xi arrays are
// read and written coalesced; the atom's internal slot (for T_e, T^lat and the
// per-atom ledger) comes from the caller-to-slot map, and those reads are
// gathers within a brick.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>

#include "l2t_internal.h"
#include "state_fp32c.h"

namespace l2t {
namespace {

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ void k_coupling(int32_t n, int64_t caller_off, const int32_t *__restrict__ inv,
                           int32_t mode, int32_t precision, const double *__restrict__ T64,
                           const float *__restrict__ Thi, const int16_t *__restrict__ Tlo,
                           const double *__restrict__ Tl64, const float *__restrict__ Tl32,
                           const double *__restrict__ eatom, double g, double dt_md,
                           double ke_eps, const double *__restrict__ v,
                           const double *__restrict__ mass, double *__restrict__ xi,
                           unsigned *__restrict__ err) {
    // workgroup b runs on XCD b mod 8: give each XCD one contiguous eighth of
    // the atoms, so the slot-order lines its gathers touch are reused in its
    // own L2 (neighbouring caller atoms share bricks)
    const unsigned G = gridDim.x, b = blockIdx.x;
    const unsigned logical = (G % 8u == 0u) ? (b % 8u) * (G / 8u) + b / 8u : b;
    const int64_t i = (int64_t)logical * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t slot = inv[caller_off + i];
    const double vx = v[i], vy = v[n + i], vz = v[2 * (int64_t)n + i];
    const double mi = mass[i];
    // a mass that is not finite and positive is reported, and its atom left undamped
    const bool bad_m = !(mi > 0.0 && mi <= DBL_MAX);
    if (bad_m) atomicOr(err, kErrMass);
    const double Ki = 0.5 * mi * (vx * vx + vy * vy + vz * vz) * kMvv2e;
    bool gated;
    double tl;
    if (precision == L2T_FP64) {
        const double t = Tl64[slot];
        gated = signbit(t);
        tl = fabs(t);
    } else {
        const float t = Tl32[slot];
        gated = signbit(t);
        tl = (double)fabsf(t);
    }
    double P;
    if (mode == L2T_XI_INSTANT) {
        const double T =
            (precision == L2T_FP64) ? T64[slot] : state_value(Thi[slot], Tlo[slot]);
        P = g * (T - tl);
    } else {
        P = eatom[slot] / dt_md;
    }
    xi[i] = (bad_m || gated || !(Ki >= ke_eps)) ? 0.0 : P / (2.0 * Ki);
}

// v_i <- v_i + dt_md (F_i / m_i + xi_i v_i); F/m converted to A/fs^2
__global__ void k_damping_step(int64_t n, double dt_md, const double *__restrict__ xi,
                               const double *__restrict__ force,
                               const double *__restrict__ mass, double *__restrict__ v,
                               unsigned *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double mi = mass[i];
    if (!(mi > 0.0 && mi <= DBL_MAX)) {   // reported; the atom's velocity is left as it is
        atomicOr(err, kErrMass);
        return;
    }
    const double inv_m = 1.0 / (mi * kMvv2e);
    const double x = xi[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double vd = v[d * n + i];
        const double a = (force ? force[d * n + i] * inv_m : 0.0) + x * vd;
        v[d * n + i] = vd + dt_md * a;
    }
}

}  // namespace

int coupling(l2t_ctx *c, int32_t sys, int32_t mode, double dt_md, const double *v_dev,
             const double *m_dev, double *xi_dev) {
    const SystemState &st = c->sys[sys];
    const int32_t n = st.desc.n_atoms;
    const unsigned grid = (nblk(n, 256) + 7u) / 8u * 8u;   // a multiple of 8 for the XCD mapping
    hipLaunchKernelGGL(k_coupling, dim3(grid), dim3(256), 0, c->stream, n, st.caller_off,
                       c->inv, mode, c->precision, c->T64[c->cur], c->Thi[c->cur], c->Tlo,
                       c->Tl64, c->Tl32, c->eatom, st.params.g, dt_md, st.params.ke_eps, v_dev,
                       m_dev, xi_dev, c->derr);
    L2T_HIP(c, hipGetLastError());
    return L2T_OK;
}

int damping_step(hipStream_t s, int64_t n, double dt_md, const double *xi, const double *force,
                 const double *mass, double *v, unsigned *err) {
    hipLaunchKernelGGL(k_damping_step, dim3(nblk(n, 256)), dim3(256), 0, s, n, dt_md, xi, force,
                       mass, v, err);
    return hipGetLastError() == hipSuccess ? L2T_OK : L2T_EHIP;
}

}  // namespace l2t
