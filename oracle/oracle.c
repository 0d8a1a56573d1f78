/*
 * oracle.c -- plain FP64 CPU oracle for the electronic-temperature sub-step
 * of the meshless two-temperature MD scheme (Ullah & Ponga, "A new approach
 * for electronic heat conduction in molecular dynamics simulations").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg use it.  It shares no source with the GPU library.
 *
 * What it computes, in the paper's order and notation:
 *   - neighbour sets N(i) = { j != i : |x_j - x_i| <= r_c } under the minimum
 *     image convention (Section 2, the cut-off of Eq. 4; Section 2.1,
 *     user-given cut-off), by brute force or by a simple cell list; every
 *     row is sorted by ascending j, which fixes the summation order;
 *   - the local lattice temperature of Eq. 4 over {i} U N(i) with the centre
 *     of mass velocity removed, plus the kinetic-energy gate of the remark
 *     after Eq. 8 (no electron-phonon exchange where K_i < epsilon);
 *   - the master equation Eq. 2 with the normalisation theta = (T - T_min) /
 *     (T_max - T_min) of Section 2, integrated with explicit forward Euler
 *     sub-steps (Section 2.1), every read taken from the step-n state;
 *   - the laser source of Eq. 10 as an energy rate per atom divided by the
 *     atom's heat capacity;
 *   - the energy and temperature ledgers (Eq. 6 rate integrated per step),
 *     per system and optionally per atom;
 *   - the lattice side: the coupling coefficient of Eq. 8 and one explicit
 *     velocity step of the damped equation of motion Eq. 5;
 *   - the two-temperature bar of Section 3.1: the lattice temperature
 *     advanced by a finite-difference Fourier law in step with Eq. 2;
 *   - the discrete adjoint of the forward-Euler map (derived from Eq. 2) and
 *     a complex-step forward run for directional derivatives.
 *
 * Each of these is pinned, in tests/test_oracle_pins.py, to something other
 * than itself: closed forms, exact invariants, brute force, a library
 * routine on a special case, quadrature, complex steps and finite
 * differences, and the constants the paper prints.  Whole trajectories at
 * the workload sizes go beyond those pins: there they are parity unpinned,
 * since the paper prints no worked trajectory.
 *
 * Built with gcc -O2 -ffp-contract=off -fopenmp: no FMA contraction.  OpenMP
 * parallelises over atoms only; every per-atom sum runs serially in
 * ascending-j order and every global sum runs serially in ascending-i order,
 * so results do not depend on the thread count.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_KB 8.617333262e-5             /* Boltzmann constant, eV/K */
#define OR_MVV2E 103.64269652680505      /* 1 amu*A^2/fs^2 in eV */
#define OR_PI 3.14159265358979323846

typedef struct {
    double T_min, T_max;      /* normalisation range, K */
    double K;                 /* pair exchange rate K_ij, 1/fs (uniform) */
    double dt;                /* electronic sub-step, fs */
    double g;                 /* G * V_atom, eV/(fs K) per atom */
    int32_t ce_model;         /* 0 const, 1 linear, 2 linear capped */
    int32_t laser_on;
    double ce_const;          /* eV/K per atom */
    double gamma;             /* eV/K^2 per atom */
    double ce_cap;            /* eV/K per atom */
    double ke_eps;            /* eV, kinetic energy gate */
    double laser_fluence;     /* absorbed fluence, eV/A^2 */
    double laser_lp;          /* penetration length, A */
    double laser_t0;          /* pulse centre, fs */
    double laser_sigma;       /* pulse standard deviation, fs */
    double laser_x0;          /* x of the free surface, A */
    double v_atom;            /* atomic volume, A^3 */
} or_params;

/* ---- Eq. 2 pair term, literal -------------------------------------------
 * theta_j (1 - theta_i) exp(Delta e_ji) - theta_i (1 - theta_j) exp(Delta e_ij)
 * with Delta e_ij = -(theta_i - theta_j). */
double or_pair(double ti, double tj)
{
    return tj * (1.0 - ti) * exp(ti - tj) - ti * (1.0 - tj) * exp(tj - ti);
}

void or_pair_batch(int64_t n, const double *ti, const double *tj, double *out)
{
    for (int64_t k = 0; k < n; ++k)
        out[k] = or_pair(ti[k], tj[k]);
}

/* d/d theta_i and d/d theta_j of the literal pair term */
static double or_pair_d1(double ti, double tj)
{
    return -ti * tj * exp(ti - tj) - (1.0 - ti) * (1.0 - tj) * exp(tj - ti);
}

static double or_pair_d2(double ti, double tj)
{
    return (1.0 - ti) * (1.0 - tj) * exp(ti - tj) + ti * tj * exp(tj - ti);
}

/* ---- heat capacity model and its integral --------------------------------- */
static double or_ce(const or_params *p, double T)
{
    if (p->ce_model == 0) return p->ce_const;
    if (p->ce_model == 1) return p->gamma * T;
    double c = p->gamma * T;
    return c < p->ce_cap ? c : p->ce_cap;
}

static double or_ce_prime(const or_params *p, double T)
{
    if (p->ce_model == 0) return 0.0;
    if (p->ce_model == 1) return p->gamma;
    return (p->gamma * T < p->ce_cap) ? p->gamma : 0.0;
}

/* electronic energy of one atom, integral of c from 0 to T */
static double or_energy_of(const or_params *p, double T)
{
    if (p->ce_model == 0) return p->ce_const * T;
    if (p->ce_model == 1) return 0.5 * p->gamma * T * T;
    double Ts = p->ce_cap / p->gamma;
    if (T <= Ts) return 0.5 * p->gamma * T * T;
    return 0.5 * p->gamma * Ts * Ts + p->ce_cap * (T - Ts);
}

/* ---- Eq. 10 source as energy per unit time per atom ------------------------
 * i_0 is taken as F V_atom / (l_p sqrt(2 pi) sigma): the depth profile
 * exp(-(x - x0)/l_p)/l_p integrates to one over depth and the Gaussian in
 * time integrates to sqrt(2 pi) sigma, so a column absorbs fluence F. */
static double or_laser_q(const or_params *p, double x, double t)
{
    if (!p->laser_on) return 0.0;
    double i0 = p->laser_fluence * p->v_atom /
                (p->laser_lp * sqrt(2.0 * OR_PI) * p->laser_sigma);
    double dtp = t - p->laser_t0;
    return i0 * exp(-(x - p->laser_x0) / p->laser_lp) *
           exp(-dtp * dtp / (2.0 * p->laser_sigma * p->laser_sigma));
}

double or_laser_q_at(const or_params *p, double x, double t)
{
    return or_laser_q(p, x, t);
}

/* ---- neighbour sets --------------------------------------------------------- */
static double or_min_image(double dx, double L, int32_t periodic)
{
    if (!periodic) return dx;
    return dx - L * nearbyint(dx / L);
}

static int or_within(const double *x, const double *y, const double *z,
                     const double *len, const int32_t *per, double rc2,
                     int32_t i, int32_t j)
{
    double dx = or_min_image(x[j] - x[i], len[0], per[0]);
    double dy = or_min_image(y[j] - y[i], len[1], per[1]);
    double dz = or_min_image(z[j] - z[i], len[2], per[2]);
    return dx * dx + dy * dy + dz * dz <= rc2;
}

static int or_cmp_i32(const void *a, const void *b)
{
    int32_t u = *(const int32_t *)a, v = *(const int32_t *)b;
    return (u > v) - (u < v);
}

typedef struct {
    int32_t nc[3];
    int64_t ncell;
    int64_t *start;   /* [ncell+1] */
    int32_t *atoms;   /* atoms by cell, ascending index inside a cell */
    int32_t *cell_of; /* [n] */
} or_cells;

static int or_cells_build(or_cells *cl, int32_t n, const double *x, const double *y,
                          const double *z, const double *lo, const double *len,
                          const int32_t *per, double rc)
{
    const double *c[3] = {x, y, z};
    cl->ncell = 1;
    for (int d = 0; d < 3; ++d) {
        int32_t k = (int32_t)floor(len[d] / rc);
        cl->nc[d] = k < 1 ? 1 : k;
        cl->ncell *= cl->nc[d];
    }
    cl->start = calloc((size_t)cl->ncell + 1, sizeof(int64_t));
    cl->atoms = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    cl->cell_of = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!cl->start || !cl->atoms || !cl->cell_of) return -1;
    for (int32_t i = 0; i < n; ++i) {
        int32_t ic[3];
        for (int d = 0; d < 3; ++d) {
            double s = c[d][i] - lo[d];
            if (per[d]) s -= len[d] * floor(s / len[d]);
            int32_t k = (int32_t)floor(s / len[d] * cl->nc[d]);
            if (k < 0) k = 0;
            if (k >= cl->nc[d]) k = cl->nc[d] - 1;
            ic[d] = k;
        }
        int32_t cell = (ic[0] * cl->nc[1] + ic[1]) * cl->nc[2] + ic[2];
        cl->cell_of[i] = cell;
        cl->start[cell + 1]++;
    }
    for (int64_t k = 0; k < cl->ncell; ++k) cl->start[k + 1] += cl->start[k];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)cl->ncell);
    if (!fill) return -1;
    memcpy(fill, cl->start, sizeof(int64_t) * (size_t)cl->ncell);
    for (int32_t i = 0; i < n; ++i) cl->atoms[fill[cl->cell_of[i]]++] = i;  /* ascending i */
    free(fill);
    return 0;
}

static void or_cells_free(or_cells *cl)
{
    free(cl->start);
    free(cl->atoms);
    free(cl->cell_of);
}

/* distinct neighbouring cell coordinates along one axis */
static int or_axis_set(int32_t c, int32_t nc, int32_t periodic, int32_t out[3])
{
    int m = 0;
    for (int o = -1; o <= 1; ++o) {
        int32_t k = c + o;
        if (periodic) {
            k = ((k % nc) + nc) % nc;
        } else if (k < 0 || k >= nc) {
            continue;
        }
        int dup = 0;
        for (int q = 0; q < m; ++q) dup |= (out[q] == k);
        if (!dup) out[m++] = k;
    }
    return m;
}

/*
 * Neighbour rows sorted by ascending j.  method 0 = brute force, 1 = cell
 * list.  Call with col == NULL to fill row_ptr (counts) only; returns the
 * number of entries, or -1 on allocation failure / -2 if cap is too small.
 */
int64_t or_neighbors(int32_t n, const double *x, const double *y, const double *z,
                     const double *box_lo, const double *box_len, const int32_t *periodic,
                     double rc, int32_t method, int64_t *row_ptr, int32_t *col, int64_t cap)
{
    const double rc2 = rc * rc;
    int32_t *cnt = calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!cnt) return -1;
    or_cells cl;
    memset(&cl, 0, sizeof(cl));
    if (method == 1 && or_cells_build(&cl, n, x, y, z, box_lo, box_len, periodic, rc) != 0) {
        free(cnt);
        return -1;
    }
    int fail = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if (pass == 1) {
            row_ptr[0] = 0;
            for (int32_t i = 0; i < n; ++i) row_ptr[i + 1] = row_ptr[i] + cnt[i];
            if (col == NULL) break;
            if (row_ptr[n] > cap) { fail = -2; break; }
        }
        #pragma omp parallel for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i) {
            int32_t m = 0;
            int32_t *dst = (pass == 1) ? col + row_ptr[i] : NULL;
            if (method == 0) {
                for (int32_t j = 0; j < n; ++j) {
                    if (j == i || !or_within(x, y, z, box_len, periodic, rc2, i, j)) continue;
                    if (dst) dst[m] = j;
                    ++m;
                }
            } else {
                int32_t ci = cl.cell_of[i];
                int32_t c0 = ci / (cl.nc[1] * cl.nc[2]);
                int32_t c1 = (ci / cl.nc[2]) % cl.nc[1];
                int32_t c2 = ci % cl.nc[2];
                int32_t sx[3], sy[3], sz[3];
                int mx = or_axis_set(c0, cl.nc[0], periodic[0], sx);
                int my = or_axis_set(c1, cl.nc[1], periodic[1], sy);
                int mz = or_axis_set(c2, cl.nc[2], periodic[2], sz);
                for (int a = 0; a < mx; ++a)
                    for (int b = 0; b < my; ++b)
                        for (int e = 0; e < mz; ++e) {
                            int32_t cell = (sx[a] * cl.nc[1] + sy[b]) * cl.nc[2] + sz[e];
                            for (int64_t q = cl.start[cell]; q < cl.start[cell + 1]; ++q) {
                                int32_t j = cl.atoms[q];
                                if (j == i || !or_within(x, y, z, box_len, periodic, rc2, i, j))
                                    continue;
                                if (dst) dst[m] = j;
                                ++m;
                            }
                        }
                if (dst) qsort(dst, (size_t)m, sizeof(int32_t), or_cmp_i32);
            }
            if (pass == 0) cnt[i] = m;
        }
    }
    int64_t nnz = (n > 0) ? row_ptr[n] : 0;
    if (method == 1) or_cells_free(&cl);
    free(cnt);
    return fail ? fail : nnz;
}

/* ---- Eq. 4 local lattice temperature and the kinetic-energy gate ----------
 * Over the set {i} U N(i): subtract the mass-weighted centre-of-mass velocity
 * (local by default, global when global_com != 0), sum 1/2 m |v|^2, divide by
 * 3/2 k_B N_j.  K_i = 1/2 m_i |v_i - v_com|^2; gated[i] = K_i < ke_eps. */
void or_lattice_temp(int32_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *vx, const double *vy, const double *vz,
                     const double *mass, double ke_eps, int32_t global_com,
                     double *T_lat, int32_t *gated)
{
    double gP[3] = {0, 0, 0}, gM = 0;
    if (global_com) {
        for (int32_t i = 0; i < n; ++i) {
            gP[0] += mass[i] * vx[i];
            gP[1] += mass[i] * vy[i];
            gP[2] += mass[i] * vz[i];
            gM += mass[i];
        }
    }
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double vc[3];
        if (global_com) {
            vc[0] = gP[0] / gM; vc[1] = gP[1] / gM; vc[2] = gP[2] / gM;
        } else {
            double P[3] = {mass[i] * vx[i], mass[i] * vy[i], mass[i] * vz[i]};
            double M = mass[i];
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                int32_t j = col[q];
                P[0] += mass[j] * vx[j];
                P[1] += mass[j] * vy[j];
                P[2] += mass[j] * vz[j];
                M += mass[j];
            }
            vc[0] = P[0] / M; vc[1] = P[1] / M; vc[2] = P[2] / M;
        }
        double ux = vx[i] - vc[0], uy = vy[i] - vc[1], uz = vz[i] - vc[2];
        double Ki = 0.5 * mass[i] * (ux * ux + uy * uy + uz * uz) * OR_MVV2E;
        double KE = Ki;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
            int32_t j = col[q];
            double wx = vx[j] - vc[0], wy = vy[j] - vc[1], wz = vz[j] - vc[2];
            KE += 0.5 * mass[j] * (wx * wx + wy * wy + wz * wz) * OR_MVV2E;
        }
        double Nj = (double)(row_ptr[i + 1] - row_ptr[i] + 1);
        T_lat[i] = KE / (1.5 * OR_KB * Nj);
        gated[i] = (Ki < ke_eps) ? 1 : 0;
    }
}

/* ---- one forward-Euler sub-step of Eq. 2 (+ coupling + source) -----------
 * Reads T (step n), writes Tn (step n+1).  Per-atom ledger terms go to
 * e2l (g_i (T_i - T_lat,i)), src (q_i) and lt (the rate of the temperature
 * ledger: (g_i (T_i - T_lat,i) - q_i) / c_i).
 * Atoms with fixed[i] != 0 hold their electronic temperature (the Dirichlet
 * electronic boundary of Section 4): their neighbours still exchange with
 * them, they keep T_i, and the exchange they would have received,
 * span K S_i, goes to the temperature ledger instead, so that
 * sum_i T_i + ledger stays invariant (the exchange sums to zero over all
 * atoms). */
static void or_step(int32_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *T, const double *T_lat, const int32_t *gated,
                    const int32_t *fixed, const double *x, const or_params *p, double t,
                    double *Tn, double *e2l, double *src, double *lt)
{
    const double span = p->T_max - p->T_min;
    #pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double ti = (T[i] - p->T_min) / span;
        double S = 0.0;
        for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
            double tj = (T[col[q]] - p->T_min) / span;
            S += or_pair(ti, tj);
        }
        double c = or_ce(p, T[i]);
        double coup = (gated && gated[i]) ? 0.0 : p->g * (T[i] - T_lat[i]);
        double qi = or_laser_q(p, x ? x[i] : 0.0, t);
        double R = span * p->K * S - coup / c + qi / c;
        e2l[i] = coup;
        src[i] = qi;
        if (fixed && fixed[i]) {
            Tn[i] = T[i];
            lt[i] = span * p->K * S;
        } else {
            Tn[i] = T[i] + p->dt * R;
            lt[i] = (coup - qi) / c;
        }
    }
}

/* Mean-field parameters of Section 2: at each MD step the heat capacity and
 * the exchange rate follow the system's mean electronic and lattice
 * temperatures, C_e = lambda mean(T_e) and kappa_e = kappa_0 mean(T_e) /
 * mean(T_lat); in Eq. 3 mean(T_e) cancels, K = 2 d kappa_0 / (lambda S
 * mean(T_lat)).  out[0] = c = lambda_atom mean(T_e) (eV/K per atom), out[1] =
 * K = k_coef / mean(T_lat) (1/fs), k_coef = 2 d kappa_0 / (lambda S) (K/fs).
 * Means over all atoms of the system in ascending order. */
void or_mean_field(int32_t n, const double *T, const double *T_lat, double lambda_atom,
                   double k_coef, double *out)
{
    double st = 0.0, sl = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        st += T[i];
        sl += T_lat[i];
    }
    out[0] = lambda_atom * (st / (double)n);
    out[1] = k_coef / (sl / (double)n);
}

static int64_t or_count_out_of_range(int32_t n, const double *T, const or_params *p)
{
    int64_t bad = 0;
    for (int32_t i = 0; i < n; ++i) {
        double th = (T[i] - p->T_min) / (p->T_max - p->T_min);
        if (!(th >= 0.0 && th <= 1.0)) ++bad;   /* also catches NaN */
    }
    return bad;
}

/*
 * Advance n_steps sub-steps from step index step0 (t_n = n dt).  T is
 * updated in place.  ledger[0..2] accumulate sum g(T-T_lat) dt (energy to
 * the lattice, eV), sum q dt (source energy, eV) and
 * sum dt (g(T-T_lat) - q)/c (temperature ledger, K).  When e_atom is not
 * NULL, e_atom[i] accumulates atom i's own share of ledger[0], the energy it
 * handed to the lattice (Eq. 6 rate times dt, summed over the sub-steps).
 * Returns the number of (atom, step) states with theta outside [0,1] or
 * non-finite.
 */
int64_t or_run(int32_t n, const int64_t *row_ptr, const int32_t *col, double *T,
               const double *T_lat, const int32_t *gated, const double *x,
               const or_params *p, int64_t step0, int32_t n_steps, double *ledger,
               double *e_atom, const int32_t *fixed)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *Tn = malloc(sz), *e2l = malloc(sz), *src = malloc(sz), *lt = malloc(sz);
    if (!Tn || !e2l || !src || !lt) { free(Tn); free(e2l); free(src); free(lt); return -1; }
    int64_t bad = or_count_out_of_range(n, T, p);
    for (int32_t s = 0; s < n_steps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        or_step(n, row_ptr, col, T, T_lat, gated, fixed, x, p, t, Tn, e2l, src, lt);
        double a = 0, b = 0, c = 0;
        for (int32_t i = 0; i < n; ++i) {
            a += e2l[i] * p->dt;
            b += src[i] * p->dt;
            c += p->dt * lt[i];
        }
        ledger[0] += a;
        ledger[1] += b;
        ledger[2] += c;
        if (e_atom)
            for (int32_t i = 0; i < n; ++i) e_atom[i] += e2l[i] * p->dt;
        memcpy(T, Tn, sz);
        bad += or_count_out_of_range(n, T, p);
    }
    free(Tn); free(e2l); free(src); free(lt);
    return bad;
}

/* ---- lattice side: Eq. 8 coupling coefficient, Eq. 5 velocity step --------
 * The damping force xi_i m_i v_i of Eq. 5 does work 2 xi_i K_i per unit time
 * (Eq. 7) with K_i = 1/2 m_i |v_i|^2; Eq. 8 sets it equal to the rate P_i at
 * which atom i's electrons hand energy to the lattice (Eq. 6):
 *   xi_i = P_i / (2 K_i).
 * mode 0: P_i = g (T_i - T_lat,i) at the current electronic temperature
 *         (Section 2.1: T_e is updated first, then xi);
 * mode 1: P_i = E_i / dt_md, the energy the atom handed over during the
 *         sub-steps of the last MD step (e_atom of or_run) spread over that
 *         step, so the work of the damping force over the step matches the
 *         electronic ledger.
 * xi_i = 0 where the kinetic-energy gate holds (remark after Eq. 8) or where
 * K_i < ke_eps.  Units: P eV/fs, K eV, xi 1/fs. */
void or_coupling(int32_t n, int32_t mode, const double *T, const double *T_lat,
                 const int32_t *gated, const double *e_atom, double g, double dt_md,
                 double ke_eps, const double *vx, const double *vy, const double *vz,
                 const double *mass, double *xi)
{
    for (int32_t i = 0; i < n; ++i) {
        double Ki = 0.5 * mass[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]) * OR_MVV2E;
        double P = (mode == 0) ? g * (T[i] - T_lat[i]) : e_atom[i] / dt_md;
        xi[i] = ((gated && gated[i]) || !(Ki >= ke_eps)) ? 0.0 : P / (2.0 * Ki);
    }
}

/* One explicit step of Eq. 5 for the velocities over the MD step dt_md:
 *   v_i <- v_i + dt_md (F_i / m_i + xi_i v_i)
 * F in eV/A (NULL components: no interatomic force), m in amu, v in A/fs;
 * F/m is converted to A/fs^2 by 1 amu A^2/fs^2 = OR_MVV2E eV. */
void or_damping_step(int32_t n, double dt_md, const double *xi, const double *fx,
                     const double *fy, const double *fz, const double *mass, double *vx,
                     double *vy, double *vz)
{
    for (int32_t i = 0; i < n; ++i) {
        double inv_m = 1.0 / (mass[i] * OR_MVV2E);
        double ax = (fx ? fx[i] * inv_m : 0.0) + xi[i] * vx[i];
        double ay = (fy ? fy[i] * inv_m : 0.0) + xi[i] * vy[i];
        double az = (fz ? fz[i] * inv_m : 0.0) + xi[i] * vz[i];
        vx[i] = vx[i] + dt_md * ax;
        vy[i] = vy[i] + dt_md * ay;
        vz[i] = vz[i] + dt_md * az;
    }
}

/* ---- two-temperature bar of Section 3.1 ------------------------------------
 * Electrons by Eq. 2 as in or_run; the lattice temperature is a state too,
 * advanced in the same forward-Euler step (every read at step n) by the
 * Fourier law with the coupling as its source (the lattice line of Eq. 9):
 *   dT_l,i/dt = K_lat sum_{j in N(i)} (T_l,j - T_l,i) + (g / c_lat) (T_i - T_l,i)
 * On a chain of spacing b with the two nearest neighbours, K_lat =
 * kappa_lat / (rho C_lat b^2) makes the sum the three-point stencil of
 * Section 3.1.  No kinetic-energy gate.  T and T_lat are updated in place;
 * ledger as in or_run. */
int64_t or_run_2t(int32_t n, const int64_t *row_ptr, const int32_t *col, double *T,
                  double *T_lat, const or_params *p, double K_lat, double c_lat, int64_t step0,
                  int32_t n_steps, double *ledger)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *Tn = malloc(sz), *Tln = malloc(sz), *e2l = malloc(sz), *src = malloc(sz);
    double *lt = malloc(sz);
    if (!Tn || !Tln || !e2l || !src || !lt) {
        free(Tn); free(Tln); free(e2l); free(src); free(lt);
        return -1;
    }
    int64_t bad = or_count_out_of_range(n, T, p);
    for (int32_t s = 0; s < n_steps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        or_step(n, row_ptr, col, T, T_lat, NULL, NULL, NULL, p, t, Tn, e2l, src, lt);
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            double L = 0.0;
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) L += T_lat[col[q]] - T_lat[i];
            Tln[i] = T_lat[i] + p->dt * (K_lat * L + (p->g / c_lat) * (T[i] - T_lat[i]));
        }
        double a = 0, b = 0, c = 0;
        for (int32_t i = 0; i < n; ++i) {
            a += e2l[i] * p->dt;
            b += src[i] * p->dt;
            c += p->dt * lt[i];
        }
        ledger[0] += a;
        ledger[1] += b;
        ledger[2] += c;
        memcpy(T, Tn, sz);
        memcpy(T_lat, Tln, sz);
        bad += or_count_out_of_range(n, T, p);
    }
    free(Tn); free(Tln); free(e2l); free(src); free(lt);
    return bad;
}

/* out[0] = sum_i E(T_i) (integral of c from 0), out[1] = sum_i T_i */
void or_energies(int32_t n, const double *T, const or_params *p, double *out)
{
    double e = 0, s = 0;
    for (int32_t i = 0; i < n; ++i) {
        e += or_energy_of(p, T[i]);
        s += T[i];
    }
    out[0] = e;
    out[1] = s;
}

/*
 * Discrete adjoint of the forward-Euler map.  Every forward state T^0 ..
 * T^{N-1} is stored.  Given w = dL/dT^N, sweeps back
 *   lambda^n = lambda^{n+1} + dt J(T^n)^T lambda^{n+1},
 * where J is the Jacobian of the right-hand side R, and accumulates
 *   dL/dK = sum_n dt sum_i lambda_i^{n+1} dR_i/dK,
 *   dL/dg = sum_n dt sum_i lambda_i^{n+1} dR_i/dg.
 * The transpose uses the literal derivatives of the pair term with respect to
 * each argument and the symmetry of the neighbour relation (k in N(i) iff i in
 * N(k)), so the scatter onto k becomes a sum over N(k).
 */
int or_adjoint(int32_t n, const int64_t *row_ptr, const int32_t *col, const double *T0,
               const double *T_lat, const int32_t *gated, const double *x,
               const or_params *p, int64_t step0, int32_t n_steps, const double *w,
               double *lam_out, double *dLdK, double *dLdg)
{
    size_t sz = sizeof(double) * (size_t)(n > 0 ? n : 1);
    double *states = malloc(sz * (size_t)(n_steps > 0 ? n_steps : 1));
    double *e2l = malloc(sz), *src = malloc(sz), *ic = malloc(sz);
    double *lam = malloc(sz), *lam_new = malloc(sz), *gK = malloc(sz), *gG = malloc(sz);
    if (!states || !e2l || !src || !ic || !lam || !lam_new || !gK || !gG) return -1;
    const double span = p->T_max - p->T_min;
    if (n_steps > 0) memcpy(states, T0, sz);
    for (int32_t s = 0; s + 1 < n_steps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        or_step(n, row_ptr, col, states + (size_t)s * n, T_lat, gated, NULL, x, p, t,
                states + (size_t)(s + 1) * n, e2l, src, ic);
    }
    memcpy(lam, w, sz);
    double accK = 0, accG = 0;
    for (int32_t s = n_steps - 1; s >= 0; --s) {
        const double *T = states + (size_t)s * n;
        double t = (double)(step0 + s) * p->dt;
        #pragma omp parallel for schedule(static)
        for (int32_t k = 0; k < n; ++k) {
            double tk = (T[k] - p->T_min) / span;
            double S = 0, D1 = 0, scat = 0;
            for (int64_t q = row_ptr[k]; q < row_ptr[k + 1]; ++q) {
                int32_t j = col[q];
                double tj = (T[j] - p->T_min) / span;
                S += or_pair(tk, tj);
                D1 += or_pair_d1(tk, tj);
                /* row j contains k: d R_j / d T_k = K * d2 f(theta_j, theta_k) */
                scat += lam[j] * or_pair_d2(tj, tk);
            }
            double c = or_ce(p, T[k]);
            double cp = or_ce_prime(p, T[k]);
            int gk = gated ? gated[k] : 0;
            double gk_eff = gk ? 0.0 : p->g;
            double qk = or_laser_q(p, x ? x[k] : 0.0, t);
            /* local part: -g (T - T_lat)/c + q/c, differentiated in T */
            double dloc = -gk_eff / c + gk_eff * (T[k] - T_lat[k]) * cp / (c * c)
                          - qk * cp / (c * c);
            double JTl = lam[k] * (p->K * D1 + dloc) + p->K * scat;
            lam_new[k] = lam[k] + p->dt * JTl;
            gK[k] = lam[k] * p->dt * span * S;
            gG[k] = lam[k] * p->dt * (gk ? 0.0 : -(T[k] - T_lat[k]) / c);
        }
        for (int32_t k = 0; k < n; ++k) { accK += gK[k]; accG += gG[k]; }
        memcpy(lam, lam_new, sz);
    }
    memcpy(lam_out, lam, sz);
    *dLdK = accK;
    *dLdg = accG;
    free(states); free(e2l); free(src); free(ic);
    free(lam); free(lam_new); free(gK); free(gG);
    return 0;
}

/*
 * Complex-step forward run: the same forward-Euler map evaluated in complex
 * arithmetic, with complex T (in/out, interleaved re/im) and complex K and g.
 * Im(T^N)/h gives the directional derivative for a perturbation i*h in the
 * inputs.  Branches of the capped heat capacity follow the real part.
 */
void or_run_cs(int32_t n, const int64_t *row_ptr, const int32_t *col, double complex *T,
               const double *T_lat, const int32_t *gated, const double *x,
               const or_params *p, double K_re, double K_im, double g_re, double g_im,
               int64_t step0, int32_t n_steps)
{
    const double span = p->T_max - p->T_min;
    const double complex Kc = K_re + K_im * I, gc = g_re + g_im * I;
    double complex *Tn = malloc(sizeof(double complex) * (size_t)(n > 0 ? n : 1));
    if (!Tn) return;
    for (int32_t s = 0; s < n_steps; ++s) {
        double t = (double)(step0 + s) * p->dt;
        #pragma omp parallel for schedule(static)
        for (int32_t i = 0; i < n; ++i) {
            double complex ti = (T[i] - p->T_min) / span;
            double complex S = 0;
            for (int64_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
                double complex tj = (T[col[q]] - p->T_min) / span;
                S += tj * (1.0 - ti) * cexp(ti - tj) - ti * (1.0 - tj) * cexp(tj - ti);
            }
            double complex c;
            if (p->ce_model == 0) c = p->ce_const;
            else if (p->ce_model == 1) c = p->gamma * T[i];
            else c = (p->gamma * creal(T[i]) < p->ce_cap) ? p->gamma * T[i] : p->ce_cap;
            double complex coup = (gated && gated[i]) ? 0.0 : gc * (T[i] - T_lat[i]);
            double qi = or_laser_q(p, x ? x[i] : 0.0, t);
            Tn[i] = T[i] + p->dt * (span * Kc * S - coup / c + qi / c);
        }
        memcpy(T, Tn, sizeof(double complex) * (size_t)n);
    }
    free(Tn);
}
