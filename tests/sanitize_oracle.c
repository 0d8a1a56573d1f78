/*
 * A program that runs the oracle under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built and run by tests/test_oracle_sanitizers.py, on the CPU).  It calls
 * every exported oracle routine on small synthetic systems: a jittered
 * periodic FCC crystal, a slab with a free axis and a laser source, and a
 * chain for the two-temperature bar.  The sanitizers abort on the first
 * invalid access or undefined operation; the program itself only checks
 * that the cell list equals brute force and that the results are finite.
 *
 * Test infrastructure: it includes the oracle's source to see its parameter
 * struct; nothing here is part of the library.
 */
#include "../oracle/oracle.c"

#include <stdio.h>

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double uniform(void)   /* splitmix64, mapped to [0, 1) */
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int fail(const char *what)
{
    fprintf(stderr, "sanitize_oracle: %s\n", what);
    return 1;
}

static int finite_all(const double *a, int64_t n)
{
    for (int64_t k = 0; k < n; ++k)
        if (!isfinite(a[k])) return 0;
    return 1;
}

/* FCC nx x ny x nz cells of edge a; jitter of amplitude j */
static int32_t fcc(int nx, int ny, int nz, double a, double j, double *x, double *y, double *z)
{
    static const double b[4][3] = {{0, 0, 0}, {0.5, 0.5, 0}, {0.5, 0, 0.5}, {0, 0.5, 0.5}};
    int32_t n = 0;
    for (int i = 0; i < nx; ++i)
        for (int k = 0; k < ny; ++k)
            for (int l = 0; l < nz; ++l)
                for (int m = 0; m < 4; ++m) {
                    x[n] = (i + b[m][0]) * a + j * (uniform() - 0.5);
                    y[n] = (k + b[m][1]) * a + j * (uniform() - 0.5);
                    z[n] = (l + b[m][2]) * a + j * (uniform() - 0.5);
                    ++n;
                }
    return n;
}

static int check_system(int32_t n, const double *x, const double *y, const double *z,
                        const double *lo, const double *len, const int32_t *per, double rc,
                        int laser)
{
    int64_t *rb = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *rcl = calloc((size_t)n + 1, sizeof(int64_t));
    if (!rb || !rcl) return fail("allocation");
    const int64_t nb = or_neighbors(n, x, y, z, lo, len, per, rc, 0, rb, NULL, 0);
    const int64_t ncl = or_neighbors(n, x, y, z, lo, len, per, rc, 1, rcl, NULL, 0);
    if (nb <= 0 || nb != ncl) return fail("neighbour counts");
    int32_t *cb = malloc(sizeof(int32_t) * (size_t)nb), *ccl = malloc(sizeof(int32_t) * (size_t)nb);
    if (!cb || !ccl) return fail("allocation");
    if (or_neighbors(n, x, y, z, lo, len, per, rc, 0, rb, cb, nb) != nb) return fail("brute fill");
    if (or_neighbors(n, x, y, z, lo, len, per, rc, 1, rcl, ccl, nb) != nb) return fail("cell fill");
    if (memcmp(rb, rcl, sizeof(int64_t) * ((size_t)n + 1)) || memcmp(cb, ccl, sizeof(int32_t) * (size_t)nb))
        return fail("cell list differs from brute force");

    double *vx = malloc(sizeof(double) * n), *vy = malloc(sizeof(double) * n);
    double *vz = malloc(sizeof(double) * n), *m = malloc(sizeof(double) * n);
    double *Tl = malloc(sizeof(double) * n), *T = malloc(sizeof(double) * n);
    double *T0 = malloc(sizeof(double) * n), *xi = malloc(sizeof(double) * n);
    double *ea = calloc((size_t)n, sizeof(double)), *w = malloc(sizeof(double) * n);
    double *lam = malloc(sizeof(double) * n), *f = malloc(sizeof(double) * n);
    int32_t *gated = malloc(sizeof(int32_t) * n), *fixed = calloc((size_t)n, sizeof(int32_t));
    double complex *Tc = malloc(sizeof(double complex) * n);
    if (!vx || !vy || !vz || !m || !Tl || !T || !T0 || !xi || !ea || !w || !lam || !f || !gated ||
        !fixed || !Tc)
        return fail("allocation");
    for (int32_t i = 0; i < n; ++i) {
        vx[i] = 2e-3 * (uniform() - 0.5);
        vy[i] = 2e-3 * (uniform() - 0.5);
        vz[i] = 2e-3 * (uniform() - 0.5);
        m[i] = 58.6934;
        T0[i] = 300.0 + 3000.0 * uniform();
        w[i] = uniform();
        f[i] = 1e-3 * (uniform() - 0.5);
        fixed[i] = (i % 17) == 0;
    }
    vx[3] = vy[3] = vz[3] = 0.0;   /* an atom at rest: the kinetic-energy gate */
    or_lattice_temp(n, rb, cb, vx, vy, vz, m, 1e-5, 0, Tl, gated);
    or_lattice_temp(n, rb, cb, vx, vy, vz, m, 1e-5, 1, Tl, gated);
    if (!finite_all(Tl, n)) return fail("lattice temperature");

    or_params p;
    memset(&p, 0, sizeof p);
    p.T_min = 0.0;
    p.T_max = 2e4;
    p.K = 0.9465;
    p.dt = 0.05;
    p.g = 2.6427e-8;
    p.ce_const = 2.7078e-5;
    p.gamma = 1e-4;
    p.ce_cap = 3.0 * OR_KB;
    p.ke_eps = 1e-5;
    p.laser_on = laser;
    p.laser_fluence = 0.05;   /* eV/A^2: a rise of tens of K in this small slab */
    p.laser_lp = 100.0;
    p.laser_t0 = 2.0;
    p.laser_sigma = 1.0;
    p.laser_x0 = lo[0];
    p.v_atom = 11.7615;
    double ledger[3], e[8];
    for (int model = 0; model < 3; ++model) {
        p.ce_model = model;
        memcpy(T, T0, sizeof(double) * n);
        memset(ledger, 0, sizeof ledger);
        if (or_run(n, rb, cb, T, Tl, gated, x, &p, 0, 20, ledger, ea, NULL) != 0)
            return fail("range error in the run");
        if (or_run(n, rb, cb, T, Tl, gated, x, &p, 20, 5, ledger, ea, fixed) != 0)
            return fail("range error in the run with held atoms");
        or_energies(n, T, &p, e);
        if (!finite_all(T, n) || !finite_all(e, 2) || !finite_all(ledger, 3)) return fail("run");
        for (int mode = 0; mode < 2; ++mode) {
            or_coupling(n, mode, T, Tl, gated, ea, p.g, 1.0, p.ke_eps, vx, vy, vz, m, xi);
            if (!finite_all(xi, n)) return fail("coupling");
        }
        or_damping_step(n, 1.0, xi, f, f, f, m, vx, vy, vz);
        or_damping_step(n, 1.0, xi, NULL, NULL, NULL, m, vx, vy, vz);
        double dK = 0.0, dg = 0.0;
        if (or_adjoint(n, rb, cb, T0, Tl, gated, x, &p, 0, 12, w, lam, &dK, &dg) != 0)
            return fail("adjoint");
        if (!finite_all(lam, n) || !isfinite(dK) || !isfinite(dg)) return fail("adjoint values");
        for (int32_t i = 0; i < n; ++i) Tc[i] = T0[i];
        or_run_cs(n, rb, cb, Tc, Tl, gated, x, &p, p.K, 1e-20, p.g, 0.0, 0, 12);
    }
    double mf[2];
    or_mean_field(n, T0, Tl, 7.818e-8, 1.0, mf);
    if (!isfinite(mf[0]) || !isfinite(mf[1])) return fail("mean field");
    free(rb); free(rcl); free(cb); free(ccl); free(vx); free(vy); free(vz); free(m); free(Tl);
    free(T); free(T0); free(xi); free(ea); free(w); free(lam); free(f); free(gated); free(fixed);
    free(Tc);
    return 0;
}

static int check_bar(void)
{
    enum { N = 41 };
    int64_t row[N + 1];
    int32_t col[2 * N];
    int64_t k = 0;
    for (int32_t i = 0; i < N; ++i) {   /* a free chain: one or two neighbours */
        row[i] = k;
        if (i > 0) col[k++] = i - 1;
        if (i < N - 1) col[k++] = i + 1;
    }
    row[N] = k;
    double T[N], Tl[N], ledger[3] = {0, 0, 0};
    for (int32_t i = 0; i < N; ++i) {
        T[i] = (i >= N / 2 - 1 && i <= N / 2 + 1) ? 6000.0 : 300.0;
        Tl[i] = 300.0;
    }
    or_params p;
    memset(&p, 0, sizeof p);
    p.T_max = 2e4;
    p.K = 0.5;
    p.dt = 0.1;
    p.g = 1e-6;
    p.ce_const = 2.7e-5;
    if (or_run_2t(N, row, col, T, Tl, &p, 0.05, 1e-4, 0, 200, ledger) != 0) return fail("bar");
    if (!finite_all(T, N) || !finite_all(Tl, N)) return fail("bar values");
    return 0;
}

int main(void)
{
    const double a = 3.61, rc = 1.2 * a;
    enum { CAP = 4 * 5 * 5 * 5 };
    double x[CAP], y[CAP], z[CAP];
    /* periodic crystal of 5^3 cells (4 cells of edge >= r_c per axis) */
    int32_t n = fcc(5, 5, 5, a, 0.1, x, y, z);
    for (int32_t i = 0; i < n; ++i) {   /* wrap the jitter into the box */
        const double L = 5 * a;
        x[i] = fmod(x[i] + L, L);
        y[i] = fmod(y[i] + L, L);
        z[i] = fmod(z[i] + L, L);
    }
    const double lo0[3] = {0, 0, 0}, len0[3] = {5 * a, 5 * a, 5 * a};
    const int32_t per0[3] = {1, 1, 1};
    if (check_system(n, x, y, z, lo0, len0, per0, rc, 0)) return 1;
    /* slab free along x, periodic y and z only two cells long, laser on */
    n = fcc(5, 3, 3, a, 0.1, x, y, z);
    for (int32_t i = 0; i < n; ++i) {
        y[i] = fmod(y[i] + 3 * a, 3 * a);
        z[i] = fmod(z[i] + 3 * a, 3 * a);
    }
    const double lo1[3] = {-a, 0, 0}, len1[3] = {7 * a, 3 * a, 3 * a};
    const int32_t per1[3] = {0, 1, 1};
    if (check_system(n, x, y, z, lo1, len1, per1, 1.1 * a, 1)) return 1;
    if (check_bar()) return 1;
    double ti[3] = {0.0, 0.5, 1.0}, tj[3] = {1.0, 0.25, 0.0}, out[3];
    or_pair_batch(3, ti, tj, out);
    if (!finite_all(out, 3)) return fail("pair");
    (void)or_laser_q_at;
    printf("sanitize_oracle: ok\n");
    return 0;
}
