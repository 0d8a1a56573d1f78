/*
 * l2t.h -- C ABI of the MI355X (gfx950) electronic-temperature sub-step
 * library for the meshless two-temperature MD scheme of Ullah & Ponga,
 * "A new approach for electronic heat conduction in molecular dynamics
 * simulations" (arXiv 1810.12357).
 *
 * What the library computes (every step runs in the library's HIP kernels):
 *   - neighbour sets within a user cut-off (Section 2.1: the electronic
 *     temperature of each atom is evaluated inside a fixed cut-off radius
 *     given by the user; Section 2, the cut-off of Eq. 4);
 *   - the local lattice temperature of Eq. 4 from neighbour velocities with
 *     the centre-of-mass velocity removed, and the kinetic-energy gate of the
 *     remark after Eq. 8 (no electron-phonon exchange where K_i < epsilon);
 *   - explicit sub-steps (Section 2.1) of the master equation Eq. 2 with the
 *     normalisation of Section 2, theta = (T - T_min)/(T_max - T_min):
 *       dT_i/dt = (T_max - T_min) K sum_{j in N(i)} f(theta_i, theta_j)
 *                 - g_i (T_i - T_i^lat)/c_i + q_i(t)/c_i
 *     where f is the pair term of Eq. 2, K the exchange rate of Eq. 3 (one
 *     value per system, so K_ij is symmetric), g = G V_atom and c = C_e V_atom
 *     the per-atom coupling and heat capacity (Section 2, C_e = lambda T_e),
 *     and q_i the laser source of Eq. 10 taken as energy per unit time per
 *     atom;
 *   - the per-system energy ledger: the exchange rate of Eq. 6 integrated
 *     over each sub-step, the source energy, and the electronic energy; on
 *     request the same exchange per atom;
 *   - the lattice side: the coupling coefficient of Eq. 8 and one explicit
 *     velocity step of the damped equation of motion Eq. 5;
 *   - the discrete adjoint of the sub-step map, for gradients of a loss on
 *     the final T_e with respect to K, G and the initial field.
 *
 * Units: Angstrom, femtosecond, eV, Kelvin, amu.
 *
 * Conventions that hold for every entry point:
 *   - Every function returns an int status (L2T_OK = 0; negative values are
 *     errors; positive values are warnings).  No C++ exception crosses the
 *     ABI.  After an error, l2t_last_error() holds a message.
 *   - A context owns all device buffers it allocates (through hipMalloc, or
 *     the caller's allocator after l2t_set_allocator); the caller owns every
 *     pointer it passes in.  Caller pointers are borrowed for the duration of
 *     the call only: host buffers are copied before the call returns; device
 *     buffers are read or written in order on the context's stream.
 *   - Per-atom arrays are in the caller's atom order of one system, FP64.
 *     Internally the library reorders atoms by cell; the order never leaks.
 *   - mem = L2T_HOST for host pointers, L2T_DEVICE for device pointers on the
 *     context's device.
 *   - A context is not thread-safe: use one context per host thread.
 *     Contexts on different threads may work at the same time.
 *   - All work runs on the HIP stream passed to l2t_create (0 = the null
 *     stream) and is asynchronous unless the function says it synchronises.
 */
#ifndef L2T_H
#define L2T_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------------- */
#define L2T_OK         0
#define L2T_WUNSTABLE  1   /* warning: explicit step may be unstable (see l2t_set_params) */
#define L2T_EINVAL    -1   /* bad argument (sizes, ranges, box, unknown enum) */
#define L2T_ENOMEM    -2   /* device allocation failed */
#define L2T_EHIP      -3   /* HIP runtime error (message in l2t_last_error) */
#define L2T_ESTATE    -4   /* call out of order (e.g. advance before neighbours) */
#define L2T_ERANGE    -5   /* theta left [0,1] or T became non-finite (sticky) */
#define L2T_ENOTIMPL  -6   /* combination not supported */

/* ---- precision of the sub-step path ---------------------------------------- */
#define L2T_FP64   0   /* plain: literal Eq. 2 pair term in FP64, one launch per sub-step per system */
#define L2T_FP32C  1   /* FP32 pair terms, FP64 neighbour sums, state = FP32 hi + 16-bit low part (39 bits), updated in FP64 */

/* ---- memory space of a caller pointer -------------------------------------- */
#define L2T_HOST    0
#define L2T_DEVICE  1

/* ---- per-atom fields (FP64 in the caller's atom order) --------------------- */
#define L2T_FIELD_TE    0   /* electronic temperature T_e, K (read/write) */
#define L2T_FIELD_TL    1   /* lattice temperature T^lat, K (read/write; >= 0) */
#define L2T_FIELD_GATE  2   /* 1.0 where the kinetic-energy gate holds, else 0.0 (read/write) */
#define L2T_FIELD_NBRS  3   /* neighbour count |N(i)| as a double (read only) */
#define L2T_FIELD_ELAT  4   /* energy the atom handed to the lattice during the last advance of its
                               system, sum over sub-steps of g (T_i - T_i^lat) dt, eV (read only;
                               recorded while L2T_OPT_ATOM_LEDGER is on) */
#define L2T_FIELD_FIXED 5   /* 1.0 where the atom holds its T_e (the fixed electronic boundary of
                               Section 4), else 0.0 (read/write; cleared by l2t_build_neighbors) */

/* ---- electronic heat capacity models (per atom) ---------------------------- */
#define L2T_CE_CONST   0   /* c = ce_const */
#define L2T_CE_LINEAR  1   /* c = gamma T (C_e = lambda T_e, Section 2) */
#define L2T_CE_CAPPED  2   /* c = min(gamma T, ce_cap) */

/* ---- tuning options (l2t_set_option) ---------------------------------------- */
#define L2T_OPT_PERSISTENT     0   /* FP32C global-gather kernel: 1 = all sub-steps in one persistent launch */
#define L2T_OPT_BLOCK          1   /* FP32C: threads per workgroup, multiple of 64 up to 512; the
                                      global-gather kernels use at most 256 (0 = autotune) */
#define L2T_OPT_RESIDENT_MAX   2   /* batched FP64 advance: largest system (slots, padded to whole
                                      64-lane slices) that one workgroup keeps whole in LDS for all
                                      sub-steps of an advance; used when every system of the context
                                      fits.  0 = the default 1024, -1 = never (one launch per
                                      sub-step).  Results are bitwise equal either way. */
#define L2T_OPT_GRAPH          3   /* how an advance issues its per-sub-step launches: 0 = one by
                                      one, 1 = replays of captured hipGraphs of 256 sub-steps,
                                      2 = FP32C: the autotuner times both on its probe and keeps the
                                      faster (default; FP64 advances and the adjoint's segments
                                      replay graphs unless it is 0).  Reading it returns the way in
                                      effect for the FP32C advance (0 or 1; 1 until timed).  Results
                                      are bitwise equal either way. */
#define L2T_OPT_AUTOTUNE       4   /* 1 = run the autotuner at the next advance, and let
                                      l2t_build_neighbors time the brick edge (default 1).  The
                                      autotuner's choice is kept per problem shape for the
                                      process and, when the environment variable
                                      L2T_AUTOTUNE_CACHE names a file, appended to it as one line
                                      (shape key|kernel persistent block graph) and read back by
                                      later processes. */
#define L2T_OPT_KERNEL         5   /* 0 = global gathers, 1 = LDS brick tiles.  FP32C: autotuned by
                                      default.  FP64: 1 by default; systems in the lattice mode, and
                                      tiles over 64 KB of FP64 values, take the global gathers.  The
                                      forms give bitwise-equal states. */
#define L2T_OPT_BRICK_EDGE     6   /* largest brick edge in cells (1..1024) for the next
                                      l2t_build_neighbors (0 = automatic: a cost model, checked
                                      by timing on large FP32C layouts, see l2t_build_neighbors) */
#define L2T_OPT_ATOM_LEDGER    7   /* 1 = record each atom's energy to the lattice during every advance
                                      (L2T_FIELD_ELAT, L2T_XI_LEDGER); costs 16 bytes per atom-substep
                                      of extra traffic while on (default 0) */

#define L2T_OPT_BATCH_FP64     8   /* FP64: 1 = one launch per sub-step over all systems; 0 = the
                                      systems one after another (default 0) */
#define L2T_OPT_SWEEP          9   /* order in which the brick launches take the bricks: 1 = the
                                      same every sub-step, 2 = reversed on every other sub-step, so
                                      that a sub-step starts with the bricks (and the table rows and
                                      temperatures) the previous one touched last; 0 = chosen at
                                      l2t_build_neighbors by timing both on large FP32C layouts
                                      (default; otherwise 1).  Reading it returns the order in
                                      effect (1 or 2).  States are bitwise the same either way. */
#define L2T_OPT_TABLE_STREAM  10   /* how the brick kernels load the neighbour table, which each
                                      sub-step reads once: 1 = cached like other loads, 2 = with
                                      the non-temporal hint, so that it does not displace from
                                      L2 the temperatures that neighbouring bricks read again;
                                      0 = chosen at l2t_build_neighbors by timing both on large
                                      FP32C layouts (default; otherwise 1).  Reading it returns
                                      the choice in effect (1 or 2).  States are bitwise the
                                      same either way. */

/* ---- source of the energy rate in the coupling coefficient (l2t_coupling) ------ */
#define L2T_XI_INSTANT  0   /* P_i = g (T_i - T_i^lat) at the current T_e (Section 2.1 order) */
#define L2T_XI_LEDGER   1   /* P_i = E_i / dt_md, E_i the recorded energy of the last advance */

typedef struct l2t_ctx l2t_ctx;

/* One independent system.  Periodic axes use the minimum image convention
 * and need box_len >= 2 r_cut; atoms on a free axis must lie inside
 * [box_lo, box_lo + box_len]. */
typedef struct {
    int32_t n_atoms;        /* > 0 */
    int32_t periodic[3];    /* 1 = periodic along x, y, z */
    double box_lo[3];       /* Angstrom */
    double box_len[3];      /* Angstrom, > 0 */
} l2t_system_desc;

/* Per-system parameters of Eq. 2, Eq. 4 gate and Eq. 10. */
typedef struct {
    double T_min, T_max;    /* normalisation range of Section 2, K (T_max > T_min) */
    double K;               /* exchange rate K_ij of Eq. 3, 1/fs (>= 0) */
    double dt;              /* electronic sub-step, fs (> 0) */
    double g;               /* G V_atom, eV/(fs K) per atom (>= 0) */
    int32_t ce_model;       /* L2T_CE_* */
    int32_t laser_on;       /* 1 = add the Eq. 10 source */
    double ce_const;        /* eV/K per atom (L2T_CE_CONST) */
    double gamma;           /* eV/K^2 per atom (L2T_CE_LINEAR, L2T_CE_CAPPED) */
    double ce_cap;          /* eV/K per atom (L2T_CE_CAPPED) */
    double ke_eps;          /* kinetic-energy gate epsilon, eV (1e-5 in the paper) */
    double laser_fluence;   /* absorbed fluence F, eV/A^2 */
    double laser_lp;        /* penetration length l_p, A (> 0 when laser_on) */
    double laser_t0;        /* pulse centre t_0, fs */
    double laser_sigma;     /* pulse standard deviation sigma, fs (> 0 when laser_on) */
    double laser_x0;        /* x of the irradiated free surface x_0, A */
    double v_atom;          /* atomic volume V_atom = V/N, A^3 */
} l2t_params;

/* Mean-field parameter mode of Section 2: the heat capacity and the exchange
 * rate follow the system's mean electronic and lattice temperatures, C_e =
 * lambda mean(T_e) and kappa_e = kappa_0 mean(T_e) / mean(T_lat).  With Eq. 3
 * the mean electronic temperature cancels from K.  The means are taken on the
 * device at the start of every advance (once per MD step of the caller) and
 * held for its sub-steps. */
typedef struct {
    int32_t on;             /* 1 = refresh c and K at the start of every advance */
    int32_t reserved;       /* 0 */
    double lambda;          /* c = lambda mean(T_e): lambda_vol V_atom, eV/K^2 per atom (> 0) */
    double k_coef;          /* K = k_coef / mean(T^lat): 2 d kappa_0 / (lambda_vol S), K/fs (> 0),
                               S the lattice sum of |r_ij|^2 as in l2t_exchange_rate */
} l2t_mean_field;

/* Two-temperature lattice of Section 3.1 (the lattice line of Eq. 9): the
 * lattice temperature becomes a state advanced with the electrons in the same
 * forward-Euler step (every read at step n),
 *     dT_l,i/dt = K_lat sum_{j in N(i)} (T_l,j - T_l,i) + (g / c_lat)(T_i - T_l,i),
 * the Fourier law over the neighbour set with the coupling as its source.  On
 * a chain of spacing b holding the two nearest neighbours, K_lat =
 * kappa_lat / (rho C_lat b^2) is the three-point stencil of Section 3.1; in
 * general K_lat = 2 d kappa_lat / (rho C_lat S), the lattice form of Eq. 3. */
typedef struct {
    int32_t on;             /* 1 = evolve T^lat */
    int32_t reserved;       /* 0 */
    double K_lat;           /* 1/fs (>= 0) */
    double c_lat;           /* lattice heat capacity per atom, rho C_lat V_atom, eV/K (> 0) */
} l2t_lattice_fd;

/* Per-system ledger, FP64.  With any heat capacity model,
 * sum_T + T_ledger_acc is conserved by the sub-step (the exchange term sums
 * to zero over the system; the exchange an atom with a fixed T_e would have
 * received is booked in T_ledger_acc); with a constant uniform c and no fixed
 * atoms, E_e + E_e_to_l - E_src is conserved too. */
typedef struct {
    double t;               /* time of the current state, fs */
    int64_t step;           /* sub-steps taken since the last l2t_set_field(TE) */
    double E_e;             /* sum_i integral_0^{T_i} c dT, eV */
    double sum_T;           /* sum_i T_i, K */
    double E_e_to_l;        /* sum over sub-steps of sum_i g_i (T_i - T_i^lat) dt, eV (Eq. 6) */
    double E_src;           /* sum over sub-steps of sum_i q_i dt, eV */
    double T_ledger_acc;    /* sum over sub-steps of sum_i dt (g_i (T_i - T_i^lat) - q_i)/c_i, K */
    double T_max_atom;      /* largest T_i, K */
    double T_min_atom;      /* smallest T_i, K */
} l2t_energy_report;

/* ---- lifecycle -------------------------------------------------------------- */

/* Create a context holding n_systems independent systems (Section 2.1: one
 * electronic temperature per atom).  descs[n_systems] is copied.  precision is
 * L2T_FP64 or L2T_FP32C.  hip_stream is a hipStream_t (may be NULL).
 * Errors: EINVAL (n_systems < 1, n_atoms < 1, box_len <= 0, bad precision),
 * ENOMEM, EHIP (no device). */
int l2t_create(l2t_ctx **out, int32_t n_systems, const l2t_system_desc *descs,
               int32_t precision, void *hip_stream);

/* Release every buffer owned by the context (synchronises its stream). */
void l2t_destroy(l2t_ctx *ctx);

/* Device memory of the context.  Every device buffer the context allocates
 * after this call comes from alloc(bytes, user), which returns device memory
 * of the context's GPU aligned to at least 256 bytes, or NULL (the call that
 * needed it then fails with ENOMEM), and goes back through free_(ptr, user),
 * for instance so that PyTorch's caching allocator owns the memory.  The
 * library synchronises its stream before it hands a block back.  Buffers
 * allocated before the call stay with the allocator that made them and are
 * released through it.  alloc = free_ = NULL restores hipMalloc / hipFree.
 * Buffers grow on demand (neighbour build, recorded advance, adjoint, host
 * staging), so the allocator can be called from any of those calls and from
 * l2t_destroy.  Errors: EINVAL (NULL context, or exactly one of alloc and
 * free_ NULL). */
int l2t_set_allocator(l2t_ctx *ctx, void *(*alloc)(size_t bytes, void *user),
                      void (*free_)(void *ptr, void *user), void *user);

/* ---- geometry --------------------------------------------------------------- */

/* Atom positions of system sys, SoA xyz[3*n]: x[0..n), y[0..n), z[0..n), A
 * (Section 2.1: every atom carries its own electronic temperature, and the
 * atoms it exchanges heat with are those inside the cut-off around its
 * position).  Positions on periodic axes are wrapped into the box.
 * Invalidates the neighbour sets.  Errors: EINVAL (sys out of range, NULL). */
int l2t_set_positions(l2t_ctx *ctx, int32_t sys, const double *xyz, int32_t mem);

/* Build the neighbour sets N(i) = { j != i : |x_j - x_i| <= r_cut } of every
 * system (Section 2.1, user-given cut-off; minimum image on periodic axes,
 * distances in FP64, inclusive).  Atoms are binned into cells of edge >=
 * r_cut and reordered by cell.  Synchronises.  Outputs (nullable): the
 * largest and the mean neighbour count over all atoms.  A rebuild (new
 * positions of the same atoms) keeps each system's T_e (bit for bit), T^lat
 * and gate, its ledger and its step counter; it clears the per-atom energy
 * record and the held atoms (L2T_FIELD_FIXED), and recomputes the source
 * weights from the new positions.  If the build fails, T_e and T^lat must be
 * written again.  An FP32C context
 * whose layout has at least one brick per CU also times the brick edge the
 * first time it builds a given problem shape in the process: the cost
 * model's edge and its two neighbours are built and each runs a short probe
 * of the sub-step kernel on stand-in data (the context's fields are not
 * used), so that first build costs two or three layouts; the sweep order and
 * the table-load policy (L2T_OPT_SWEEP, L2T_OPT_TABLE_STREAM, when left at 0)
 * are timed on the chosen layout.  L2T_OPT_AUTOTUNE = 0, L2T_OPT_BRICK_EDGE
 * or a pinned launch form skip the timing.
 * Errors: ESTATE (positions missing), EINVAL (r_cut <= 0, periodic box_len <
 * 2 r_cut, atom outside the box on a free axis). */
int l2t_build_neighbors(l2t_ctx *ctx, double r_cut, int32_t *max_nbrs, double *mean_nbrs);

/* Copy the neighbour sets of system sys to host arrays in the caller's atom
 * order, each row sorted by ascending j: row_ptr[n+1], col[cap].  With
 * col == NULL only row_ptr is written.  Synchronises.
 * Errors: ESTATE (no neighbours), EINVAL (cap < entries). */
int l2t_get_neighbors(l2t_ctx *ctx, int32_t sys, int64_t *row_ptr, int32_t *col, int64_t cap);

/* ---- parameters and fields -------------------------------------------------- */

/* Parameters of system sys (Eq. 2, Eq. 3 value K, Eq. 4 gate epsilon,
 * Eq. 10 source).  Returns L2T_WUNSTABLE (a warning, parameters are still set)
 * when the neighbour sets exist and the Gershgorin bound of the linearised
 * explicit step, 2 K dt max_i |N(i)|, exceeds 2.
 * Errors: EINVAL (T_max <= T_min, dt <= 0, K < 0, g < 0, unknown ce_model,
 * non-positive heat capacity constants, laser_lp or laser_sigma <= 0). */
int l2t_set_params(l2t_ctx *ctx, int32_t sys, const l2t_params *p);

/* Mean-field parameter mode of system sys (Section 2, see l2t_mean_field).
 * While on, the system's ce_model and ce_const and its K are replaced at the
 * start of every advance: c = lambda mean(T_e) (constant over the system and
 * over the advance), K = k_coef / mean(T^lat).  Needs T^lat for the advance.
 * Errors: EINVAL (lambda or k_coef not > 0 while on), ESTATE (parameters not
 * set).  An advance whose mean T^lat is not > 0 reports ERANGE. */
int l2t_set_mean_field(l2t_ctx *ctx, int32_t sys, const l2t_mean_field *mf);

/* Two-temperature lattice mode of system sys (Section 3.1, see
 * l2t_lattice_fd).  FP64 contexts only.  The initial T^lat comes from
 * l2t_set_field(L2T_FIELD_TL) or l2t_set_velocities and is read back with
 * l2t_get_field; while on, the kinetic-energy gate is ignored.  With a
 * constant c, sum_i (c T_i + c_lat T_l,i) is conserved.
 * Errors: EINVAL (K_lat < 0, c_lat <= 0 while on), ENOTIMPL (FP32C context),
 * ESTATE (parameters not set). */
int l2t_set_lattice_fd(l2t_ctx *ctx, int32_t sys, const l2t_lattice_fd *lf);

/* The parameters of system sys in effect for the last (or next) sub-step:
 * those of l2t_set_params, with K, ce_model and ce_const as the last
 * mean-field refresh set them.  Synchronises. */
int l2t_get_params(l2t_ctx *ctx, int32_t sys, l2t_params *out);

/* Write a per-atom field of system sys from src[n] (FP64, caller order):
 * the per-atom electronic temperature T_e of Section 2.1, the lattice
 * temperature T^lat of Eq. 4 (when it is not derived from velocities), the
 * kinetic-energy gate of the remark after Eq. 8, or the fixed-T_e flag of the
 * Section 4 boundary.  Writing L2T_FIELD_TE restarts the system's ledger and
 * step counter.  An FP32C context stores T_e as the FP32 value hi = fl32(T)
 * and a 16-bit low part q with T = hi + q 2^(max(f, -125) - 39) (f the frexp
 * exponent of hi), rounding T by at most 2^-38 of itself; a value read back
 * with l2t_get_field and written again gives the same stored pair.
 * Synchronises.  Errors: ESTATE (neighbours not built), EINVAL (unknown or
 * read-only field, T^lat < 0), ERANGE (a T_e outside [T_min, T_max] or
 * non-finite; nothing is written). */
int l2t_set_field(l2t_ctx *ctx, int32_t sys, int32_t field, const double *src, int32_t mem);

/* Read a per-atom field of system sys into dst[n] (FP64, caller order): the
 * per-atom T_e of Section 2.1, T^lat of Eq. 4, the gate, the neighbour count,
 * the energy handed to the lattice (Eq. 6 integrated over the last advance)
 * or the fixed-T_e flag.  FP32C temperatures are returned as hi + q s, exact
 * in FP64 (see l2t_set_field).
 * Synchronises when mem == L2T_HOST. */
int l2t_get_field(l2t_ctx *ctx, int32_t sys, int32_t field, double *dst, int32_t mem);

/* Eq. 4: local lattice temperature from velocities v[3*n] (SoA, A/fs) and
 * masses m[n] (amu) over {i} U N(i) with the centre-of-mass velocity of that
 * set removed (global_com = 1: the system's centre of mass instead), and the
 * gate of the remark after Eq. 8: K_i = 1/2 m_i |v_i - v_com|^2 < ke_eps
 * switches the coupling of atom i off.  Uses ke_eps of the system's
 * parameters.  Synchronises.  Errors: ESTATE (neighbours or parameters
 * missing), EINVAL (mass <= 0). */
int l2t_set_velocities(l2t_ctx *ctx, int32_t sys, const double *v, const double *mass,
                       int32_t mem, int32_t global_com);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight MD loops, harnesses that forbid hipMalloc): the same Eq. 4
 * update as l2t_set_velocities, with v[3*n] and mass[n] DEVICE pointers on
 * the context's device (no host staging), staged through a fixed array that
 * the library holds on each GPU until the process ends instead of the
 * context's grow-on-demand buffer.  The call allocates nothing: no hipMalloc,
 * hipFree or caller allocator.  Limit: 4 doubles per atom slot (atoms of the
 * system padded to a multiple of 64) + 4 <= 32 MiB, i.e. systems of at most
 * 1,048,512 atoms; larger systems return EINVAL.  Every context on a GPU
 * shares that GPU's array, so calls that overlap in time on one GPU (two
 * host threads, or two contexts on different streams) race: serialise them.
 * Results are bitwise those of l2t_set_velocities.  Synchronises.
 * Errors: EINVAL (sys out of range, NULL, system over the limit, a mass not
 * finite and > 0), ESTATE (neighbours or parameters missing), EHIP. */
int l2t_set_velocities_noalloc(l2t_ctx *ctx, int32_t sys, const double *v, const double *mass,
                               int32_t global_com);

/* ---- time stepping ---------------------------------------------------------- */

/* Advance every system by n_substeps explicit forward-Euler sub-steps of
 * Eq. 2 (Section 2.1), Jacobi-synchronous: every read in sub-step n sees the
 * step-n state.  Atoms flagged L2T_FIELD_FIXED keep their T_e; their
 * neighbours exchange with them as usual.  L2T_FP64: one launch per sub-step
 * per system, the systems one after another (L2T_OPT_BATCH_FP64: all systems
 * together, one launch per sub-step, or one launch for all sub-steps when
 * every system fits a workgroup, see L2T_OPT_RESIDENT_MAX).  L2T_FP32C: all
 * systems together, one launch per sub-step; with L2T_OPT_PERSISTENT, all
 * sub-steps in one persistent launch.  Every form gives bitwise-equal results.
 * Asynchronous; a range violation is reported by the next synchronising call
 * as ERANGE.
 * Errors: ESTATE (neighbours, parameters or T_e missing), EINVAL. */
int l2t_advance(l2t_ctx *ctx, int32_t n_substeps);

/* Advance system sys alone (same arithmetic as l2t_advance). */
int l2t_advance_system(l2t_ctx *ctx, int32_t sys, int32_t n_substeps);

/* As l2t_advance, and record the forward trajectory for l2t_adjoint: the
 * state is stored every ckpt_every sub-steps (device memory, about
 * ceil(n/ckpt) * 8 bytes per atom) and the sub-steps in between are recomputed
 * by the adjoint with the same kernels, so the recomputation is bitwise equal
 * to the forward.  Errors: as l2t_advance; EINVAL (ckpt_every < 1); ENOMEM;
 * ENOTIMPL (a system with fixed atoms or in the mean-field mode). */
int l2t_advance_recorded(l2t_ctx *ctx, int32_t n_substeps, int32_t ckpt_every);

/* Discrete adjoint of the last recorded advance (derived from Eq. 2 by
 * differentiating the forward-Euler map).  Given dL_dTN = dL/dT^N for all
 * atoms of all systems (FP64, systems concatenated in order, caller order
 * inside each), writes dL/dK and dL/dg per system (host arrays
 * [n_systems], FP64) and, if dL_dT0 is not NULL, dL/dT^0 (same layout as
 * dL_dTN, memory space mem).  The reverse sub-step is a gather over the same
 * neighbour sets (no atomics): (J^T lambda)_k = K sum_{j in N(k)}
 * d1f(theta_k, theta_j) (lambda_k - lambda_j) + local terms.  Synchronises.
 * Errors: ESTATE (no recorded advance), EINVAL. */
int l2t_adjoint(l2t_ctx *ctx, const double *dL_dTN, int32_t mem, double *dL_dK,
                double *dL_dg, double *dL_dT0);

/* Checkpoint / resume of a system's counters.  Writing L2T_FIELD_TE resets
 * the system's sub-step counter (the time of the Eq. 10 source is step * dt)
 * and its ledger accumulators; a resumed run calls this after restoring T_e
 * (from L2T_FIELD_TE of the saved run, which restores the state bitwise) to
 * set them to the saved report's step, E_e_to_l, E_src and T_ledger_acc.
 * The sub-steps that follow then equal those of the uninterrupted run bit
 * for bit; later ledger totals equal its totals up to FP64 summation order.
 * Synchronises.  Errors: EINVAL (bad system, step < 0, a non-finite value),
 * ESTATE (neighbours or T_e not set). */
int l2t_set_counters(l2t_ctx *ctx, int32_t sys, int64_t step, double E_e_to_l, double E_src,
                     double T_ledger_acc);

/* Per-system energy report (FP64 reductions on the device): the electronic
 * energy sum_i integral_0^{T_i} c dT, the energy handed to the lattice at the
 * exchange rate of Eq. 6 integrated over the sub-steps, and the energy the
 * Eq. 10 source deposited, whose balance Section 3.2 examines; also sum T and
 * the temperature ledger that keeps sum T + ledger invariant.  Synchronises;
 * returns
 * ERANGE if any sub-step since the last check produced theta outside [0,1]
 * or a non-finite T (the ledger is still written). */
int l2t_energies(l2t_ctx *ctx, int32_t sys, l2t_energy_report *out);

/* Wait for the context's stream; reports a pending ERANGE. */
int l2t_sync(l2t_ctx *ctx);

/* Set a tuning option L2T_OPT_* (see above). */
int l2t_set_option(l2t_ctx *ctx, int32_t option, int64_t value);

/* Read a tuning choice the autotuner or the caller made. */
int l2t_get_option(l2t_ctx *ctx, int32_t option, int64_t *value);

/* ---- lattice side (Eq. 5 - Eq. 8) ---------------------------------------------- */

/* Coupling coefficient of the damping force of Eq. 5 for every atom of
 * system sys: the damping force xi_i m_i v_i does work 2 xi_i K_i per unit time
 * (Eq. 7), with K_i = 1/2 m_i |v_i|^2 the atom's kinetic energy; Eq. 8 sets it
 * equal to the rate P_i at which the atom's electrons hand energy to the
 * lattice (Eq. 6):
 *     xi_i = P_i / (2 K_i)                                  [1/fs]
 * mode L2T_XI_INSTANT: P_i = g (T_i - T_i^lat) from the current T_e, as the
 *   paper's implementation does once the sub-steps of an MD step are done;
 * mode L2T_XI_LEDGER: P_i = E_i / dt_md with E_i = L2T_FIELD_ELAT, the energy
 *   the atom handed over during the last advance (which spans the MD step
 *   dt_md), so that one velocity step of Eq. 5 gives the lattice that energy
 *   to first order in dt_md.
 * xi_i = 0 where the kinetic-energy gate of l2t_set_velocities holds (the
 * remark after Eq. 8) and where K_i < ke_eps.  v[3*n] (SoA, A/fs) and
 * mass[n] (amu) are the velocities the damping force will act on; xi[n] is
 * written (FP64, caller order).  All three live in memory space mem.
 * Asynchronous on the context's stream when mem == L2T_DEVICE (no host
 * synchronisation, so it can be captured in a caller's graph); synchronises
 * when mem == L2T_HOST.
 * Errors: EINVAL (bad mode, dt_md <= 0 in ledger mode, NULL), ESTATE (T_e or
 * T^lat not set; ledger mode without a recorded advance of this system).
 * A mass that is not finite and > 0 gives xi = 0 for its atom and EINVAL,
 * returned by this call when mem == L2T_HOST and otherwise by the next call
 * that synchronises (as ERANGE from l2t_advance is). */
int l2t_coupling(l2t_ctx *ctx, int32_t sys, int32_t mode, double dt_md, const double *v,
                 const double *mass, double *xi, int32_t mem);

/* One explicit step of the damped equation of motion Eq. 5 for the atoms of
 * system sys over the MD step dt_md:
 *     v_i <- v_i + dt_md (F_i / m_i + xi_i v_i)
 * in place on v[3*n] (SoA, A/fs), with forces force[3*n] (SoA, eV/A; NULL =
 * no interatomic force), masses mass[n] (amu) and xi[n] (1/fs, e.g. from
 * l2t_coupling); F/m is converted with 1 amu A^2/fs^2 = 103.6427 eV.  The
 * library's MD integrator is the caller's: this step is the reference form of
 * Eq. 5 (and what the energy check against L2T_FIELD_ELAT uses).  All arrays
 * live in memory space mem.  Asynchronous when mem == L2T_DEVICE; synchronises
 * when mem == L2T_HOST.
 * Errors: EINVAL (NULL, dt_md <= 0).  An atom whose mass is not finite and
 * > 0 keeps its velocity and raises EINVAL, reported as for l2t_coupling. */
int l2t_damping_step(l2t_ctx *ctx, int32_t sys, double dt_md, const double *xi,
                     const double *force, const double *mass, double *v, int32_t mem);

/* ---- helpers ------------------------------------------------------------------ */

/* Eq. 3 for a multi-shell cut-off: K = 2 kappa_e d / (C_e S) with S the lattice
 * sum of |r_ij|^2 over one atom's neighbour set (S = Z b^2 for a single
 * shell).  SI inputs (W/m/K, J/m^3/K, m^2) give 1/s.  Returns NaN for
 * non-positive inputs. */
double l2t_exchange_rate(double kappa_e, double C_e, int32_t dim, double lattice_sum);

/* FP32 pair term of Eq. 2 as the FP32C path evaluates it, for n pairs of
 * normalised temperatures on the device (ti, tj, out are device pointers,
 * FP32): out[k] = f(ti[k], tj[k]).  The cancellation-free product form
 * f = d h(m, d^2) with d = theta_j - theta_i and m = (theta_i + theta_j)/2 is
 * used, so f(a, b) = -f(b, a) holds bitwise.  Asynchronous on hip_stream.
 * Errors: EINVAL (n < 0, NULL with n > 0). */
int l2t_pair_fp32(const float *ti, const float *tj, float *out, int64_t n, void *hip_stream);

/* Static text of a status code. */
const char *l2t_strerror(int status);

/* Message of the last error on this context ("" if none). */
const char *l2t_last_error(const l2t_ctx *ctx);

/* ABI version (major * 10000 + minor * 100 + patch). */
int l2t_version(void);

#ifdef __cplusplus
}
#endif
#endif /* L2T_H */
