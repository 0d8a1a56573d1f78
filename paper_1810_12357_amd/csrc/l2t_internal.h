// Internal declarations shared by the library's own sources (host API, kernel
// launchers, autotuner).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "l2t.h"

namespace l2t {

constexpr int kWave = 64;                          // CDNA wavefront width
constexpr double kBoltzmann = 8.617333262e-5;      // eV/K
constexpr double kMvv2e = 103.64269652680505;      // 1 amu*A^2/fs^2 in eV

// error bits of the device-side sticky flag
constexpr unsigned kErrRange = 1u;      // theta outside [0,1] or non-finite T
constexpr unsigned kErrBox = 2u;        // atom outside the box on a free axis
constexpr unsigned kErrBarrier = 4u;    // persistent-kernel barrier spin limit hit
constexpr unsigned kErrCellOverflow = 8u;
constexpr unsigned kErrMeanField = 16u;  // mean T^lat not > 0 at a mean-field refresh
constexpr unsigned kErrMass = 32u;       // a mass not finite and > 0 (lattice-side kernels)

// One wavefront-sized slice of 64 consecutive internal atoms.  The neighbour
// indices of the slice are stored column-major: entry k of lane l lives at
// col[64 * col_base64 + 64 * k + l]; lanes with fewer than `width` neighbours
// are padded with their own index, whose pair term is exactly zero.
struct SliceInfo {
    int32_t sys;
    int32_t width;
    int32_t col_base64;
    int32_t n_valid;
    int32_t brick;      // brick that owns the slice
    int32_t colw_base64;  // packed brick-local table: word k/2 of lane l at 64*(colw_base64 + k/2) + l
    int32_t flags;      // kSliceHeld: some atom of the slice holds its T_e
    int32_t pad_;
};
constexpr int32_t kSliceHeld = 1;

// A brick of up to b x b x b cells: its own slots (padded to 64) and the halo
// atoms of the surrounding one-cell shell, staged together in LDS.  shell maps
// a shell position (o - 1 .. o + e, per axis) to -1 (own cell), -2 (outside a
// free boundary) or the cell's offset in the brick's halo list.
struct BrickInfo {
    int32_t slot0, n_own, n_own_pad, slice0;
    int32_t halo_off, n_halo, shell_off, sys;
    int32_t o[3];       // first cell of the brick (grid coordinates)
    int32_t sh[3];      // shell extent per axis (brick extent + 2)
};

struct HaloCell {
    int32_t brick, start_index, offset, pos_base;
};

// Per-system constants as the kernels read them.
struct DevParams {
    double T_min, span, inv_span, K, A, dt, g;
    double ce_const, gamma, ce_cap;
    double i0, lp, t0, sigma, inv_sigma, x0;
    int32_t ce_model, laser_on;
    int32_t atom_off, n_pad;
    int32_t slice0, n_slices;
    // FP32 copies for the compensated path
    float f_inv_span, f_half_inv_span, f_m_off, f_A, f_K, f_dt, f_g;
    float f_ce_const, f_gamma, f_ce_cap, f_T_min, f_T_max, f_i0;
    float f_inv2, f_c_tiny, f_w_tiny;
    // fixed electronic temperatures (sign bit of the source weight) and the
    // mean-field refresh of c and K at the start of every advance
    int32_t has_fixed, mean_field;
    int32_t n_atoms, pad_;
    double mf_lambda, mf_kcoef;
    int32_t mf_chunk0, mf_nchunk;   // this system's chunks in the mean-field chunk table
    // two-temperature lattice (Section 3.1): T^lat evolves with the electrons
    int32_t lat_fd, pad2_;
    double K_lat, g_over_clat;
};

// mean-field reduction: a system's slices in chunks of kMfChunk slices
constexpr int32_t kMfChunk = 32;
struct MfChunk {
    int32_t sys, slice_begin, slice_end, pad_;
};

struct SystemState {
    l2t_system_desc desc{};
    l2t_params params{};
    bool has_pos = false, has_params = false, has_te = false, has_tl = false;
    int64_t caller_off = 0;      // offset of this system in concatenated caller arrays
    int32_t atom_off = 0;        // first internal slot
    int32_t n_pad = 0;           // internal slots (multiple of 64)
    int32_t slice0 = 0, n_slices = 0;
    int32_t list0 = 0, n_list = 0;   // this system's non-empty bricks in the brick list
    int32_t nc[3] = {1, 1, 1};
    int64_t cell_off = 0, ncell = 0;
    int64_t step = 0;            // sub-steps since the last T_e write
    bool eatom_valid = false;    // the per-atom ledger holds this system's last advance
    bool has_fixed = false;      // some atoms hold their T_e
    l2t_mean_field mf{};         // mean-field parameter mode
    l2t_lattice_fd lf{};         // two-temperature lattice mode
    int32_t max_nbrs = 0;
};

struct GraphKey {
    int32_t n, mode, sys;
    bool operator<(const GraphKey &o) const {
        if (n != o.n) return n < o.n;
        if (mode != o.mode) return mode < o.mode;
        return sys < o.sys;
    }
};

// sub-steps per captured hipGraph of the FP32C advance (even, so a replay
// leaves the state in the buffer it started from)
constexpr int32_t kGraphChunk = 256;

// grow-only temporary buffers of the neighbour build (tmp_buf slots)
constexpr int kTmpSlots = 17;

constexpr int kKernelSliced = 0;   // global gathers through the int32 table
constexpr int kKernelBrick = 1;    // LDS tile per brick, uint16 table
constexpr int kBrickBlockMax = 512;   // threads per workgroup, brick kernel
// entries a brick's halo list takes: its length rounded up to a multiple of 4
__host__ __device__ constexpr int32_t halo_padded(int32_t n_halo) { return (n_halo + 3) & ~3; }

constexpr int32_t kMaxBrickEdge = 1024;  // largest brick edge (cells) the layout considers
constexpr int kSlicedBlockMax = 256;  // threads per workgroup, global-gather kernels
constexpr int kResidentMaxSlots = 1024;  // largest system one workgroup keeps in LDS

// one system of a resident (whole system per workgroup) launch
struct ResidentSys {
    int32_t sys, slot0, n_pad, slice0;
};

struct Tuning {
    int kernel = kKernelBrick;
    int persistent = 0;
    int block = kBrickBlockMax;
    int resident_max = 0;    // 0 = autotune
    int graph = 2;           // L2T_OPT_GRAPH as set: 0 = direct, 1 = graphs, 2 = timed by the autotuner
    int graph_used = 1;      // FP32C advance, in effect: 0 = direct launches, 1 = graph replays
    int autotune = 1;
    int brick_edge = 0;      // 0 = chosen by the layout builder
    int sweep = 0;           // L2T_OPT_SWEEP as set: 0 = chosen at neighbour build, 1, 2
    int sweep_used = 1;      // in effect: 1 = fixed order, 2 = reversed on odd sub-steps
    int table = 0;           // L2T_OPT_TABLE_STREAM as set: 0 = chosen at neighbour build, 1, 2
    int table_used = 1;      // in effect: 1 = cached table loads, 2 = non-temporal
    bool tuned = false;
    bool pinned = false;     // an explicit option was set: keep the choice
};

struct Recording {
    bool valid = false;
    int32_t n_steps = 0, ckpt = 0;
    int64_t n_ckpt = 0;
    std::vector<int64_t> step0;   // per-system step index at the start
    void *buf = nullptr;          // checkpoints [n_ckpt][state words per atom][n_int]
    size_t bytes = 0;
};

}  // namespace l2t

struct l2t_ctx {
    int precision = L2T_FP32C;
    hipStream_t stream = nullptr;
    // the caller's device allocator (l2t_set_allocator); unset: hipMalloc / hipFree
    void *(*ualloc)(size_t, void *) = nullptr;
    void (*ufree)(void *, void *) = nullptr;
    void *uarg = nullptr;
    // blocks that came from a caller allocator, with the call that releases each
    struct UserBlock {
        void (*free_)(void *, void *);
        void *arg;
    };
    std::unordered_map<void *, UserBlock> user_blocks;
    hipStream_t cap_stream = nullptr;   // private stream used only to capture graphs
    int device = 0;
    int n_cu = 256;
    size_t lds_per_block = 65536;
    std::vector<l2t::SystemState> sys;
    int64_t n_tot = 0;           // sum of caller atoms
    int32_t n_int = 0;           // internal slots (systems padded to 64)
    int32_t n_slices = 0;
    int32_t max_n = 0;
    double r_cut = 0.0;
    bool nbrs_built = false;
    bool layout_built = false;   // an internal order exists (kept by l2t_set_positions)
    int32_t max_nbrs = 0;
    double mean_nbrs = 0.0;

    // device buffers (owned)
    double *pos = nullptr;       // caller order SoA [3][n_tot]
    double *pos_int = nullptr;   // internal order SoA [3][n_int]
    int32_t *perm = nullptr;     // internal slot -> caller-global index (-1 = padding)
    int32_t *inv = nullptr;      // caller-global index -> internal slot
    int32_t *cell_start = nullptr;
    int32_t *cell_scratch = nullptr;
    int32_t *cell_of = nullptr;  // caller order [n_tot]
    int32_t *cell_int = nullptr; // internal order [n_int]
    int32_t *sorted_local = nullptr;
    int32_t *cnt = nullptr;      // internal [n_int]
    l2t::SliceInfo *slices = nullptr;
    int32_t *col = nullptr;
    uint32_t *colw = nullptr;    // brick-local table: two LDS byte offsets per word
    int64_t colw_len = 0;
    int32_t *pos_slot = nullptr; // caller layout [n_tot]: cell-order position -> slot
    l2t::BrickInfo *bricks = nullptr;
    int32_t *brick_list = nullptr;   // non-empty bricks
    // launch list of the all-system brick kernels: the brick list cut into 8
    // contiguous ranges of equal estimated work, range x at [x G/8, (x+1) G/8)
    // followed by -1 holes, so that workgroup b (on XCD b mod 8) takes entry
    // (b mod 8) G/8 + b/8; G = n_xcd_list.  A second list of G entries follows
    // with every range reversed (the odd sub-steps of the alternating sweep).
    int32_t *xcd_list = nullptr;
    int32_t n_xcd_list = 0;
    size_t cap_xl = 0;
    std::vector<int32_t> h_xcd_list;   // host copy (the upload reads it asynchronously)
    int32_t *shell = nullptr;
    int32_t *halo = nullptr;
    int32_t n_bricks = 0, n_brick_list = 0, tile_max = 0, brick_edge_used = 0;
    int64_t col_len = 0;
    int64_t col_used = 0;
    double mean_width = 0.0;     // mean row length of the sliced table (padding included)
    int64_t cells_total = 0;

    double *T64[2] = {nullptr, nullptr};
    double *Tl64 = nullptr;
    double *Tl64b = nullptr;     // second T^lat buffer of the two-temperature lattice mode
    double *srcw64 = nullptr;
    float *Thi[2] = {nullptr, nullptr};
    int16_t *Tlo = nullptr;   // FP32C state: the 16-bit low part q of every slot
    float *Tl32 = nullptr;
    float *srcw32 = nullptr;
    int cur = 0;

    double *ledger = nullptr;    // [n_slices][3]
    l2t::MfChunk *mf_chunks = nullptr;   // mean-field chunk table
    std::vector<l2t::MfChunk> h_mf_chunks;   // its host copy (source of the upload)
    int32_t n_mf_chunks = 0, mf_chunks_cap = 0;
    double *eatom = nullptr;     // internal [n_int]: energy to the lattice over the last advance
    bool atom_ledger = false;    // record eatom during advances
    bool batch_fp64 = false;     // FP64: one launch per sub-step over all systems
    l2t::ResidentSys *res = nullptr;       // resident launch table (device)
    std::vector<l2t::ResidentSys> h_res;   // its host copy (source of the upload)
    size_t res_cap = 0;
    bool res_valid = false;                // false after a rebuild
    bool eatom_valid = false;    // eatom holds the record of the last advance
    double *slice_red = nullptr; // [n_slices][4]
    double *energy_out = nullptr;// [n_sys][8]
    l2t::DevParams *dparams = nullptr;
    int64_t *dstep = nullptr;    // per-system step index
    unsigned *derr = nullptr;
    unsigned *dbar = nullptr;    // grid barrier words
    double *stage = nullptr;     // staging [max(n_tot, 3 * max_n)]
    void *scratch = nullptr;     // temporary (autotune snapshot, velocities)
    size_t scratch_bytes = 0;
    double *carry = nullptr;     // T_e, T^lat and gate in caller order across a rebuild
    size_t carry_len = 0;
    // grow-only capacities of the internal-order buffers and the brick tables
    size_t cap_ni = 0, cap_nb = 0, cap_nl = 0, cap_sh = 0, cap_ha = 0;
    // grow-only temporaries of the neighbour build, one per use
    void *tmp[l2t::kTmpSlots] = {};
    size_t tmp_cap[l2t::kTmpSlots] = {};

    std::vector<l2t::DevParams> hparams;
    l2t::Tuning tune;
    std::map<l2t::GraphKey, hipGraphExec_t> graphs;
    l2t::Recording rec;
    std::string last_error;
};

namespace l2t {

// ---- status helpers (api.cpp) ---------------------------------------------
int fail(l2t_ctx *c, int status, const std::string &msg);
int hip_fail(l2t_ctx *c, hipError_t e, const char *what);

#define L2T_HIP(ctx, expr)                                              \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return ::l2t::hip_fail((ctx), e_, #expr); \
    } while (0)

// ---- geometry (k_geometry.hip) ---------------------------------------------
int build_neighbors(l2t_ctx *c, double r_cut);
int permute_in(l2t_ctx *c, int32_t sys, const double *src_dev, int32_t field);
int permute_out(l2t_ctx *c, int32_t sys, int32_t field, double *dst_dev);
int mark_held_slices(l2t_ctx *c, int32_t sys);   // kSliceHeld from the held atoms
int lattice_temperature(l2t_ctx *c, int32_t sys, const double *v_caller, const double *m_caller,
                        int32_t global_com);
// Eq. 4 staged through the file-scope device array of k_geometry.hip instead
// of the context's scratch buffer: allocates nothing.  EINVAL when the system
// needs more than kStaticScratchBytes (4 doubles per padded slot + 4).
int lattice_temperature_static(l2t_ctx *c, int32_t sys, const double *v_dev, const double *m_dev,
                               int32_t global_com);
// device address of that array on `device` (current), looked up once per device
int static_scratch_init(int device);
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
int neighbors_to_host(l2t_ctx *c, int32_t sys, int64_t *row_ptr, int32_t *col, int64_t cap);
int source_weights(l2t_ctx *c, int32_t sys);
int check_field_range(l2t_ctx *c, const double *src_dev, int64_t n, double lo, double hi,
                      bool *ok);

// ---- sub-steps (k_step.hip) ------------------------------------------------
int upload_params(l2t_ctx *c);
int advance_plain(l2t_ctx *c, int32_t sys, int32_t n);    // FP64 or FP32C, one launch per sub-step
int advance_fp32c(l2t_ctx *c, int32_t n);                 // all systems, tuned path
int reset_ledger(l2t_ctx *c, int32_t sys);
int energies(l2t_ctx *c, int32_t sys, l2t_energy_report *out);
int pair_fp32(const float *ti, const float *tj, float *out, int64_t n, hipStream_t s);
int fp32c_launch(l2t_ctx *c, int32_t n, int kernel, int persistent, int block, double *eatom);
// n FP32C sub-steps of all systems captured into an executable graph (the caller destroys it)
int capture_fp32c(l2t_ctx *c, int32_t n, int kernel, int persistent, int block, double *eatom,
                  hipGraphExec_t *out);
// time n brick-kernel sub-steps of the current layout on a stand-in state in
// scratch memory (the context's fields are not touched)
int brick_probe(l2t_ctx *c, int32_t n, bool alternate, bool stream, float *ms);
// the launch list of sub-step k of an advance (the reversed one on odd k when
// the alternating sweep is in effect)
inline const int32_t *xcd_list_for(const l2t_ctx *c, int64_t k) {
    return c->xcd_list + ((c->tune.sweep_used == 2 && (k & 1)) ? c->n_xcd_list : 0);
}
// per-atom record of the energy handed to the lattice (nullptr while off)
inline double *atom_ledger_ptr(l2t_ctx *c) { return c->atom_ledger ? c->eatom : nullptr; }
int zero_atom_ledger(l2t_ctx *c, int32_t sys);   // sys < 0: every system
// c and K of mean-field systems from their current means (sys < 0: all)
int mean_field_refresh(l2t_ctx *c, int32_t sys);
int bump_steps(l2t_ctx *c, int32_t sys, int32_t n);
void drop_graphs(l2t_ctx *c);
int brick_step_fp32c(l2t_ctx *c, int block, const float *Thi, float *Thi_n, const int16_t *lo_in,
                     int16_t *Tlo, const int64_t *dstep, int32_t rel, double *ledger);

// ---- lattice side (k_lattice.hip) ------------------------------------------
int coupling(l2t_ctx *c, int32_t sys, int32_t mode, double dt_md, const double *v_dev,
             const double *m_dev, double *xi_dev);
int damping_step(hipStream_t s, int64_t n, double dt_md, const double *xi, const double *force,
                 const double *mass, double *v, unsigned *err);

// ---- adjoint (k_adjoint.hip) ------------------------------------------------
int record_checkpoint(l2t_ctx *c, int64_t slot);
int adjoint(l2t_ctx *c, const double *dL_dTN_dev, double *dL_dK, double *dL_dg,
            double *dL_dT0_dev);

// ---- autotuner (autotune.cpp) ------------------------------------------------
int autotune(l2t_ctx *c);

// ---- buffers ---------------------------------------------------------------
int ensure_scratch(l2t_ctx *c, size_t bytes);
// every device buffer of a context: from the caller's allocator when one is
// set, else hipMalloc; dev_free releases a block through whichever made it
hipError_t dev_malloc(l2t_ctx *c, void **p, size_t bytes);
void dev_free(l2t_ctx *c, void *p);
// temporary device buffer `slot` of at least n elements (kept for the next call)
void *tmp_buf(l2t_ctx *c, int slot, size_t bytes);
template <class T>
inline T *tmp_of(l2t_ctx *c, int slot, int64_t n) {
    return static_cast<T *>(tmp_buf(c, slot, sizeof(T) * (size_t)(n > 0 ? n : 1)));
}
// (re)allocate every internal-order buffer for n_int slots and the brick tables
int alloc_internal(l2t_ctx *c, int32_t n_int, int32_t n_bricks, int32_t n_list, int64_t shell_len,
                   int64_t halo_len);


}  // namespace l2t
