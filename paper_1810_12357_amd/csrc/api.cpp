// Host side of the C ABI declared in include/l2t.h: argument validation,
// device buffers, call-order state, error reporting.  All arithmetic of the
// method runs in the kernels of k_geometry.hip, k_step.hip and k_adjoint.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "l2t_internal.h"

using l2t::SystemState;

namespace l2t {

int fail(l2t_ctx *c, int status, const std::string &msg) {
    if (c) c->last_error = msg;
    return status;
}

int hip_fail(l2t_ctx *c, hipError_t e, const char *what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return fail(c, L2T_ENOMEM, m);
    return fail(c, L2T_EHIP, m);
}

hipError_t dev_malloc(l2t_ctx *c, void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 1;
    if (!c->ualloc) return hipMalloc(p, bytes);
    void *q = c->ualloc(bytes, c->uarg);
    if (!q) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {   // the kernels stage 16-byte vectors
        c->ufree(q, c->uarg);
        return hipErrorInvalidValue;
    }
    c->user_blocks[q] = l2t_ctx::UserBlock{c->ufree, c->uarg};
    *p = q;
    return hipSuccess;
}

void dev_free(l2t_ctx *c, void *p) {
    if (!p) return;
    auto it = c->user_blocks.find(p);
    if (it == c->user_blocks.end()) {
        (void)hipFree(p);
        return;
    }
    const l2t_ctx::UserBlock b = it->second;
    c->user_blocks.erase(it);
    // the block goes back to the caller: nothing queued on the stream may use it
    (void)hipStreamSynchronize(c->stream);
    b.free_(p, b.arg);
}

int ensure_scratch(l2t_ctx *c, size_t bytes) {
    if (bytes <= c->scratch_bytes) return L2T_OK;
    if (c->scratch) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, c->scratch);
    }
    c->scratch = nullptr;
    c->scratch_bytes = 0;
    if (dev_malloc(c, &c->scratch, bytes) != hipSuccess)
        return fail(c, L2T_ENOMEM, "scratch allocation failed");
    c->scratch_bytes = bytes;
    return L2T_OK;
}

}  // namespace l2t

namespace {

template <typename T>
int dalloc(l2t_ctx *c, T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    void *q = nullptr;
    hipError_t e = l2t::dev_malloc(c, &q, sizeof(T) * count);
    if (e != hipSuccess) return l2t::hip_fail(c, e, "device allocation");
    *p = (T *)q;
    e = hipMemsetAsync(*p, 0, sizeof(T) * count, c->stream);
    if (e != hipSuccess) return l2t::hip_fail(c, e, "hipMemsetAsync");
    return L2T_OK;
}

template <typename T>
void dfree(l2t_ctx *c, T *&p) {
    l2t::dev_free(c, (void *)p);
    p = nullptr;
}

}  // namespace

namespace l2t {

void *tmp_buf(l2t_ctx *c, int slot, size_t bytes) {
    if (bytes > c->tmp_cap[slot]) {
        (void)hipStreamSynchronize(c->stream);
        dev_free(c, c->tmp[slot]);
        c->tmp[slot] = nullptr;
        c->tmp_cap[slot] = 0;
        if (dev_malloc(c, &c->tmp[slot], bytes) != hipSuccess) return nullptr;
        c->tmp_cap[slot] = bytes;
    }
    return c->tmp[slot];
}

// Size the internal-order buffers for n_int slots and the brick tables.
// Buffers only grow: a rebuild of the same shape (every pass of an MD loop)
// keeps every allocation.  Their contents are rewritten by the build and by
// the field setters, which a rebuild requires anyway.
int alloc_internal(l2t_ctx *c, int32_t n_int, int32_t n_bricks, int32_t n_list, int64_t shell_len,
                   int64_t halo_len) {
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    c->n_int = n_int;
    c->n_slices = n_int / kWave;
    c->n_bricks = n_bricks;
    c->n_brick_list = n_list;
    c->cur = 0;
    int rc = L2T_OK;
#define ALLOC(p, n)                                    \
    if (rc == L2T_OK) rc = dalloc(c, &(p), (size_t)(n));
    if ((size_t)n_int > c->cap_ni) {
        dfree(c, c->pos_int);
        dfree(c, c->perm);
        dfree(c, c->cell_int);
        dfree(c, c->cnt);
        dfree(c, c->slices);
        for (int b = 0; b < 2; ++b) {
            dfree(c, c->T64[b]);
            dfree(c, c->Thi[b]);
        }
        dfree(c, c->Tl64);
        dfree(c, c->Tl64b);
        dfree(c, c->srcw64);
        dfree(c, c->Tlo);
        dfree(c, c->Tl32);
        dfree(c, c->srcw32);
        dfree(c, c->ledger);
        dfree(c, c->eatom);
        dfree(c, c->slice_red);
        c->cap_ni = 0;
        const size_t NI = (size_t)n_int, NS = NI / kWave;
        ALLOC(c->pos_int, 3 * NI);
        ALLOC(c->perm, NI);
        ALLOC(c->cell_int, NI);
        ALLOC(c->cnt, NI);
        ALLOC(c->slices, NS);
        if (c->precision == L2T_FP64) {
            ALLOC(c->T64[0], NI);
            ALLOC(c->T64[1], NI);
            ALLOC(c->Tl64, NI);
            ALLOC(c->Tl64b, NI);
            ALLOC(c->srcw64, NI);
        } else {
            ALLOC(c->Thi[0], NI);
            ALLOC(c->Thi[1], NI);
            ALLOC(c->Tlo, NI);
            ALLOC(c->Tl32, NI);
            ALLOC(c->srcw32, NI);
        }
        ALLOC(c->ledger, 3 * NS);
        ALLOC(c->eatom, NI);
        ALLOC(c->slice_red, 4 * NS);
        if (rc == L2T_OK) c->cap_ni = NI;
    }
    auto grow = [&](auto *&p, size_t &cap, size_t n) {
        if (rc != L2T_OK || n <= cap) return;
        dfree(c, p);
        cap = 0;
        rc = dalloc(c, &p, n);
        if (rc == L2T_OK) cap = n;
    };
    grow(c->bricks, c->cap_nb, (size_t)n_bricks);
    grow(c->brick_list, c->cap_nl, (size_t)n_list);
    grow(c->shell, c->cap_sh, (size_t)shell_len);
    grow(c->halo, c->cap_ha, (size_t)halo_len);
#undef ALLOC
    if (rc != L2T_OK) return fail(c, L2T_ENOMEM, "internal buffer allocation failed");
    return L2T_OK;
}

}  // namespace l2t

namespace {

bool bad_sys(const l2t_ctx *c, int32_t sys) {
    return !c || sys < 0 || sys >= (int32_t)c->sys.size();
}

// copy a caller buffer to device memory if it lives on the host
int stage_in(l2t_ctx *c, const double *src, size_t count, int32_t mem, double *staging,
             const double **dev) {
    if (mem == L2T_DEVICE) {
        *dev = src;
        return L2T_OK;
    }
    if (mem != L2T_HOST) return l2t::fail(c, L2T_EINVAL, "mem must be L2T_HOST or L2T_DEVICE");
    L2T_HIP(c, hipMemcpyAsync(staging, src, sizeof(double) * count, hipMemcpyHostToDevice,
                              c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    *dev = staging;
    return L2T_OK;
}

int check_err(l2t_ctx *c) {
    unsigned h = 0;
    L2T_HIP(c, hipMemcpyAsync(&h, c->derr, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    if (h) L2T_HIP(c, hipMemsetAsync(c->derr, 0, sizeof(unsigned), c->stream));
    if (h & l2t::kErrBarrier)
        return l2t::fail(c, L2T_EHIP, "persistent sub-step launch: grid barrier spin limit reached");
    if (h & l2t::kErrRange)
        return l2t::fail(c, L2T_ERANGE,
                         "a sub-step produced theta outside [0,1] or a non-finite temperature");
    if (h & l2t::kErrMeanField)
        return l2t::fail(c, L2T_ERANGE, "mean-field refresh: a system's mean T_lat is not > 0");
    if (h & l2t::kErrMass)
        return l2t::fail(c, L2T_EINVAL, "coupling or damping step: a mass is not finite and > 0");
    return L2T_OK;
}

// start of an advance over systems [s0, s1): clear their per-atom ledger
// while recording; otherwise the old record no longer describes the last advance
int begin_atom_ledger(l2t_ctx *c, int32_t s0, int32_t s1) {
    for (int32_t s = s0; s < s1; ++s) c->sys[s].eatom_valid = c->atom_ledger;
    if (!c->atom_ledger) return L2T_OK;
    if (s1 - s0 == (int32_t)c->sys.size()) return l2t::zero_atom_ledger(c, -1);
    for (int32_t s = s0; s < s1; ++s) {
        int rc = l2t::zero_atom_ledger(c, s);
        if (rc != L2T_OK) return rc;
    }
    return L2T_OK;
}

bool ready_to_advance(l2t_ctx *c, int32_t s0, int32_t s1, std::string *why) {
    if (!c->nbrs_built) {
        *why = "neighbour sets not built";
        return false;
    }
    for (int32_t s = s0; s < s1; ++s) {
        const SystemState &st = c->sys[s];
        if (!st.has_params) {
            *why = "parameters of system " + std::to_string(s) + " not set";
            return false;
        }
        if (!st.has_te) {
            *why = "T_e of system " + std::to_string(s) + " not set";
            return false;
        }
        if (st.params.g > 0.0 && !st.has_tl) {
            *why = "T_lat of system " + std::to_string(s) + " not set (G > 0)";
            return false;
        }
    }
    return true;
}

}  // namespace

extern "C" {

int l2t_version(void) { return 10100; }

const char *l2t_strerror(int status) {
    switch (status) {
        case L2T_OK: return "ok";
        case L2T_WUNSTABLE: return "warning: explicit sub-step may be unstable";
        case L2T_EINVAL: return "invalid argument";
        case L2T_ENOMEM: return "out of device memory";
        case L2T_EHIP: return "HIP runtime error";
        case L2T_ESTATE: return "call out of order";
        case L2T_ERANGE: return "temperature outside [T_min, T_max] or non-finite";
        case L2T_ENOTIMPL: return "not implemented";
        default: return "unknown status";
    }
}

const char *l2t_last_error(const l2t_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

double l2t_exchange_rate(double kappa_e, double C_e, int32_t dim, double lattice_sum) {
    if (!(kappa_e > 0.0) || !(C_e > 0.0) || dim < 1 || !(lattice_sum > 0.0)) return NAN;
    return 2.0 * kappa_e * (double)dim / (C_e * lattice_sum);
}

void l2t_destroy(l2t_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    l2t::drop_graphs(c);
    dfree(c, c->res);
    dfree(c, c->pos);
    dfree(c, c->pos_int);
    dfree(c, c->perm);
    dfree(c, c->inv);
    dfree(c, c->cell_start);
    dfree(c, c->cell_scratch);
    dfree(c, c->cell_of);
    dfree(c, c->cell_int);
    dfree(c, c->sorted_local);
    dfree(c, c->cnt);
    dfree(c, c->slices);
    dfree(c, c->col);
    dfree(c, c->colw);
    dfree(c, c->pos_slot);
    dfree(c, c->bricks);
    dfree(c, c->brick_list);
    dfree(c, c->xcd_list);
    dfree(c, c->shell);
    dfree(c, c->halo);
    for (int b = 0; b < 2; ++b) {
        dfree(c, c->T64[b]);
        dfree(c, c->Thi[b]);
    }
    dfree(c, c->Tl64);
    dfree(c, c->Tl64b);
    dfree(c, c->srcw64);
    dfree(c, c->Tlo);
    dfree(c, c->Tl32);
    dfree(c, c->srcw32);
    dfree(c, c->ledger);
    dfree(c, c->eatom);
    dfree(c, c->slice_red);
    dfree(c, c->energy_out);
    l2t::dev_free(c, c->mf_chunks);
    dfree(c, c->dparams);
    dfree(c, c->dstep);
    dfree(c, c->derr);
    dfree(c, c->dbar);
    dfree(c, c->stage);
    l2t::dev_free(c, c->scratch);
    l2t::dev_free(c, c->carry);
    for (void *p : c->tmp) l2t::dev_free(c, p);
    l2t::dev_free(c, c->rec.buf);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

int l2t_create(l2t_ctx **out, int32_t n_systems, const l2t_system_desc *descs, int32_t precision,
               void *hip_stream) {
    if (!out) return L2T_EINVAL;
    *out = nullptr;
    if (n_systems < 1 || !descs) return L2T_EINVAL;
    if (precision != L2T_FP64 && precision != L2T_FP32C) return L2T_EINVAL;
    int64_t n_tot = 0, n_int = 0;
    for (int32_t s = 0; s < n_systems; ++s) {
        const l2t_system_desc &d = descs[s];
        if (d.n_atoms < 1) return L2T_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!(d.box_len[k] > 0.0) || !std::isfinite(d.box_lo[k]) || !std::isfinite(d.box_len[k]))
                return L2T_EINVAL;
        n_tot += d.n_atoms;
        n_int += (d.n_atoms + l2t::kWave - 1) / l2t::kWave * l2t::kWave;
    }
    if (n_tot > INT32_MAX / 4 || n_int > INT32_MAX / 4) return L2T_EINVAL;
    int dev = 0, ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return L2T_EHIP;
    if (hipGetDevice(&dev) != hipSuccess) return L2T_EHIP;
    l2t_ctx *c = new (std::nothrow) l2t_ctx();
    if (!c) return L2T_ENOMEM;
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    c->device = dev;
    // device address of the allocation-free entry point's staging array on
    // this device (looked up once per device; a failure is reported by that
    // entry point, not here)
    (void)l2t::static_scratch_init(dev);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        c->n_cu = prop.multiProcessorCount;
        c->lds_per_block = prop.sharedMemPerBlock;
    }
    c->sys.resize(n_systems);
    int64_t coff = 0;
    int32_t aoff = 0;
    for (int32_t s = 0; s < n_systems; ++s) {
        SystemState &st = c->sys[s];
        st.desc = descs[s];
        st.caller_off = coff;
        st.atom_off = aoff;
        st.n_pad = (descs[s].n_atoms + l2t::kWave - 1) / l2t::kWave * l2t::kWave;
        st.slice0 = aoff / l2t::kWave;
        st.n_slices = st.n_pad / l2t::kWave;
        coff += descs[s].n_atoms;
        aoff += st.n_pad;
        c->max_n = std::max(c->max_n, descs[s].n_atoms);
    }
    c->n_tot = n_tot;
    c->n_int = (int32_t)n_int;
    c->n_slices = (int32_t)(n_int / l2t::kWave);
    const size_t S = (size_t)n_systems, NT = (size_t)n_tot;
    int rc = L2T_OK;
#define ALLOC(p, n)                                    \
    if (rc == L2T_OK) rc = dalloc(c, &(p), (size_t)(n));
    ALLOC(c->pos, 3 * NT);
    ALLOC(c->inv, NT);
    ALLOC(c->cell_of, NT);
    ALLOC(c->sorted_local, NT);
    ALLOC(c->pos_slot, NT);
    ALLOC(c->energy_out, 8);
    ALLOC(c->dparams, S);
    ALLOC(c->dstep, S);
    ALLOC(c->derr, 4);
    ALLOC(c->dbar, 4);
    ALLOC(c->stage, std::max<size_t>(NT, 4 * (size_t)c->max_n));
#undef ALLOC
    if (rc == L2T_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = L2T_EHIP;
    if (rc != L2T_OK) {
        l2t_destroy(c);
        return rc;
    }
    *out = c;
    return L2T_OK;
}

int l2t_set_positions(l2t_ctx *c, int32_t sys, const double *xyz, int32_t mem) {
    if (bad_sys(c, sys) || !xyz) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    SystemState &st = c->sys[sys];
    const int32_t n = st.desc.n_atoms;
    const hipMemcpyKind kind = mem == L2T_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    for (int d = 0; d < 3; ++d)
        L2T_HIP(c, hipMemcpyAsync(c->pos + (size_t)d * c->n_tot + st.caller_off,
                                  xyz + (size_t)d * n, sizeof(double) * n, kind, c->stream));
    if (mem == L2T_HOST) L2T_HIP(c, hipStreamSynchronize(c->stream));
    st.has_pos = true;
    c->nbrs_built = false;
    return L2T_OK;
}

static int restore_counters(l2t_ctx *c, int32_t sys, int64_t step, double E_e_to_l, double E_src,
                            double T_ledger_acc);

int l2t_build_neighbors(l2t_ctx *c, double r_cut, int32_t *max_nbrs, double *mean_nbrs) {
    if (!c) return L2T_EINVAL;
    if (!(r_cut > 0.0) || !std::isfinite(r_cut)) return l2t::fail(c, L2T_EINVAL, "r_cut <= 0");
    for (size_t s = 0; s < c->sys.size(); ++s)
        if (!c->sys[s].has_pos)
            return l2t::fail(c, L2T_ESTATE, "positions of system " + std::to_string(s) + " not set");
    // each system's T_e, T^lat and gate leave the old internal order for the
    // caller's, and come back in the new order after the build (the FP32C
    // state round-trips through FP64 bit for bit); the ledger and the step
    // counter run on
    const int32_t S = (int32_t)c->sys.size();
    std::vector<char> keep_te(S, 0), keep_tl(S, 0);
    bool keep = false;
    for (int32_t s = 0; s < S && c->layout_built; ++s) {
        keep_te[s] = c->sys[s].has_te;
        keep_tl[s] = c->sys[s].has_tl;
        keep |= keep_te[s] || keep_tl[s];
    }
    const size_t nt = (size_t)c->n_tot;
    if (keep && 3 * nt > c->carry_len) {
        L2T_HIP(c, hipStreamSynchronize(c->stream));
        l2t::dev_free(c, c->carry);
        c->carry = nullptr;
        c->carry_len = 0;
        void *m = nullptr;
        if (l2t::dev_malloc(c, &m, sizeof(double) * 3 * nt) != hipSuccess)
            return l2t::fail(c, L2T_ENOMEM, "field carry buffer allocation failed");
        c->carry = static_cast<double *>(m);
        c->carry_len = 3 * nt;
    }
    // the ledger rows follow the slices, which the build lays out anew: the
    // kept systems' totals and step counters go back into their first rows
    std::vector<l2t_energy_report> kept(S);
    for (int32_t s = 0; s < S && keep; ++s) {
        double *base = c->carry + c->sys[s].caller_off;
        int rc = L2T_OK;
        if (keep_te[s]) rc = l2t::energies(c, s, &kept[s]);
        if (rc == L2T_OK && keep_te[s]) rc = l2t::permute_out(c, s, L2T_FIELD_TE, base);
        if (rc == L2T_OK && keep_tl[s]) rc = l2t::permute_out(c, s, L2T_FIELD_TL, base + nt);
        if (rc == L2T_OK && keep_tl[s]) rc = l2t::permute_out(c, s, L2T_FIELD_GATE, base + 2 * nt);
        if (rc != L2T_OK) return rc;
    }
    l2t::drop_graphs(c);
    c->rec.valid = false;
    int rc = l2t::build_neighbors(c, r_cut);
    if (rc != L2T_OK) {
        for (auto &st : c->sys) st.has_te = st.has_tl = false;   // the fields are lost
        c->layout_built = false;
        return rc;
    }
    c->nbrs_built = true;
    c->layout_built = true;
    c->res_valid = false;
    if (!c->tune.pinned) c->tune.tuned = false;   // new layout: tune again unless pinned
    for (auto &st : c->sys) {
        st.has_te = false;   // internal order changed: written again below where kept
        st.has_tl = false;
        st.eatom_valid = false;
        st.has_fixed = false;
    }
    // per-atom fields start at zero (T^lat = 0, no gate, no fixed atoms)
    if (c->precision == L2T_FP64) {
        L2T_HIP(c, hipMemsetAsync(c->Tl64, 0, sizeof(double) * c->n_int, c->stream));
        L2T_HIP(c, hipMemsetAsync(c->srcw64, 0, sizeof(double) * c->n_int, c->stream));
    } else {
        L2T_HIP(c, hipMemsetAsync(c->Tl32, 0, sizeof(float) * c->n_int, c->stream));
        L2T_HIP(c, hipMemsetAsync(c->srcw32, 0, sizeof(float) * c->n_int, c->stream));
    }
    rc = l2t::upload_params(c);   // new layout offsets, no fixed atoms
    if (rc != L2T_OK) return rc;
    for (int32_t s = 0; s < (int32_t)c->sys.size(); ++s)
        if (c->sys[s].has_params) {
            rc = l2t::source_weights(c, s);
            if (rc != L2T_OK) return rc;
        }
    for (int32_t s = 0; s < S && keep; ++s) {
        const double *base = c->carry + c->sys[s].caller_off;
        if (keep_te[s]) {
            rc = l2t::permute_in(c, s, base, L2T_FIELD_TE);
            if (rc == L2T_OK)
                rc = restore_counters(c, s, kept[s].step, kept[s].E_e_to_l, kept[s].E_src,
                                      kept[s].T_ledger_acc);
            if (rc != L2T_OK) return rc;
            c->sys[s].has_te = true;
        }
        if (keep_tl[s]) {
            rc = l2t::permute_in(c, s, base + nt, L2T_FIELD_TL);
            if (rc == L2T_OK) rc = l2t::permute_in(c, s, base + 2 * nt, L2T_FIELD_GATE);
            if (rc != L2T_OK) return rc;
            c->sys[s].has_tl = true;
        }
    }
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    if (max_nbrs) *max_nbrs = c->max_nbrs;
    if (mean_nbrs) *mean_nbrs = c->mean_nbrs;
    return L2T_OK;
}

int l2t_get_neighbors(l2t_ctx *c, int32_t sys, int64_t *row_ptr, int32_t *col, int64_t cap) {
    if (bad_sys(c, sys) || !row_ptr) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    return l2t::neighbors_to_host(c, sys, row_ptr, col, cap);
}

int l2t_set_params(l2t_ctx *c, int32_t sys, const l2t_params *p) {
    if (bad_sys(c, sys) || !p) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    const l2t_params &q = *p;
    auto fin = [](double v) { return std::isfinite(v); };
    if (!fin(q.T_min) || !fin(q.T_max) || !(q.T_max > q.T_min) || q.T_min < 0.0)
        return l2t::fail(c, L2T_EINVAL, "need 0 <= T_min < T_max");
    if (!(q.dt > 0.0) || !fin(q.dt)) return l2t::fail(c, L2T_EINVAL, "dt must be > 0");
    if (!(q.K >= 0.0) || !fin(q.K)) return l2t::fail(c, L2T_EINVAL, "K must be >= 0");
    if (!(q.g >= 0.0) || !fin(q.g)) return l2t::fail(c, L2T_EINVAL, "g must be >= 0");
    if (q.ce_model == L2T_CE_CONST) {
        if (!(q.ce_const > 0.0)) return l2t::fail(c, L2T_EINVAL, "ce_const must be > 0");
    } else if (q.ce_model == L2T_CE_LINEAR) {
        if (!(q.gamma > 0.0)) return l2t::fail(c, L2T_EINVAL, "gamma must be > 0");
    } else if (q.ce_model == L2T_CE_CAPPED) {
        if (!(q.gamma > 0.0) || !(q.ce_cap > 0.0))
            return l2t::fail(c, L2T_EINVAL, "gamma and ce_cap must be > 0");
    } else {
        return l2t::fail(c, L2T_EINVAL, "unknown ce_model");
    }
    if (q.laser_on) {
        if (!(q.laser_lp > 0.0) || !(q.laser_sigma > 0.0) || !(q.laser_fluence >= 0.0) ||
            !(q.v_atom > 0.0) || !fin(q.laser_t0) || !fin(q.laser_x0))
            return l2t::fail(c, L2T_EINVAL, "laser needs l_p, sigma, V_atom > 0 and F >= 0");
    }
    if (!(q.ke_eps >= 0.0)) return l2t::fail(c, L2T_EINVAL, "ke_eps must be >= 0");
    SystemState &st = c->sys[sys];
    st.params = q;
    st.has_params = true;
    int rc = l2t::upload_params(c);
    if (rc != L2T_OK) return rc;
    if (c->nbrs_built) {
        rc = l2t::source_weights(c, sys);
        if (rc != L2T_OK) return rc;
    }
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    // Gershgorin: the linearised exchange operator has eigenvalues in
    // [-2 K c max|N(i)|, 0] with c <= 1, so forward Euler is stable if
    // 2 K dt max|N(i)| <= 2.
    if (c->nbrs_built && q.K * q.dt * (double)st.max_nbrs > 1.0) {
        c->last_error = "Gershgorin bound 2 K dt max|N(i)| exceeds 2";
        return L2T_WUNSTABLE;
    }
    return L2T_OK;
}

int l2t_set_field(l2t_ctx *c, int32_t sys, int32_t field, const double *src, int32_t mem) {
    if (bad_sys(c, sys) || !src) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (field != L2T_FIELD_TE && field != L2T_FIELD_TL && field != L2T_FIELD_GATE &&
        field != L2T_FIELD_FIXED)
        return l2t::fail(c, L2T_EINVAL, "unknown or read-only field");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    SystemState &st = c->sys[sys];
    if (field == L2T_FIELD_TE && !st.has_params)
        return l2t::fail(c, L2T_ESTATE, "set parameters before T_e");
    const double *dsrc = nullptr;
    int rc = stage_in(c, src, st.desc.n_atoms, mem, c->stage, &dsrc);
    if (rc != L2T_OK) return rc;
    bool ok = true;
    if (field == L2T_FIELD_TE) {
        rc = l2t::check_field_range(c, dsrc, st.desc.n_atoms, st.params.T_min, st.params.T_max, &ok);
        if (rc != L2T_OK) return rc;
        if (!ok) return l2t::fail(c, L2T_ERANGE, "T_e outside [T_min, T_max] or non-finite");
    } else if (field == L2T_FIELD_TL) {
        rc = l2t::check_field_range(c, dsrc, st.desc.n_atoms, 0.0, HUGE_VAL, &ok);
        if (rc != L2T_OK) return rc;
        if (!ok) return l2t::fail(c, L2T_EINVAL, "T_lat must be finite and >= 0");
    }
    rc = l2t::permute_in(c, sys, dsrc, field);
    if (rc != L2T_OK) return rc;
    if (field == L2T_FIELD_TE) {
        rc = l2t::reset_ledger(c, sys);
        if (rc != L2T_OK) return rc;
        L2T_HIP(c, hipMemsetAsync(c->dstep + sys, 0, sizeof(int64_t), c->stream));
        st.step = 0;
        st.has_te = true;
        c->rec.valid = false;
    } else if (field == L2T_FIELD_TL) {
        st.has_tl = true;
    } else if (field == L2T_FIELD_FIXED) {
        // any nonzero entry marks the system as holding some atoms
        bool none = true;
        rc = l2t::check_field_range(c, dsrc, st.desc.n_atoms, 0.0, 0.0, &none);
        if (rc != L2T_OK) return rc;
        st.has_fixed = !none;
        c->rec.valid = false;
        rc = l2t::mark_held_slices(c, sys);
        if (rc != L2T_OK) return rc;
        rc = l2t::upload_params(c);
        if (rc != L2T_OK) return rc;
    }
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    return L2T_OK;
}

int l2t_get_field(l2t_ctx *c, int32_t sys, int32_t field, double *dst, int32_t mem) {
    if (bad_sys(c, sys) || !dst) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (field < L2T_FIELD_TE || field > L2T_FIELD_FIXED)
        return l2t::fail(c, L2T_EINVAL, "unknown field");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    const SystemState &st = c->sys[sys];
    if (field == L2T_FIELD_ELAT && !st.eatom_valid)
        return l2t::fail(c, L2T_ESTATE, "no advance of this system recorded with L2T_OPT_ATOM_LEDGER");
    double *d = mem == L2T_DEVICE ? dst : c->stage;
    int rc = l2t::permute_out(c, sys, field, d);
    if (rc != L2T_OK) return rc;
    if (mem == L2T_HOST) {
        L2T_HIP(c, hipMemcpyAsync(dst, c->stage, sizeof(double) * st.desc.n_atoms,
                                  hipMemcpyDeviceToHost, c->stream));
        L2T_HIP(c, hipStreamSynchronize(c->stream));
    }
    return L2T_OK;
}

int l2t_set_velocities(l2t_ctx *c, int32_t sys, const double *v, const double *mass, int32_t mem,
                       int32_t global_com) {
    if (bad_sys(c, sys) || !v || !mass) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    SystemState &st = c->sys[sys];
    if (!st.has_params) return l2t::fail(c, L2T_ESTATE, "set parameters before velocities");
    const int32_t n = st.desc.n_atoms;
    const double *dv = v, *dm = mass;
    if (mem == L2T_HOST) {
        L2T_HIP(c, hipMemcpyAsync(c->stage, v, sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                                  c->stream));
        L2T_HIP(c, hipMemcpyAsync(c->stage + 3 * (size_t)n, mass, sizeof(double) * n,
                                  hipMemcpyHostToDevice, c->stream));
        dv = c->stage;
        dm = c->stage + 3 * (size_t)n;
    }
    bool ok = true;
    int rc = l2t::check_field_range(c, dm, n, 1e-300, HUGE_VAL, &ok);
    if (rc != L2T_OK) return rc;
    if (!ok) return l2t::fail(c, L2T_EINVAL, "masses must be finite and > 0");
    rc = l2t::lattice_temperature(c, sys, dv, dm, global_com);
    if (rc != L2T_OK) return rc;
    st.has_tl = true;
    return L2T_OK;
}

int l2t_set_velocities_noalloc(l2t_ctx *c, int32_t sys, const double *v, const double *mass,
                               int32_t global_com) {
    if (bad_sys(c, sys) || !v || !mass) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    SystemState &st = c->sys[sys];
    if (4 * (size_t)st.n_pad + 4 > l2t::kStaticScratchBytes / sizeof(double))
        return l2t::fail(c, L2T_EINVAL, "system larger than the static staging array");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    if (!st.has_params) return l2t::fail(c, L2T_ESTATE, "set parameters before velocities");
    for (const void *p : {(const void *)v, (const void *)mass}) {
        hipPointerAttribute_t a{};
        hipError_t e = hipPointerGetAttributes(&a, p);
        if (e != hipSuccess) (void)hipGetLastError();
        if (e != hipSuccess || a.device != c->device ||
            (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged))
            return l2t::fail(c, L2T_EINVAL, "v and mass must be device memory of the context's GPU");
    }
    bool ok = true;
    int rc = l2t::check_field_range(c, mass, st.desc.n_atoms, 1e-300, HUGE_VAL, &ok);
    if (rc != L2T_OK) return rc;
    if (!ok) return l2t::fail(c, L2T_EINVAL, "masses must be finite and > 0");
    rc = l2t::lattice_temperature_static(c, sys, v, mass, global_com);
    if (rc != L2T_OK) return rc;
    st.has_tl = true;
    return L2T_OK;
}

int l2t_set_allocator(l2t_ctx *c, void *(*alloc)(size_t, void *), void (*free_)(void *, void *),
                      void *user) {
    if (!c) return L2T_EINVAL;
    if ((alloc == nullptr) != (free_ == nullptr))
        return l2t::fail(c, L2T_EINVAL, "give both alloc and free_, or neither");
    c->ualloc = alloc;
    c->ufree = free_;
    c->uarg = alloc ? user : nullptr;
    return L2T_OK;
}

int l2t_set_option(l2t_ctx *c, int32_t option, int64_t value) {
    if (!c) return L2T_EINVAL;
    l2t::Tuning &t = c->tune;
    switch (option) {
        case L2T_OPT_PERSISTENT:
            t.persistent = value ? 1 : 0;
            if (value) t.kernel = l2t::kKernelSliced;
            break;
        case L2T_OPT_BLOCK:
            if (value != 0 && (value < 64 || value > l2t::kBrickBlockMax || value % 64))
                return l2t::fail(c, L2T_EINVAL, "block must be 0 or a multiple of 64 up to 512");
            if (value == 0) {
                t.block = l2t::kBrickBlockMax;
                t.tuned = false;
                l2t::drop_graphs(c);
                return L2T_OK;
            }
            t.block = (int)value;
            break;
        case L2T_OPT_RESIDENT_MAX: t.resident_max = (int)value; break;
        case L2T_OPT_GRAPH:
            // how launches are issued, not a launch shape: leaves the tuned
            // shape alone; an explicit choice applies at once, 2 has the
            // autotuner time it at the next advance (if it is on and not pinned)
            if (value < 0 || value > 2) return l2t::fail(c, L2T_EINVAL, "graph must be 0, 1 or 2");
            t.graph = (int)value;
            if (value != 2) {
                t.graph_used = (int)value;
            } else if (t.autotune && !t.pinned) {
                t.tuned = false;
            } else {
                t.graph_used = 1;
            }
            l2t::drop_graphs(c);
            return L2T_OK;
        case L2T_OPT_BRICK_EDGE:
            if (value < 0 || value > l2t::kMaxBrickEdge)
                return l2t::fail(c, L2T_EINVAL, "brick edge must be 0..1024");
            t.brick_edge = (int)value;
            return L2T_OK;
        case L2T_OPT_ATOM_LEDGER:
            // not a tuning choice: leaves the tuned launch shape alone
            if ((value != 0) != c->atom_ledger) l2t::drop_graphs(c);
            c->atom_ledger = value != 0;
            return L2T_OK;
        case L2T_OPT_BATCH_FP64:
            c->batch_fp64 = value != 0;
            return L2T_OK;
        case L2T_OPT_SWEEP:
            // the order of the bricks in a launch, not a launch shape: leaves the
            // tuned form alone; an explicit order applies at once
            if (value < 0 || value > 2) return l2t::fail(c, L2T_EINVAL, "sweep must be 0, 1 or 2");
            t.sweep = (int)value;
            if (value != 0) t.sweep_used = (int)value;
            l2t::drop_graphs(c);
            return L2T_OK;
        case L2T_OPT_TABLE_STREAM:
            // a cache hint of the table loads, not a launch shape: leaves the
            // tuned form alone; an explicit choice applies at once
            if (value < 0 || value > 2)
                return l2t::fail(c, L2T_EINVAL, "table stream must be 0, 1 or 2");
            t.table = (int)value;
            if (value != 0) t.table_used = (int)value;
            l2t::drop_graphs(c);
            return L2T_OK;
        case L2T_OPT_KERNEL:
            if (value != l2t::kKernelSliced && value != l2t::kKernelBrick)
                return l2t::fail(c, L2T_EINVAL, "kernel must be 0 (global) or 1 (brick)");
            t.kernel = (int)value;
            break;
        case L2T_OPT_AUTOTUNE:
            t.autotune = value ? 1 : 0;
            if (value) t.tuned = false;
            break;
        default: return l2t::fail(c, L2T_EINVAL, "unknown option");
    }
    if (option != L2T_OPT_AUTOTUNE) {
        t.tuned = true;    // an explicit choice overrides tuning, also across rebuilds
        t.pinned = true;
    } else {
        t.pinned = false;
    }
    l2t::drop_graphs(c);
    return L2T_OK;
}

int l2t_get_option(l2t_ctx *c, int32_t option, int64_t *value) {
    if (!c || !value) return L2T_EINVAL;
    const l2t::Tuning &t = c->tune;
    switch (option) {
        case L2T_OPT_PERSISTENT: *value = t.persistent; break;
        case L2T_OPT_BLOCK: *value = t.block; break;
        case L2T_OPT_RESIDENT_MAX: *value = t.resident_max; break;
        case L2T_OPT_GRAPH: *value = t.graph_used; break;
        case L2T_OPT_AUTOTUNE: *value = t.autotune; break;
        case L2T_OPT_KERNEL: *value = t.kernel; break;
        case L2T_OPT_ATOM_LEDGER: *value = c->atom_ledger ? 1 : 0; break;
        case L2T_OPT_BATCH_FP64: *value = c->batch_fp64 ? 1 : 0; break;
        case L2T_OPT_BRICK_EDGE: *value = c->brick_edge_used; break;
        case L2T_OPT_SWEEP: *value = t.sweep_used; break;
        case L2T_OPT_TABLE_STREAM: *value = t.table_used; break;
        default: return l2t::fail(c, L2T_EINVAL, "unknown option");
    }
    return L2T_OK;
}

int l2t_advance(l2t_ctx *c, int32_t n) {
    if (!c || n < 0) return l2t::fail(c, L2T_EINVAL, "n_substeps must be >= 0");
    std::string why;
    if (!ready_to_advance(c, 0, (int32_t)c->sys.size(), &why)) return l2t::fail(c, L2T_ESTATE, why);
    c->rec.valid = false;
    if (n == 0) return L2T_OK;
    int rc0 = begin_atom_ledger(c, 0, (int32_t)c->sys.size());
    if (rc0 != L2T_OK) return rc0;
    if (c->precision == L2T_FP64) {
        if (c->batch_fp64) return l2t::advance_plain(c, -1, n);
        for (int32_t s = 0; s < (int32_t)c->sys.size(); ++s) {
            int rc = l2t::advance_plain(c, s, n);
            if (rc != L2T_OK) return rc;
        }
        return L2T_OK;
    }
    if (c->tune.autotune && !c->tune.tuned) {
        int rc = l2t::autotune(c);
        if (rc != L2T_OK) return rc;
    }
    return l2t::advance_fp32c(c, n);
}

int l2t_advance_system(l2t_ctx *c, int32_t sys, int32_t n) {
    if (bad_sys(c, sys) || n < 0) return l2t::fail(c, L2T_EINVAL, "bad system index or n < 0");
    std::string why;
    if (!ready_to_advance(c, sys, sys + 1, &why)) return l2t::fail(c, L2T_ESTATE, why);
    c->rec.valid = false;
    if (n == 0) return L2T_OK;
    int rc = begin_atom_ledger(c, sys, sys + 1);
    if (rc != L2T_OK) return rc;
    return l2t::advance_plain(c, sys, n);
}

int l2t_advance_recorded(l2t_ctx *c, int32_t n, int32_t ckpt_every) {
    if (!c || n < 1 || ckpt_every < 1) return l2t::fail(c, L2T_EINVAL, "need n >= 1, ckpt >= 1");
    if (c->precision != L2T_FP32C)
        return l2t::fail(c, L2T_ENOTIMPL, "the adjoint is provided for the FP32C path");
    for (const auto &st : c->sys)
        if (st.has_fixed || st.mf.on)
            return l2t::fail(c, L2T_ENOTIMPL,
                             "the adjoint is not provided for fixed atoms or the mean-field mode");
    std::string why;
    if (!ready_to_advance(c, 0, (int32_t)c->sys.size(), &why)) return l2t::fail(c, L2T_ESTATE, why);
    l2t::Recording &r = c->rec;
    r.valid = false;
    r.n_steps = n;
    r.ckpt = ckpt_every;
    r.n_ckpt = (n + ckpt_every - 1) / ckpt_every;
    size_t need = (size_t)r.n_ckpt * 2 * sizeof(float) * (size_t)c->n_int;
    if (need > r.bytes) {
        l2t::dev_free(c, r.buf);
        r.buf = nullptr;
        r.bytes = 0;
        if (l2t::dev_malloc(c, &r.buf, need) != hipSuccess)
            return l2t::fail(c, L2T_ENOMEM, "checkpoint allocation failed");
        r.bytes = need;
    }
    r.step0.resize(c->sys.size());
    for (size_t s = 0; s < c->sys.size(); ++s) r.step0[s] = c->sys[s].step;
    // the segments between checkpoints run in the tuned launch form (all forms
    // give the same states bit for bit), which the adjoint's recomputation follows
    if (c->tune.autotune && !c->tune.tuned) {
        int rc = l2t::autotune(c);
        if (rc != L2T_OK) return rc;
    }
    int rc0 = begin_atom_ledger(c, 0, (int32_t)c->sys.size());
    if (rc0 != L2T_OK) return rc0;
    for (int64_t k = 0; k < r.n_ckpt; ++k) {
        int rc = l2t::record_checkpoint(c, k);
        if (rc != L2T_OK) return rc;
        int32_t len = (int32_t)std::min<int64_t>(ckpt_every, n - k * ckpt_every);
        rc = l2t::advance_fp32c(c, len);
        if (rc != L2T_OK) return rc;
    }
    r.valid = true;
    return L2T_OK;
}

int l2t_adjoint(l2t_ctx *c, const double *dL_dTN, int32_t mem, double *dL_dK, double *dL_dg,
                double *dL_dT0) {
    if (!c || !dL_dTN || !dL_dK || !dL_dg) return l2t::fail(c, L2T_EINVAL, "NULL argument");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    if (!c->rec.valid) return l2t::fail(c, L2T_ESTATE, "no recorded advance");
    const double *dw = nullptr;
    int rc = stage_in(c, dL_dTN, (size_t)c->n_tot, mem, c->stage, &dw);
    if (rc != L2T_OK) return rc;
    // dL/dT^0 goes straight to a device destination, else through the
    // staging buffer (free again once the adjoint has read dL/dT^N)
    double *d0 = dL_dT0 ? (mem == L2T_DEVICE ? dL_dT0 : c->stage) : nullptr;
    rc = l2t::adjoint(c, dw, dL_dK, dL_dg, d0);
    if (rc != L2T_OK) return rc;
    if (dL_dT0 && mem == L2T_HOST) {
        L2T_HIP(c, hipMemcpyAsync(dL_dT0, d0, sizeof(double) * (size_t)c->n_tot,
                                  hipMemcpyDeviceToHost, c->stream));
        L2T_HIP(c, hipStreamSynchronize(c->stream));
    }
    return check_err(c);
}

int l2t_set_mean_field(l2t_ctx *c, int32_t sys, const l2t_mean_field *mf) {
    if (bad_sys(c, sys) || !mf) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    SystemState &st = c->sys[sys];
    if (!st.has_params) return l2t::fail(c, L2T_ESTATE, "set parameters before the mean-field mode");
    if (mf->on && (!(mf->lambda > 0.0) || !std::isfinite(mf->lambda) || !(mf->k_coef > 0.0) ||
                   !std::isfinite(mf->k_coef)))
        return l2t::fail(c, L2T_EINVAL, "lambda and k_coef must be finite and > 0");
    st.mf = *mf;
    st.mf.on = mf->on ? 1 : 0;
    c->rec.valid = false;
    l2t::drop_graphs(c);
    int rc = l2t::upload_params(c);
    if (rc != L2T_OK) return rc;
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    return L2T_OK;
}

int l2t_set_lattice_fd(l2t_ctx *c, int32_t sys, const l2t_lattice_fd *lf) {
    if (bad_sys(c, sys) || !lf) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (c->precision != L2T_FP64)
        return l2t::fail(c, L2T_ENOTIMPL, "the two-temperature lattice runs in FP64 contexts");
    SystemState &st = c->sys[sys];
    if (!st.has_params) return l2t::fail(c, L2T_ESTATE, "set parameters before the lattice mode");
    if (lf->on && (!(lf->K_lat >= 0.0) || !std::isfinite(lf->K_lat) || !(lf->c_lat > 0.0) ||
                   !std::isfinite(lf->c_lat)))
        return l2t::fail(c, L2T_EINVAL, "need K_lat >= 0 and c_lat > 0");
    st.lf = *lf;
    st.lf.on = lf->on ? 1 : 0;
    int rc = l2t::upload_params(c);
    if (rc != L2T_OK) return rc;
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    return L2T_OK;
}

int l2t_get_params(l2t_ctx *c, int32_t sys, l2t_params *out) {
    if (bad_sys(c, sys) || !out) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    const SystemState &st = c->sys[sys];
    if (!st.has_params) return l2t::fail(c, L2T_ESTATE, "parameters not set");
    l2t::DevParams p{};
    L2T_HIP(c, hipMemcpyAsync(&p, c->dparams + sys, sizeof(p), hipMemcpyDeviceToHost, c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));
    *out = st.params;
    out->K = p.K;
    out->ce_model = p.ce_model;
    out->ce_const = p.ce_const;
    return L2T_OK;
}

int l2t_coupling(l2t_ctx *c, int32_t sys, int32_t mode, double dt_md, const double *v,
                 const double *mass, double *xi, int32_t mem) {
    if (bad_sys(c, sys) || !v || !mass || !xi)
        return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    if (mode != L2T_XI_INSTANT && mode != L2T_XI_LEDGER)
        return l2t::fail(c, L2T_EINVAL, "mode must be L2T_XI_INSTANT or L2T_XI_LEDGER");
    if (mode == L2T_XI_LEDGER && !(dt_md > 0.0 && std::isfinite(dt_md)))
        return l2t::fail(c, L2T_EINVAL, "dt_md must be > 0");
    if (!c->nbrs_built) return l2t::fail(c, L2T_ESTATE, "neighbour sets not built");
    const SystemState &st = c->sys[sys];
    if (!st.has_te || !st.has_tl || !st.has_params)
        return l2t::fail(c, L2T_ESTATE, "T_e, T_lat and parameters must be set");
    if (mode == L2T_XI_LEDGER && !st.eatom_valid)
        return l2t::fail(c, L2T_ESTATE, "no advance of this system recorded with L2T_OPT_ATOM_LEDGER");
    const int64_t n = st.desc.n_atoms;
    const double *dv = v, *dm = mass;
    double *dxi = xi;
    if (mem == L2T_HOST) {
        if (l2t::ensure_scratch(c, sizeof(double) * 5 * (size_t)n) != L2T_OK)
            return l2t::fail(c, L2T_ENOMEM, "staging allocation failed");
        double *sc = (double *)c->scratch;
        L2T_HIP(c, hipMemcpyAsync(sc, v, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
        L2T_HIP(c, hipMemcpyAsync(sc + 3 * n, mass, sizeof(double) * n, hipMemcpyHostToDevice,
                                  c->stream));
        dv = sc;
        dm = sc + 3 * n;
        dxi = sc + 4 * n;
    }
    int rc = l2t::coupling(c, sys, mode, dt_md, dv, dm, dxi);
    if (rc != L2T_OK) return rc;
    if (mem == L2T_HOST) {
        L2T_HIP(c, hipMemcpyAsync(xi, dxi, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
        return check_err(c);   // synchronises; reports a bad mass now
    }
    return L2T_OK;
}

int l2t_damping_step(l2t_ctx *c, int32_t sys, double dt_md, const double *xi,
                     const double *force, const double *mass, double *v, int32_t mem) {
    if (bad_sys(c, sys) || !xi || !mass || !v)
        return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (mem != L2T_HOST && mem != L2T_DEVICE) return l2t::fail(c, L2T_EINVAL, "bad mem");
    if (!(dt_md > 0.0 && std::isfinite(dt_md))) return l2t::fail(c, L2T_EINVAL, "dt_md must be > 0");
    const int64_t n = c->sys[sys].desc.n_atoms;
    const double *dxi = xi, *dF = force, *dm = mass;
    double *dv = v;
    if (mem == L2T_HOST) {
        if (l2t::ensure_scratch(c, sizeof(double) * 8 * (size_t)n) != L2T_OK)
            return l2t::fail(c, L2T_ENOMEM, "staging allocation failed");
        double *sc = (double *)c->scratch;
        L2T_HIP(c, hipMemcpyAsync(sc, v, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
        L2T_HIP(c, hipMemcpyAsync(sc + 3 * n, mass, sizeof(double) * n, hipMemcpyHostToDevice,
                                  c->stream));
        L2T_HIP(c, hipMemcpyAsync(sc + 4 * n, xi, sizeof(double) * n, hipMemcpyHostToDevice,
                                  c->stream));
        if (force)
            L2T_HIP(c, hipMemcpyAsync(sc + 5 * n, force, sizeof(double) * 3 * n,
                                      hipMemcpyHostToDevice, c->stream));
        dv = sc;
        dm = sc + 3 * n;
        dxi = sc + 4 * n;
        dF = force ? sc + 5 * n : nullptr;
    }
    int rc = l2t::damping_step(c->stream, n, dt_md, dxi, dF, dm, dv, c->derr);
    if (rc != L2T_OK) return l2t::fail(c, rc, "damping step launch failed");
    if (mem == L2T_HOST) {
        L2T_HIP(c, hipMemcpyAsync(v, dv, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
        return check_err(c);   // synchronises; reports a bad mass now
    }
    return L2T_OK;
}

int l2t_energies(l2t_ctx *c, int32_t sys, l2t_energy_report *out) {
    if (bad_sys(c, sys) || !out) return l2t::fail(c, L2T_EINVAL, "bad system index or NULL");
    if (!c->nbrs_built || !c->sys[sys].has_params || !c->sys[sys].has_te)
        return l2t::fail(c, L2T_ESTATE, "neighbours, parameters and T_e must be set");
    int rc = l2t::energies(c, sys, out);
    if (rc != L2T_OK) return rc;
    out->t = (double)c->sys[sys].step * c->sys[sys].params.dt;
    return check_err(c);
}

// a system's ledger totals into its first ledger row (the report sums its
// rows, the others are cleared) and its step counter
static int restore_counters(l2t_ctx *c, int32_t sys, int64_t step, double E_e_to_l, double E_src,
                            double T_ledger_acc) {
    SystemState &st = c->sys[sys];
    int rc = l2t::reset_ledger(c, sys);
    if (rc != L2T_OK) return rc;
    const double row[3] = {E_e_to_l, E_src, T_ledger_acc};
    L2T_HIP(c, hipMemcpyAsync(c->ledger + 3 * (int64_t)st.slice0, row, sizeof row,
                              hipMemcpyHostToDevice, c->stream));
    L2T_HIP(c, hipMemcpyAsync(c->dstep + sys, &step, sizeof step, hipMemcpyHostToDevice,
                              c->stream));
    L2T_HIP(c, hipStreamSynchronize(c->stream));   // the sources are locals
    st.step = step;
    return L2T_OK;
}

int l2t_set_counters(l2t_ctx *c, int32_t sys, int64_t step, double E_e_to_l, double E_src,
                     double T_ledger_acc) {
    if (bad_sys(c, sys) || step < 0 || !std::isfinite(E_e_to_l) || !std::isfinite(E_src) ||
        !std::isfinite(T_ledger_acc))
        return l2t::fail(c, L2T_EINVAL, "bad system index, step < 0 or non-finite ledger value");
    SystemState &st = c->sys[sys];
    if (!c->nbrs_built || !st.has_te)
        return l2t::fail(c, L2T_ESTATE, "restore T_e before the counters (writing T_e resets them)");
    const int rc = restore_counters(c, sys, step, E_e_to_l, E_src, T_ledger_acc);
    if (rc != L2T_OK) return rc;
    c->rec.valid = false;
    return L2T_OK;
}

int l2t_sync(l2t_ctx *c) {
    if (!c) return L2T_EINVAL;
    return check_err(c);
}

int l2t_pair_fp32(const float *ti, const float *tj, float *out, int64_t n, void *hip_stream) {
    if (n < 0 || (n > 0 && (!ti || !tj || !out))) return L2T_EINVAL;
    return l2t::pair_fp32(ti, tj, out, n, (hipStream_t)hip_stream);
}

}  // extern "C"
