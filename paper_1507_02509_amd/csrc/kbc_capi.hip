// kbc_capi.hip -- the C ABI declared in include/kbc.h.
//
// A context borrows the caller's two population buffers and records the
// lattice parameters, the step counter and the buffer that holds the current
// state.  Its only allocations are the scratch arrays of lbm_diagnostics.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "kbc.h"
#include "kbc_launch.hpp"

struct lbm_ctx {
    lbm_params p;
    kbc::Lattice L;
    void* buf[2];
    int cur;                // index of the buffer holding the current state
    int64_t steps;
    kbc::StepShape shape;
    int fuse;               // time steps per launch of lbm_step: 1 or 2
    int fuse_rows;          // output tile height of the fused launch: 8, 16, 24 or 32
    double* dscratch;       // ux, uy, omega fields + diagnostics partials
    size_t dscratch_elems;
    double* ascratch;       // adjoint: block partials + initial-state stencil fields
    size_t ascratch_elems;
    double* sscratch;       // spectra: velocity fields and their transforms
    size_t sscratch_elems;
    void* fft_plan;         // spectra: cached FFT plan
    int graph_chunk;        // lbm_step: steps per graph replay (0: every launch eager)
    hipStream_t cap_stream; // private stream the graphs are captured on
    hipGraphExec_t gexec[2];  // captured graph_chunk steps, by the buffer holding the start state
    int gnext[2];           // buffer holding the state after one replay
    int ens_refs;           // live ensembles holding this context (lbm_free refuses while > 0)
    uint64_t gen;           // parameter generation: bumped when beta changes, so that an
                            // ensemble holding the context rebuilds its member table
    int device;             // HIP device current at lbm_init
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

int launch_result(int rc, const char* what) {
    if (rc == 0) return LBM_OK;
    if (rc == -1) return fail(LBM_EINVAL, "%s: invalid configuration", what);
    if (rc == -5) return fail(LBM_EUNSUPPORTED, "%s: combination not built", what);
    if (rc == kbc::kTooLarge)
        return fail(LBM_EUNSUPPORTED, "%s: lattice too large for one launch (2^32 - 1 work-items)", what);
    return fail(LBM_EHIP, "%s: kernel launch failed: %s", what, hipGetErrorString(hipGetLastError()));
}

size_t form_bytes(int32_t form) {
    switch (form) {
        case LBM_F16DEV_F32: return 2;
        case LBM_F32DEV_F32: return 4;
        case LBM_F64: return 8;
        default: return 0;
    }
}

int check_params(const lbm_params* p) {
    if (!p) return fail(LBM_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(LBM_EINVAL, "nx, ny must be >= 3 (got %d x %d)", p->nx, p->ny);
    if (p->nx > kbc::kMaxSide || p->ny > kbc::kMaxSide)
        return fail(LBM_EINVAL, "nx, ny must be <= 2^28 (got %d x %d)", p->nx, p->ny);
    if (!(p->beta > 0.0 && p->beta <= 1.0)) return fail(LBM_EINVAL, "beta must be in (0, 1] (got %g)", p->beta);
    if (!(p->rho0 > 0.0) || !isfinite(p->rho0)) return fail(LBM_EINVAL, "rho0 must be > 0");
    if (p->collision != LBM_LBGK && p->collision != LBM_KBC) return fail(LBM_EINVAL, "unknown collision %d", p->collision);
    if (p->variant < LBM_KBC_A || p->variant > LBM_KBC_D) return fail(LBM_EINVAL, "unknown variant %d", p->variant);
    if (form_bytes(p->form) == 0) return fail(LBM_EINVAL, "unknown form %d", p->form);
    if (p->gamma_mode < LBM_GAMMA_ESTIMATE || p->gamma_mode > LBM_GAMMA_EXACT)
        return fail(LBM_EINVAL, "unknown gamma_mode %d", p->gamma_mode);
    if (!(p->gamma_guard >= 0.0) || !isfinite(p->gamma_guard)) return fail(LBM_EINVAL, "gamma_guard must be finite and >= 0");
    if (p->gamma_mode == LBM_GAMMA_FIXED && !isfinite(p->gamma_fixed)) return fail(LBM_EINVAL, "gamma_fixed must be finite");
    return LBM_OK;
}

// Whether the state should be written with plain rather than non-temporal
// stores, given the bytes of all state buffers a step reads and writes:
// plain where they outgrow the L2s but fit the 256 MiB last-level cache,
// which then still holds the new state when the next step reads it.
// Measured on MI355X (KBC-B, default tiles, fused steps): FP32 1024^2 8.97
// against 11.14 us per step, 1792^2 23.2 against 27.3; FP64 1024^2 15.8
// against 18.1; below the lower bound (FP32 640^2, FP64 512^2) and above
// 256 MiB (FP32 2048^2, FP64 1536^2) non-temporal stores were 1-10 % faster.
// FP16, bound by vector issue, gains least and only from 80 MB on.
bool plain_stores_pay(int32_t form, double state_bytes) {
    const double lo = (form == LBM_F16DEV_F32) ? 80e6 : 40e6;
    return state_bytes >= lo && state_bytes <= 256.0 * 1024.0 * 1024.0;
}

// Default step tile per storage form, from a sweep on MI355X at 16384^2
// (the autotuner in the Python package can replace it per lattice).
kbc::StepShape default_shape(int32_t form) {
    kbc::StepShape s;
    switch (form) {
        case LBM_F16DEV_F32: s.width = 256; s.rpt = 4; s.nt = 1; break;
        case LBM_F64: s.width = 128; s.rpt = 1; s.nt = 1; break;
        default: s.width = 256; s.rpt = 1; s.nt = 1; break;
    }
    return s;
}

kbc::Lattice lattice_of(const lbm_params& p, size_t pitch) {
    kbc::Lattice L;
    L.nx = p.nx;
    L.ny = p.ny;
    L.pitch = static_cast<int64_t>(pitch);
    L.form = p.form;
    L.collision = p.collision;
    L.variant = p.variant;
    L.gamma_mode = p.gamma_mode;
    L.beta = p.beta;
    L.rho0 = p.rho0;
    L.guard = p.gamma_guard;
    L.gamma_fixed = p.gamma_fixed;
    L.stream = static_cast<hipStream_t>(p.stream);
    L.adj_frozen = 0;
    return L;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_err; }

size_t lbm_required_pitch(int32_t nx, int32_t form) {
    if (nx < 1 || nx > kbc::kMaxSide || form_bytes(form) == 0) return 0;
    return (static_cast<size_t>(nx) + 63) / 64 * 64;
}

size_t lbm_buffer_bytes(int32_t nx, int32_t ny, int32_t form) {
    const size_t pitch = lbm_required_pitch(nx, form);
    if (pitch == 0 || ny < 1) return 0;
    return 9 * static_cast<size_t>(ny) * pitch * form_bytes(form);
}

int lbm_init(lbm_ctx** out, const lbm_params* p, void* buf_a, void* buf_b, size_t pitch_elems,
             const double* rho, const double* ux, const double* uy, const double* grad, int32_t mode) {
    g_err[0] = 0;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    if (!buf_a || !buf_b) return fail(LBM_EINVAL, "population buffers must not be NULL");
    const size_t need = lbm_required_pitch(p->nx, p->form);
    if (pitch_elems < need || pitch_elems % 64 != 0)
        return fail(LBM_EINVAL, "pitch %zu must be >= %zu and a multiple of 64", pitch_elems, need);
    const size_t bytes = 9 * static_cast<size_t>(p->ny) * pitch_elems * form_bytes(p->form);
    const char* a = static_cast<const char*>(buf_a);
    const char* b = static_cast<const char*>(buf_b);
    if (a < b + bytes && b < a + bytes) return fail(LBM_EINVAL, "population buffers overlap");
    if (mode < LBM_INIT_EQ || mode > LBM_INIT_GRAD_GIVEN) return fail(LBM_EINVAL, "unknown init mode %d", mode);
    if (!ux || !uy) return fail(LBM_EINVAL, "ux and uy must not be NULL");
    if (mode == LBM_INIT_GRAD_GIVEN && !grad) return fail(LBM_EINVAL, "LBM_INIT_GRAD_GIVEN needs grad");

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "context allocation failed");
    c->p = *p;
    c->L = lattice_of(*p, pitch_elems);
    c->buf[0] = buf_a;
    c->buf[1] = buf_b;
    c->cur = 0;
    c->steps = 0;
    c->shape = default_shape(p->form);
    if (plain_stores_pay(p->form, 2.0 * static_cast<double>(bytes))) c->shape.nt = 0;
    // two fused steps per launch by default for every form (measured for
    // KBC-B at 16384^2: FP32 +38 %, FP64 +25 %, FP16 +6 % over single steps;
    // the ring of extra step-1 collisions costs less than the HBM pass it saves)
    c->fuse = 2;
    c->fuse_rows = (p->form == LBM_F64) ? 8 : 16;
    // smaller lattices: 8-row tiles double the workgroup count, which pays
    // below about 1792 tiles of 16 rows (FP32, us per step with 8 / 16 rows:
    // 512^2 3.7 / 4.2, 1152^2 11.5 / 12.1, 1280^2 13.5 / 14.1, 1408^2 a tie;
    // FP16 alike)
    if (static_cast<int64_t>((p->nx + 63) / 64) * ((p->ny + 15) / 16) < 1792) c->fuse_rows = 8;
    c->dscratch = nullptr;
    c->dscratch_elems = 0;
    c->ascratch = nullptr;
    c->ascratch_elems = 0;
    c->sscratch = nullptr;
    c->sscratch_elems = 0;
    c->fft_plan = nullptr;
    c->graph_chunk = 0;
    c->cap_stream = nullptr;
    c->gexec[0] = c->gexec[1] = nullptr;
    c->gnext[0] = 0;
    c->gnext[1] = 1;
    c->ens_refs = 0;
    c->gen = 0;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = -1;
    rc = kbc::launch_init(c->L, buf_a, rho, ux, uy, grad, mode);
    if (rc) {
        delete c;
        return launch_result(rc, "lbm_init");
    }
    *out = c;
    return LBM_OK;
}

}  // extern "C"

namespace {

// The launches of nsteps steps on c->L.stream, with the context's buffer
// index and step counter advanced as they are enqueued.
int step_eager(lbm_ctx* c, int32_t nsteps) {
    int32_t s = 0;
    if (c->fuse == 2) {
        for (; s + 2 <= nsteps; s += 2) {
            const int rc = kbc::launch_step2(c->L, c->buf[c->cur], c->buf[c->cur ^ 1], c->fuse_rows, c->shape.nt);
            if (rc) return launch_result(rc, "lbm_step (two fused steps)");
            c->cur ^= 1;
            c->steps += 2;
        }
    }
    for (; s < nsteps; ++s) {
        const int rc = kbc::launch_step(c->L, c->buf[c->cur], c->buf[c->cur ^ 1], c->shape);
        if (rc) return launch_result(rc, "lbm_step");
        c->cur ^= 1;
        ++c->steps;
    }
    return LBM_OK;
}

// Discard the captured graphs (after a change to what the launches do).
int graph_reset(lbm_ctx* c) {
    if (!c->gexec[0] && !c->gexec[1]) return LBM_OK;
    int rc = LBM_OK;
    hipError_t e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) rc = hip_fail(e, "graph reset sync");
    for (int k = 0; k < 2; ++k) {
        if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        c->gexec[k] = nullptr;
    }
    return rc;
}

// One replay of graph_chunk steps, capturing the graph first if this start
// buffer has none: the eager launches are recorded on the private stream
// (nothing runs), the context's bookkeeping is rolled back, and the graph is
// then launched on the context's stream.
int step_graph(lbm_ctx* c) {
    const int k = c->cur;
    if (!c->gexec[k]) {
        hipError_t e;
        if (!c->cap_stream) {
            e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                c->cap_stream = nullptr;
                return hip_fail(e, "graph capture stream");
            }
        }
        const hipStream_t user = c->L.stream;
        const int64_t steps0 = c->steps;
        e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture begin");
        c->L.stream = c->cap_stream;
        const int rc = step_eager(c, c->graph_chunk);
        c->L.stream = user;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &g);
        c->gnext[k] = c->cur;
        c->cur = k;
        c->steps = steps0;
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        e = hipGraphInstantiate(&c->gexec[k], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            c->gexec[k] = nullptr;
            return hip_fail(e, "graph instantiate");
        }
    }
    const hipError_t e = hipGraphLaunch(c->gexec[k], c->L.stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    c->cur = c->gnext[k];
    c->steps += c->graph_chunk;
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_step(lbm_ctx* c, int32_t nsteps) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (c->L.halo_lo) {
        // a slab: the halo buffers hold the neighbours' rows at the current
        // time, enough for one launch
        if (nsteps > c->fuse)
            return fail(LBM_EINVAL, "a slab steps at most %d step(s) per call (its halo holds the rows for one launch)",
                        c->fuse);
        return step_eager(c, nsteps);
    }
    if (c->graph_chunk >= 2) {
        for (; nsteps >= c->graph_chunk; nsteps -= c->graph_chunk) {
            const int rc = step_graph(c);
            if (rc) return rc;
        }
    }
    return step_eager(c, nsteps);
}

int lbm_set_graph(lbm_ctx* c, int32_t chunk) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (chunk != 0 && c->L.halo_lo) return fail(LBM_EINVAL, "a slab (halo buffers set) does not replay graphs");
    if (chunk != 0 && (chunk < 2 || chunk > (1 << 20)))
        return fail(LBM_EINVAL, "graph chunk must be 0 or in [2, 2^20] (got %d)", chunk);
    if (chunk == c->graph_chunk) return LBM_OK;
    const int rc = graph_reset(c);
    c->graph_chunk = chunk;
    return rc;
}

int lbm_get_graph(const lbm_ctx* c) { return c ? c->graph_chunk : -1; }

int lbm_set_fusion(lbm_ctx* c, int32_t steps_per_launch, int32_t rows) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (steps_per_launch != 1 && steps_per_launch != 2)
        return fail(LBM_EINVAL, "steps_per_launch must be 1 or 2 (got %d)", steps_per_launch);
    if (rows != 0 && rows != 8 && rows != 16 && rows != 24 && rows != 32)
        return fail(LBM_EINVAL, "rows must be 0 (keep), 8, 16, 24 or 32 (got %d)", rows);
    if (rows == 32 && c->p.form == LBM_F64)
        return fail(LBM_EUNSUPPORTED, "a 32-row fused FP64 tile does not fit the LDS of a CU");
    if (c->L.halo_lo && (rows ? rows : c->fuse_rows) != 8 && (rows ? rows : c->fuse_rows) != 16)
        return fail(LBM_EUNSUPPORTED, "a slab (halo buffers set) runs fused tiles of 8 or 16 rows");
    const int rc = graph_reset(c);
    if (rc) return rc;
    c->fuse = steps_per_launch;
    if (rows) c->fuse_rows = rows;
    return LBM_OK;
}

int lbm_get_fusion(const lbm_ctx* c, int32_t* rows) {
    if (!c) return -1;
    if (rows) *rows = c->fuse_rows;
    return c->fuse;
}

int lbm_moments(lbm_ctx* c, double* rho, double* ux, double* uy, double* gamma) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!rho && !ux && !uy && !gamma) return LBM_OK;
    return launch_result(kbc::launch_moments(c->L, c->buf[c->cur], rho, ux, uy, gamma), "lbm_moments");
}

int lbm_get_populations(lbm_ctx* c, double* f) {
    if (!c || !f) return fail(LBM_EINVAL, "ctx and f must not be NULL");
    return launch_result(kbc::launch_get_pop(c->L, c->buf[c->cur], f), "lbm_get_populations");
}

int lbm_set_populations(lbm_ctx* c, const double* f) {
    if (!c || !f) return fail(LBM_EINVAL, "ctx and f must not be NULL");
    return launch_result(kbc::launch_set_pop(c->L, c->buf[c->cur], f), "lbm_set_populations");
}

int lbm_diagnostics(lbm_ctx* c, lbm_diag* out) {
    if (!c || !out) return fail(LBM_EINVAL, "ctx and out must not be NULL");
    const size_t N = static_cast<size_t>(c->p.nx) * c->p.ny;
    const size_t need = 3 * N + static_cast<size_t>(kbc::kDiagBlocks) * kbc::kDiagSlots;
    if (c->dscratch_elems < need) {
        if (c->dscratch) {
            hipError_t e = hipStreamSynchronize(c->L.stream);
            if (e != hipSuccess) return hip_fail(e, "lbm_diagnostics sync");
            (void)hipFree(c->dscratch);
            c->dscratch = nullptr;
            c->dscratch_elems = 0;
        }
        hipError_t e = hipMalloc(&c->dscratch, need * sizeof(double));
        if (e != hipSuccess) {
            c->dscratch = nullptr;
            return fail(LBM_ENOMEM, "diagnostics scratch: %s", hipGetErrorString(e));
        }
        c->dscratch_elems = need;
    }
    double* ux_s = c->dscratch;
    double* uy_s = ux_s + N;
    double* w_s = uy_s + N;
    double* part = w_s + N;
    int rc = kbc::launch_diag(c->L, c->buf[c->cur], ux_s, uy_s, w_s, part);
    if (rc) return launch_result(rc, "lbm_diagnostics");
    std::vector<double> h(static_cast<size_t>(kbc::kDiagBlocks) * kbc::kDiagSlots);
    hipError_t e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_diagnostics copy");
    e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_diagnostics sync");
    double s[kbc::kDiagSlots] = {0};
    for (int b = 0; b < kbc::kDiagBlocks; ++b)
        for (int k = 0; k < kbc::kDiagSlots; ++k) s[k] += h[static_cast<size_t>(b) * kbc::kDiagSlots + k];
    const double n = static_cast<double>(N);
    auto sd = [n](double sum, double sum2) {
        const double m = sum / n;
        const double v = sum2 / n - m * m;
        return v > 0.0 ? sqrt(v) : 0.0;
    };
    out->mass = s[0];
    out->jx = s[1];
    out->jy = s[2];
    out->E = s[3] / n;
    out->E_std = sd(s[3], s[4]);
    out->S = s[5] / n;
    out->gamma = s[6] / n;
    out->gamma_std = sd(s[6], s[7]);
    out->n_nonfinite = s[8];
    out->n_feq_nonpos = s[9];
    out->rho_std = sd(s[0], s[10]);
    out->Z = s[11] / n;
    out->Z_std = sd(s[11], s[12]);
    out->P = s[13] / n;
    out->P_std = sd(s[13], s[14]);
    out->reserved = 0.0;
    return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->steps : -1; }

int lbm_set_step(lbm_ctx* c, int64_t n) {
    if (!c || n < 0) return fail(LBM_EINVAL, "invalid ctx or step");
    c->steps = n;
    return LBM_OK;
}

void* lbm_state_buffer(const lbm_ctx* c) { return c ? c->buf[c->cur] : nullptr; }
void* lbm_work_buffer(const lbm_ctx* c) { return c ? c->buf[c->cur ^ 1] : nullptr; }

int lbm_set_tile(lbm_ctx* c, int32_t width, int32_t rows_per_thread, int32_t flags) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    kbc::StepShape s;
    s.width = width;
    s.rpt = rows_per_thread;
    s.nt = (flags & LBM_TILE_NONTEMPORAL) ? 1 : 0;
    if ((flags & ~LBM_TILE_NONTEMPORAL) != 0) return fail(LBM_EINVAL, "unknown tile flags %d", flags);
    if (!kbc::valid_shape(s)) return fail(LBM_EINVAL, "tile width must be 64, 128 or 256 and rows per thread 1, 2 or 4");
    const int rc = graph_reset(c);
    if (rc) return rc;
    c->shape = s;
    return LBM_OK;
}

int lbm_get_tile(const lbm_ctx* c, int32_t* width, int32_t* rows_per_thread, int32_t* flags) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (width) *width = c->shape.width;
    if (rows_per_thread) *rows_per_thread = c->shape.rpt;
    if (flags) *flags = c->shape.nt ? LBM_TILE_NONTEMPORAL : 0;
    return LBM_OK;
}

int lbm_set_beta(lbm_ctx* c, double beta) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(LBM_EINVAL, "beta must be in (0, 1]");
    if (beta != c->p.beta) {
        const int rc = graph_reset(c);
        if (rc) return rc;
        ++c->gen;
    }
    c->p.beta = beta;
    c->L.beta = beta;
    return LBM_OK;
}

int lbm_free(lbm_ctx* c) {
    if (!c) return LBM_OK;
    if (c->ens_refs > 0)
        return fail(LBM_EINVAL, "context is a member of %d live ensemble(s): free them first", c->ens_refs);
    int rc = LBM_OK;
    if (c->dscratch || c->ascratch || c->sscratch || c->fft_plan || c->gexec[0] || c->gexec[1] || c->cap_stream) {
        hipError_t e = hipStreamSynchronize(c->L.stream);
        if (e != hipSuccess) rc = hip_fail(e, "lbm_free sync");
        for (int k = 0; k < 2; ++k)
            if (c->gexec[k]) (void)hipGraphExecDestroy(c->gexec[k]);
        if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
        if (c->dscratch) (void)hipFree(c->dscratch);
        if (c->ascratch) (void)hipFree(c->ascratch);
        if (c->sscratch) (void)hipFree(c->sscratch);
        kbc::destroy_spectra_plan(c->fft_plan);
    }
    delete c;
    return rc;
}

int lbm_spectra(lbm_ctx* c, int32_t kmax, double* E_k, double* Z_k) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (c->p.nx != c->p.ny) return fail(LBM_EUNSUPPORTED, "spectra need a square lattice (%d x %d)", c->p.nx, c->p.ny);
    if (kmax < 0) return fail(LBM_EINVAL, "kmax must be >= 0");
    if (!E_k && !Z_k) return LBM_OK;
    const size_t n = static_cast<size_t>(c->p.nx);
    const size_t need = 2 * n * n + 4 * n * (n / 2 + 1);
    if (c->sscratch_elems < need) {
        if (c->sscratch) {
            hipError_t e = hipStreamSynchronize(c->L.stream);
            if (e != hipSuccess) return hip_fail(e, "spectra scratch sync");
            (void)hipFree(c->sscratch);
            c->sscratch = nullptr;
            c->sscratch_elems = 0;
        }
        hipError_t e = hipMalloc(&c->sscratch, need * sizeof(double));
        if (e != hipSuccess) {
            c->sscratch = nullptr;
            return fail(LBM_ENOMEM, "spectra scratch: %s", hipGetErrorString(e));
        }
        c->sscratch_elems = need;
    }
    return launch_result(kbc::launch_spectra(c->L, c->buf[c->cur], &c->fft_plan, c->sscratch, kmax, E_k, Z_k),
                         "lbm_spectra");
}

size_t lbm_adjoint_bytes(int32_t nx, int32_t ny, int32_t form) {
    const size_t pitch = lbm_required_pitch(nx, form);
    if (pitch == 0 || ny < 1) return 0;
    return 9 * static_cast<size_t>(ny) * pitch * (form == LBM_F64 ? 8 : 4);
}

int lbm_step_buffers(lbm_ctx* c, const void* src, void* dst) {
    if (!c || !src || !dst || src == dst) return fail(LBM_EINVAL, "invalid ctx or buffers");
    return launch_result(kbc::launch_step(c->L, src, dst, c->shape), "lbm_step_buffers");
}

namespace {
int ensure_ascratch(lbm_ctx* c, size_t need) {
    if (c->ascratch_elems >= need) return LBM_OK;
    if (c->ascratch) {
        hipError_t e = hipStreamSynchronize(c->L.stream);
        if (e != hipSuccess) return hip_fail(e, "adjoint scratch sync");
        (void)hipFree(c->ascratch);
        c->ascratch = nullptr;
        c->ascratch_elems = 0;
    }
    hipError_t e = hipMalloc(&c->ascratch, need * sizeof(double));
    if (e != hipSuccess) {
        c->ascratch = nullptr;
        return fail(LBM_ENOMEM, "adjoint scratch: %s", hipGetErrorString(e));
    }
    c->ascratch_elems = need;
    return LBM_OK;
}
}  // namespace

int lbm_set_adjoint_gamma(lbm_ctx* c, int32_t mode) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (mode != LBM_ADJ_GAMMA_FULL && mode != LBM_ADJ_GAMMA_FROZEN) return fail(LBM_EINVAL, "unknown adjoint gamma mode %d", mode);
    c->L.adj_frozen = (mode == LBM_ADJ_GAMMA_FROZEN) ? 1 : 0;
    return LBM_OK;
}

int lbm_adjoint_seed(lbm_ctx* c, const void* state, const double* dL_drho, const double* dL_dux,
                     const double* dL_duy, void* lam) {
    if (!c || !state || !lam) return fail(LBM_EINVAL, "ctx, state and lam must not be NULL");
    return launch_result(kbc::launch_adjoint_seed(c->L, state, dL_drho, dL_dux, dL_duy, lam), "lbm_adjoint_seed");
}

int lbm_adjoint_step_slab(lbm_ctx* c, const void* state, const void* state_lo, const void* state_hi,
                          const void* lam_in, const void* lam_lo, const void* lam_hi, void* lam_out, double* dbeta) {
    if (!c || !state || !lam_in || !lam_out || lam_in == lam_out)
        return fail(LBM_EINVAL, "ctx, state and two distinct adjoint buffers are required");
    if (!state_lo || !state_hi || !lam_lo || !lam_hi) return fail(LBM_EINVAL, "all four halo buffers are required");
    kbc::Lattice L = c->L;
    L.adj_halo[0] = state_lo;
    L.adj_halo[1] = state_hi;
    L.adj_halo[2] = lam_lo;
    L.adj_halo[3] = lam_hi;
    const int64_t nb = kbc::adjoint_partials(L), ng = kbc::adjoint_slice_len(L);
    int rc = ensure_ascratch(c, static_cast<size_t>(nb + ng));
    if (rc) return rc;
    return launch_result(kbc::launch_adjoint_step(L, state, lam_in, lam_out, c->ascratch, c->ascratch + nb, dbeta),
                         "lbm_adjoint_step_slab");
}

int lbm_adjoint_step(lbm_ctx* c, const void* state, const void* lam_in, void* lam_out, double* dbeta) {
    if (!c || !state || !lam_in || !lam_out || lam_in == lam_out)
        return fail(LBM_EINVAL, "ctx, state and two distinct adjoint buffers are required");
    const int64_t nb = kbc::adjoint_partials(c->L), ng = kbc::adjoint_slice_len(c->L);
    int rc = ensure_ascratch(c, static_cast<size_t>(nb + ng));
    if (rc) return rc;
    return launch_result(kbc::launch_adjoint_step(c->L, state, lam_in, lam_out, c->ascratch, c->ascratch + nb, dbeta),
                         "lbm_adjoint_step");
}

}  // extern "C"

namespace {

// Scratch of lbm_adjoint_step_noalloc: a fixed device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses the
// name itself (on the host it is only a stand-in for the symbol): the
// device's address comes from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) double scratch[LBM_NOALLOC_SCRATCH_DOUBLES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch` (the device must be current), or NULL
// with the error set.
double* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) {
        fail(LBM_EINVAL, "device %d out of the supported range", dev);
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "lbm_adjoint_step_noalloc scratch address");
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int lbm_adjoint_step_noalloc(lbm_ctx* c, const void* state, const void* lam_in, void* lam_out, double* dbeta) {
    if (!c || !state || !lam_in || !lam_out || lam_in == lam_out)
        return fail(LBM_EINVAL, "ctx, state and two distinct adjoint buffers are required");
    const int64_t nb = kbc::adjoint_partials(c->L), ng = kbc::adjoint_slice_len(c->L);
    if (nb + ng > static_cast<int64_t>(LBM_NOALLOC_SCRATCH_DOUBLES))
        return fail(LBM_EINVAL,
                    "lbm_adjoint_step_noalloc: this %d x %d lattice needs %lld doubles of scratch, above the "
                    "fixed %d (use lbm_adjoint_step)",
                    c->p.nx, c->p.ny, static_cast<long long>(nb + ng), LBM_NOALLOC_SCRATCH_DOUBLES);
    int dev = -1;
    const hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "lbm_adjoint_step_noalloc");
    if (dev != c->device)
        return fail(LBM_EINVAL, "lbm_adjoint_step_noalloc: device %d is current, the context's is %d", dev,
                    c->device);
    double* p = noalloc_scratch(dev);
    if (!p) return LBM_EHIP;
    return launch_result(kbc::launch_adjoint_step(c->L, state, lam_in, lam_out, p, p + nb, dbeta),
                         "lbm_adjoint_step_noalloc");
}

int lbm_adjoint_segment(lbm_ctx* c, const void* state0, void* const* slots, int32_t k, void* lam_in,
                        void* lam_out, double* dbeta, int32_t* which) {
    if (!c || !state0 || k < 1 || (k > 1 && !slots) || !lam_in || !lam_out || lam_in == lam_out || !which)
        return fail(LBM_EINVAL, "invalid adjoint segment arguments");
    for (int32_t i = 0; i + 1 < k; ++i)
        if (!slots[i]) return fail(LBM_EINVAL, "slot %d is NULL", i);
    // every adjoint step of the segment writes its dL/dbeta partials to a
    // slice of its own; one reduction at the end adds the slices, in step
    // order, to *dbeta
    const int64_t nb = kbc::adjoint_partials(c->L), ng = kbc::adjoint_slice_len(c->L);
    // room for k rounded up to 64 slices, so that segments of different
    // lengths in one backward pass do not reallocate (which synchronises)
    const int64_t kr = (static_cast<int64_t>(k) + 63) / 64 * 64;
    int rc = ensure_ascratch(c, static_cast<size_t>(nb + ng * kr + kr));
    if (rc) return rc;
    // recompute f^{s+1} .. f^{s+k-1}
    for (int32_t i = 1; i < k; ++i) {
        const void* src = (i == 1) ? state0 : slots[i - 2];
        rc = kbc::launch_step(c->L, src, slots[i - 1], c->shape);
        if (rc) return launch_result(rc, "lbm_adjoint_segment recompute");
    }
    void* a = lam_in;
    void* b = lam_out;
    for (int32_t n = k - 1; n >= 0; --n) {
        const void* st = (n == 0) ? state0 : slots[n - 1];
        rc = kbc::launch_adjoint_step(c->L, st, a, b, c->ascratch, c->ascratch + nb + static_cast<int64_t>(n) * ng,
                                      nullptr);
        if (rc) return launch_result(rc, "lbm_adjoint_segment");
        void* t = a;
        a = b;
        b = t;
    }
    rc = kbc::launch_sum_slices(c->ascratch + nb, ng, k, c->ascratch + nb + ng * kr, dbeta, c->L.stream);
    if (rc) return launch_result(rc, "lbm_adjoint_segment sum");
    *which = (a == lam_in) ? 0 : 1;
    return LBM_OK;
}

int lbm_adjoint_rollout(lbm_ctx* c, const void* const* ckpts, int32_t nsteps, int32_t seglen,
                        void* const* slots_a, void* const* slots_b, void* lam_in, void* lam_out, double* dbeta,
                        int32_t* which) {
    if (!c || !ckpts || nsteps < 1 || seglen < 1 || !lam_in || !lam_out || lam_in == lam_out || !which)
        return fail(LBM_EINVAL, "invalid adjoint rollout arguments");
    const int32_t nseg = (nsteps + seglen - 1) / seglen;
    for (int32_t j = 0; j < nseg; ++j)
        if (!ckpts[j]) return fail(LBM_EINVAL, "checkpoint %d is NULL", j);
    if (seglen > 1) {
        if (!slots_a || !slots_b) return fail(LBM_EINVAL, "two slot sets of seglen - 1 buffers are required");
        for (int32_t i = 0; i + 1 < seglen; ++i)
            if (!slots_a[i] || !slots_b[i] || slots_a[i] == slots_b[i])
                return fail(LBM_EINVAL, "slot %d is NULL or shared by both sets", i);
    }
    const int64_t nb = kbc::adjoint_partials(c->L), ng = kbc::adjoint_slice_len(c->L);
    const int64_t kr = (static_cast<int64_t>(seglen) + 63) / 64 * 64;
    int rc = ensure_ascratch(c, static_cast<size_t>(nb + ng * kr + kr));
    if (rc) return rc;
    void* const* sets[2] = {slots_a, slots_b};
    auto seg_len = [&](int32_t j) { return std::min(seglen, nsteps - j * seglen); };
    // source of recomputed state t + 1 (t = 0 .. k - 2) of segment j
    auto fsrc = [&](int32_t j, int set, int32_t t) -> const void* { return t == 0 ? ckpts[j] : sets[set][t - 1]; };
    // the last segment's states on their own
    for (int32_t t = 0; t + 1 < seg_len(nseg - 1); ++t) {
        const int r = kbc::launch_step(c->L, fsrc(nseg - 1, 0, t), sets[0][t], c->shape);
        if (r) return launch_result(r, "lbm_adjoint_rollout recompute");
    }
    void* a = lam_in;
    void* b = lam_out;
    for (int32_t j = nseg - 1; j >= 0; --j) {
        const int set = (nseg - 1 - j) & 1, nxt = set ^ 1;
        const int32_t k = seg_len(j);
        const int32_t kn = (j > 0) ? seg_len(j - 1) - 1 : 0;   // states to recompute for segment j - 1
        // adjoint step t of the segment runs backward from n = k - 1; the
        // same launch recomputes state t + 1 of segment j - 1 into the other
        // slot set (read by nothing in this segment)
        for (int32_t t = 0; t < k; ++t) {
            const int32_t n = k - 1 - t;
            const void* st = (n == 0) ? ckpts[j] : sets[set][n - 1];
            const bool fwd = t < kn;
            const int r = kbc::launch_adjoint_step(c->L, st, a, b, c->ascratch,
                                                   c->ascratch + nb + static_cast<int64_t>(n) * ng, nullptr,
                                                   fwd ? fsrc(j - 1, nxt, t) : nullptr, fwd ? sets[nxt][t] : nullptr);
            if (r) return launch_result(r, "lbm_adjoint_rollout");
            std::swap(a, b);
        }
        for (int32_t t = k; t < kn; ++t) {
            const int r = kbc::launch_step(c->L, fsrc(j - 1, nxt, t), sets[nxt][t], c->shape);
            if (r) return launch_result(r, "lbm_adjoint_rollout recompute");
        }
        const int r = kbc::launch_sum_slices(c->ascratch + nb, ng, k, c->ascratch + nb + ng * kr, dbeta, c->L.stream);
        if (r) return launch_result(r, "lbm_adjoint_rollout sum");
    }
    *which = (a == lam_in) ? 0 : 1;
    return LBM_OK;
}

int lbm_adjoint_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, int32_t mode,
                     const void* lam0, double* grad_ux, double* grad_uy, double* dbeta) {
    if (!c || !ux || !uy || !lam0 || !grad_ux || !grad_uy)
        return fail(LBM_EINVAL, "ctx, ux, uy, lam0 and both gradient outputs are required");
    if (mode != LBM_INIT_EQ && mode != LBM_INIT_GRAD_CD)
        return fail(LBM_EUNSUPPORTED, "adjoint of init mode %d is not built", mode);
    const size_t N = static_cast<size_t>(c->p.nx) * c->p.ny;
    const size_t nb = (N + 255) / 256;
    // the adjoint step's partials and folds come first
    const size_t off = static_cast<size_t>(kbc::adjoint_partials(c->L) + kbc::adjoint_slice_len(c->L));
    int rc = ensure_ascratch(c, off + nb + 4 * N);
    if (rc) return rc;
    return launch_result(kbc::launch_adjoint_init(c->L, rho, ux, uy, mode == LBM_INIT_GRAD_CD ? 1 : 0, lam0,
                                                  grad_ux, grad_uy, c->ascratch + off + nb, c->ascratch + off,
                                                  static_cast<int64_t>(nb), dbeta),
                         "lbm_adjoint_init");
}

// ------------------------------------------------------------------ ensemble
struct lbm_ens {
    std::vector<lbm_ctx*> m;
    kbc::Lattice L;             // common form, collision, variant, stabiliser, stream
    kbc::StepShape shape;
    kbc::EnsEntry* dtab;        // member table for single-step tiles
    int ntiles;
    kbc::EnsSync* dsync;        // grid-barrier state of the persistent launches
    uint32_t spin_limit;        // polls of the barrier counter before a persistent launch gives up
    int fuse;                   // steps per launch: 1 or 2
    int rows;                   // fused tile height: 8 or 16
    kbc::EnsEntry* dtab2;       // member table for fused 64 x rows tiles
    int ntiles2;
    int32_t* dmap2;             // member of each fused tile (one scalar load per workgroup)
    int64_t dmap2_len;
    int32_t* dmap;              // member of each single-step tile
    int64_t dmap_len;
    std::vector<uint64_t> gens; // member parameter generations the tables were built from
};

namespace {

const kbc::EnsSync kZeroSync{};

bool ens_shape_ok(const kbc::StepShape& s) {
    return ((s.width == 128 && s.rpt == 2) || (s.width == 256 && (s.rpt == 1 || s.rpt == 2))) &&
           (s.nt == 0 || s.nt == 1);
}

// Member table for tiles tw x th; returns the number of tiles or -1.
int64_t ens_table(const lbm_ens* e, int tw, int th, std::vector<kbc::EnsEntry>& tab) {
    tab.assign(e->m.size(), kbc::EnsEntry{});
    int64_t tiles = 0;
    for (size_t r = 0; r < e->m.size(); ++r) {
        const lbm_ctx* c = e->m[r];
        kbc::EnsEntry& t = tab[r];
        t.buf[0] = c->buf[0];
        t.buf[1] = c->buf[1];
        t.nx = c->p.nx;
        t.ny = c->p.ny;
        t.ntx = (c->p.nx + tw - 1) / tw;
        t.pitch = c->L.pitch;
        t.tile_start = static_cast<int32_t>(tiles);
        tiles += static_cast<int64_t>(t.ntx) * ((c->p.ny + th - 1) / th);
        if (!kbc::grid_fits(8 * ((tiles + 7) / 8), 256)) return -1;
        t.beta = c->L.beta;
        t.inv_beta = 1.0 / c->L.beta;
        t.two_m_inv_beta = 2.0 - 1.0 / c->L.beta;
        t.rho0 = c->L.rho0;
        t.guard = c->L.guard;
        t.gamma_fixed = c->L.gamma_fixed;
    }
    return tiles;
}

int ens_upload(lbm_ens* e, kbc::EnsEntry** dst, const std::vector<kbc::EnsEntry>& tab) {
    if (!*dst) {
        hipError_t err = hipMalloc(dst, tab.size() * sizeof(kbc::EnsEntry));
        if (err != hipSuccess) {
            *dst = nullptr;
            return fail(LBM_ENOMEM, "ensemble table: %s", hipGetErrorString(err));
        }
    }
    hipError_t err = hipStreamSynchronize(e->L.stream);
    if (err == hipSuccess)
        err = hipMemcpy(*dst, tab.data(), tab.size() * sizeof(kbc::EnsEntry), hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err, "ensemble table upload");
    return LBM_OK;
}

// Member index of every tile of a table (tiles in member order), uploaded to
// *dst, which is reallocated when the tile count changes.
int ens_map(lbm_ens* e, const std::vector<kbc::EnsEntry>& tab, int64_t tiles, int32_t** dst, int64_t* len) {
    std::vector<int32_t> map(static_cast<size_t>(tiles));
    for (size_t r = 0; r < tab.size(); ++r) {
        const int64_t end = (r + 1 < tab.size()) ? tab[r + 1].tile_start : tiles;
        for (int64_t t = tab[r].tile_start; t < end; ++t) map[static_cast<size_t>(t)] = static_cast<int32_t>(r);
    }
    hipError_t err = hipStreamSynchronize(e->L.stream);
    if (err != hipSuccess) return hip_fail(err, "ensemble tile map");
    if (*dst && *len != tiles) {
        (void)hipFree(*dst);
        *dst = nullptr;
    }
    if (!*dst) {
        err = hipMalloc(dst, static_cast<size_t>(tiles > 0 ? tiles : 1) * sizeof(int32_t));
        if (err != hipSuccess) {
            *dst = nullptr;
            return fail(LBM_ENOMEM, "ensemble tile map: %s", hipGetErrorString(err));
        }
        *len = tiles;
    }
    err = hipMemcpy(*dst, map.data(), map.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    return err == hipSuccess ? LBM_OK : hip_fail(err, "ensemble tile map upload");
}

int ens_build(lbm_ens* e) {
    std::vector<kbc::EnsEntry> tab;
    const int64_t tiles = ens_table(e, e->shape.width, (256 / e->shape.width) * e->shape.rpt, tab);
    const int64_t tiles2 = tiles < 0 ? -1 : ens_table(e, 64, e->rows, tab);
    if (tiles < 0 || tiles2 < 0)
        return fail(LBM_EUNSUPPORTED, "ensemble has too many tiles for one launch (2^32 - 1 work-items)");
    int rc = ens_upload(e, &e->dtab2, tab);
    if (rc) return rc;
    e->ntiles2 = static_cast<int>(tiles2);
    rc = ens_map(e, tab, tiles2, &e->dmap2, &e->dmap2_len);
    if (rc) return rc;
    ens_table(e, e->shape.width, (256 / e->shape.width) * e->shape.rpt, tab);
    rc = ens_upload(e, &e->dtab, tab);
    if (rc) return rc;
    rc = ens_map(e, tab, tiles, &e->dmap, &e->dmap_len);
    if (rc) return rc;
    e->ntiles = static_cast<int>(tiles);
    e->gens.resize(e->m.size());
    for (size_t r = 0; r < e->m.size(); ++r) e->gens[r] = e->m[r]->gen;
    return LBM_OK;
}

}  // namespace

int lbm_set_halo(lbm_ctx* c, const void* lo, const void* hi) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if ((lo == nullptr) != (hi == nullptr)) return fail(LBM_EINVAL, "set both halo buffers or neither");
    if (lo && c->ens_refs > 0) return fail(LBM_EINVAL, "the context belongs to a live ensemble");
    if (lo && c->fuse_rows != 8 && c->fuse_rows != 16)
        return fail(LBM_EUNSUPPORTED, "a slab runs fused tiles of 8 or 16 rows (set with lbm_set_fusion)");
    int rc = graph_reset(c);
    if (rc) return rc;
    if (lo) c->graph_chunk = 0;
    c->L.halo_lo = lo;
    c->L.halo_hi = hi;
    return LBM_OK;
}

int lbm_get_edge_rows(lbm_ctx* c, void* lo_rows, void* hi_rows) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!lo_rows || !hi_rows) return fail(LBM_EINVAL, "lo_rows and hi_rows must not be NULL");
    const size_t es = c->p.form == LBM_F16DEV_F32 ? 2 : (c->p.form == LBM_F32DEV_F32 ? 4 : 8);
    const size_t row = 9 * static_cast<size_t>(c->L.pitch) * es;   // one lattice row: nine population rows
    const char* cur = static_cast<const char*>(c->buf[c->cur]);
    hipError_t e = hipMemcpyAsync(lo_rows, cur, 2 * row, hipMemcpyDeviceToDevice, c->L.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hi_rows, cur + static_cast<size_t>(c->p.ny - 2) * row, 2 * row, hipMemcpyDeviceToDevice,
                           c->L.stream);
    return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_get_edge_rows");
}

int lbm_ensemble_create(lbm_ens** out, lbm_ctx* const* members, int32_t count) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!members || count < 1) return fail(LBM_EINVAL, "need at least one member");
    const lbm_ctx* m0 = members[0];
    for (int32_t r = 0; r < count; ++r) {
        const lbm_ctx* c = members[r];
        if (!c) return fail(LBM_EINVAL, "member %d is NULL", r);
        if (c->L.halo_lo) return fail(LBM_EINVAL, "member %d is a slab (halo buffers set); members are periodic", r);
        if (c->p.form != m0->p.form || c->p.collision != m0->p.collision ||
            (c->p.collision == LBM_KBC && c->p.variant != m0->p.variant) || c->p.gamma_mode != m0->p.gamma_mode ||
            c->p.stream != m0->p.stream)
            return fail(LBM_EINVAL, "member %d differs in form, collision, variant, stabiliser or stream", r);
        for (int32_t q = 0; q < r; ++q)
            if (members[q] == c) return fail(LBM_EINVAL, "member %d repeats member %d", r, q);
    }
    lbm_ens* e = new (std::nothrow) lbm_ens();
    if (!e) return fail(LBM_ENOMEM, "ensemble allocation failed");
    e->m.assign(members, members + count);
    e->L = m0->L;
    e->shape = default_shape(m0->p.form);
    if (!ens_shape_ok(e->shape)) {
        e->shape.width = 128;
        e->shape.rpt = 2;
    }
    {
        // every member's two buffers pass through each launch
        double state = 0.0;
        for (const lbm_ctx* c : e->m)
            state += 2.0 * 9.0 * c->p.ny * static_cast<double>(c->L.pitch) * form_bytes(c->p.form);
        if (plain_stores_pay(m0->p.form, state)) e->shape.nt = 0;
    }
    e->dtab = nullptr;
    e->dtab2 = nullptr;
    e->dmap2 = nullptr;
    e->dmap2_len = 0;
    e->dmap = nullptr;
    e->dmap_len = 0;
    e->dsync = nullptr;
    e->spin_limit = LBM_ENSEMBLE_SPIN_DEFAULT;
    // two fused steps per launch, as for single lattices
    e->fuse = 2;
    e->rows = (m0->p.form == LBM_F64) ? 8 : 16;
    int rc = ens_build(e);
    if (!rc) {
        hipError_t err = hipMalloc(&e->dsync, sizeof(kbc::EnsSync));
        if (err == hipSuccess) err = hipMemcpy(e->dsync, &kZeroSync, sizeof(kbc::EnsSync), hipMemcpyHostToDevice);
        if (err != hipSuccess) rc = fail(LBM_ENOMEM, "ensemble barrier state: %s", hipGetErrorString(err));
    }
    if (rc) {
        if (e->dsync) (void)hipFree(e->dsync);
        if (e->dtab) (void)hipFree(e->dtab);
        if (e->dtab2) (void)hipFree(e->dtab2);
        if (e->dmap2) (void)hipFree(e->dmap2);
        if (e->dmap) (void)hipFree(e->dmap);
        delete e;
        return rc;
    }
    for (lbm_ctx* c : e->m) ++c->ens_refs;
    *out = e;
    return LBM_OK;
}

int lbm_ensemble_set_tile(lbm_ens* e, int32_t width, int32_t rows_per_thread, int32_t flags) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    kbc::StepShape s;
    s.width = width;
    s.rpt = rows_per_thread;
    s.nt = (flags & LBM_TILE_NONTEMPORAL) ? 1 : 0;
    if ((flags & ~LBM_TILE_NONTEMPORAL) != 0 || !ens_shape_ok(s))
        return fail(LBM_EINVAL, "ensemble tiles: 128 x 4, 256 x 1 or 256 x 2");
    e->shape = s;
    return ens_build(e);
}

int lbm_ensemble_blocks(const lbm_ens* e) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    int blocks = 0;
    kbc::EnsLaunch a{};
    a.shape = e->shape;
    a.rows = e->rows;
    a.query_blocks = &blocks;
    const int rc = (e->fuse == 2) ? kbc::launch_ensemble2(e->L, a) : kbc::launch_ensemble(e->L, a);
    if (rc) return launch_result(rc, "lbm_ensemble_blocks");
    return blocks;
}

int lbm_ensemble_set_spin_limit(lbm_ens* e, uint32_t polls) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    if (polls > LBM_ENSEMBLE_SPIN_MAX)
        return fail(LBM_EINVAL, "spin limit %u above the maximum %u", polls, LBM_ENSEMBLE_SPIN_MAX);
    e->spin_limit = polls;
    return LBM_OK;
}

int lbm_ensemble_check(lbm_ens* e) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    hipError_t err = hipStreamSynchronize(e->L.stream);
    if (err != hipSuccess) return hip_fail(err, "lbm_ensemble_check sync");
    uint32_t failed = 0;
    err = hipMemcpy(&failed, &e->dsync->failed.v, sizeof failed, hipMemcpyDeviceToHost);
    if (err != hipSuccess) return hip_fail(err, "lbm_ensemble_check read");
    if (!failed) return LBM_OK;
    const uint32_t zero = 0;
    err = hipMemcpy(&e->dsync->failed.v, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (err != hipSuccess) return hip_fail(err, "lbm_ensemble_check clear");
    return fail(LBM_ESYNC,
                "a persistent ensemble launch gave up at a grid barrier (not every workgroup was resident "
                "within the spin limit); the members' states are invalid");
}

int lbm_ensemble_step(lbm_ens* e, int32_t nsteps, int32_t persistent) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (persistent != 0 && persistent != 1) return fail(LBM_EINVAL, "persistent must be 0 or 1");
    if (nsteps == 0) return LBM_OK;
    // a member whose parameters changed since the tables were built (e.g.
    // lbm_set_beta): rebuild them, so the ensemble keeps stepping exactly as
    // lbm_step on every member would
    for (size_t r = 0; r < e->m.size(); ++r)
        if (e->m[r]->gen != e->gens[r]) {
            const int rc = ens_build(e);
            if (rc) return rc;
            break;
        }
    const int cur = e->m[0]->cur;
    for (size_t r = 1; r < e->m.size(); ++r)
        if (e->m[r]->cur != cur) return fail(LBM_EINVAL, "members hold their states in different buffers");
    const int pairs = (e->fuse == 2) ? nsteps / 2 : 0;
    const int singles = nsteps - 2 * pairs;
    kbc::EnsLaunch a{};
    a.nmem = static_cast<int>(e->m.size());
    a.sync = e->dsync;
    a.spin_limit = e->spin_limit;
    a.shape = e->shape;
    a.stream = e->L.stream;
    a.rows = e->rows;
    int par = cur;
    if (pairs) {
        a.table = e->dtab2;
        a.tile_member = e->dmap2;
        a.ntiles = e->ntiles2;
        a.nsteps = pairs;
        a.parity = par;
        a.persistent = persistent != 0;
        const int rc = kbc::launch_ensemble2(e->L, a);
        if (rc) return launch_result(rc, "lbm_ensemble_step (two fused steps)");
        par ^= (pairs & 1);
    }
    if (singles) {
        a.table = e->dtab;
        a.tile_member = e->dmap;
        a.ntiles = e->ntiles;
        a.nsteps = singles;
        a.parity = par;
        // one leftover single step after pairs is an ordinary launch
        a.persistent = persistent != 0 && singles > 1;
        const int rc = kbc::launch_ensemble(e->L, a);
        if (rc) return launch_result(rc, "lbm_ensemble_step");
        par ^= (singles & 1);
    }
    for (lbm_ctx* c : e->m) {
        c->cur = par;
        c->steps += nsteps;
    }
    return LBM_OK;
}

int lbm_ensemble_set_fusion(lbm_ens* e, int32_t steps_per_launch, int32_t rows) {
    if (!e) return fail(LBM_EINVAL, "ensemble is NULL");
    if (steps_per_launch != 1 && steps_per_launch != 2)
        return fail(LBM_EINVAL, "steps_per_launch must be 1 or 2 (got %d)", steps_per_launch);
    if (rows != 0 && rows != 8 && rows != 16) return fail(LBM_EINVAL, "rows must be 0 (keep), 8 or 16 (got %d)", rows);
    e->fuse = steps_per_launch;
    if (rows && rows != e->rows) {
        e->rows = rows;
        return ens_build(e);
    }
    return LBM_OK;
}

int lbm_ensemble_get_fusion(const lbm_ens* e, int32_t* rows) {
    if (!e) return -1;
    if (rows) *rows = e->rows;
    return e->fuse;
}

int lbm_ensemble_free(lbm_ens* e) {
    if (!e) return LBM_OK;
    int rc = LBM_OK;
    if (e->dtab || e->dtab2 || e->dmap2 || e->dmap || e->dsync) {
        hipError_t err = hipStreamSynchronize(e->L.stream);
        if (err != hipSuccess) rc = hip_fail(err, "lbm_ensemble_free sync");
        if (e->dsync) (void)hipFree(e->dsync);
        if (e->dtab) (void)hipFree(e->dtab);
        if (e->dtab2) (void)hipFree(e->dtab2);
        if (e->dmap2) (void)hipFree(e->dmap2);
        if (e->dmap) (void)hipFree(e->dmap);
    }
    for (lbm_ctx* c : e->m) --c->ens_refs;
    delete e;
    return rc;
}

int lbm_copy_probe(void* dst, const void* src, size_t n_words, void* stream) {
    if (!dst || !src) return fail(LBM_EINVAL, "dst and src must not be NULL");
    return launch_result(kbc::launch_copy(dst, src, n_words, static_cast<hipStream_t>(stream)), "lbm_copy_probe");
}

}  // extern "C"
