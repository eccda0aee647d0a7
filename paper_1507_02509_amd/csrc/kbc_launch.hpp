// kbc_launch.hpp -- host-side launch interface between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kbc_device.hpp"

namespace kbc {

// Largest lattice side: a lane's byte offset within a population row (x times
// the element size, at most 8 bytes) stays a 32-bit value.
constexpr int32_t kMaxSide = 1 << 28;

// A dispatch's grid size is a 32-bit count of work-items, so one launch holds
// at most 2^32 - 1 of them.  Launch helpers return kTooLarge when a lattice
// would need more.
constexpr int kTooLarge = -6;
inline bool grid_fits(int64_t blocks, int64_t threads_per_block) {
    return blocks >= 1 && blocks <= (int64_t{0xffffffff} / threads_per_block);
}

// Everything a kernel launch needs about one lattice.
struct Lattice {
    int nx, ny;
    int64_t pitch;          // elements per row
    int form, collision, variant, gamma_mode;
    double beta, rho0, guard, gamma_fixed;
    hipStream_t stream;
    int adj_frozen;         // adjoint holds gamma at its forward value
    // slab of a domain split in y: rows -2, -1 (lo) and ny, ny + 1 (hi) of
    // the current state, [2][9][pitch] each in the storage form; null for a
    // periodic lattice.  Only the step launches read them.
    const void* halo_lo = nullptr;
    const void* halo_hi = nullptr;
    // adjoint step of a slab: the same two-row halos of the state f^n (lo,
    // hi) and of the incoming adjoint lambda^(n+1) (lo, hi; [2][9][pitch] of
    // the adjoint type); null for a periodic lattice
    const void* adj_halo[4] = {nullptr, nullptr, nullptr, nullptr};
};

// step kernel tile: `width` in {64, 128, 256} nodes, each thread walks `rpt`
// in {1, 2, 4} rows; the tile is width x (256 / width) * rpt nodes; `nt`
// selects non-temporal stores
struct StepShape {
    int width;
    int rpt;
    int nt;
};
bool valid_shape(const StepShape& s);

int launch_step(const Lattice& L, const void* src, void* dst, const StepShape& shape);
// two fused steps src -> dst (kbc_step2.hip): output tiles of 64 x rows
// nodes, rows in {8, 16, 24, 32} (32 not for FP64); nt: non-temporal stores
int launch_step2(const Lattice& L, const void* src, void* dst, int rows, int nt);
int launch_init(const Lattice& L, void* dst, const double* rho, const double* ux, const double* uy,
                const double* grad, int mode);
int launch_moments(const Lattice& L, const void* src, double* rho, double* ux, double* uy,
                   double* gamma);
int launch_get_pop(const Lattice& L, const void* src, double* f);
int launch_set_pop(const Lattice& L, void* dst, const double* f);

// diagnostics: three passes writing per-block FP64 partials (kDiagSlots each)
constexpr int kDiagSlots = 16;
constexpr int kDiagBlocks = 1024;
int launch_diag(const Lattice& L, const void* src, double* ux_s, double* uy_s, double* w_s,
                double* partials);

int launch_copy(void* dst, const void* src, size_t n_words, hipStream_t stream);

// ensemble (kbc_ensemble.hip): one table entry per member lattice
struct EnsEntry {
    void* buf[2];           // the member's two population buffers
    int32_t nx, ny;
    int32_t ntx;            // tiles per row for the ensemble's tile shape
    int32_t tile_start;     // first global tile index of this member
    int64_t pitch;
    double beta, inv_beta, two_m_inv_beta, rho0, guard, gamma_fixed;
};
// Grid-barrier state of a persistent ensemble launch (device memory owned by
// the ensemble): eight group arrival counters (one per XCD band of
// workgroups), the count of groups that have arrived, this launch's give-up
// flag and the bands' tile counters are reset by a small kernel before every
// persistent launch;
// `failed` is sticky until the host reads it (lbm_ensemble_check).  Each word
// has a 128-byte line of its own.
struct EnsSync {
    struct Line {
        uint32_t v;
        uint32_t pad[31];
    };
    Line group[8];
    Line count;
    Line abort;
    Line failed;
    Line claim[8];          // tile counters of the eight bands, through all steps of a launch
};
struct EnsLaunch {
    const EnsEntry* table;  // device copy of the member table
    int nmem, ntiles, nsteps, parity;
    bool persistent;        // one launch of resident workgroups for all nsteps
    EnsSync* sync;          // persistent: barrier state
    uint32_t spin_limit;    // persistent: polls of the barrier counter before giving up
    StepShape shape;        // (128,2), (256,1) or (256,2), with or without nt
    hipStream_t stream;
    int* query_blocks;      // if set: only report the persistent launch's grid size
    int rows;               // fused launches: output tile height (8 or 16)
    const int32_t* tile_member;   // member of each tile (device)
};
int launch_ensemble(const Lattice& L, const EnsLaunch& a);
// two fused steps per launch for every member; a.nsteps counts launches, the
// table's tiles are 64 x a.rows (kbc_ensemble.hip)
int launch_ensemble2(const Lattice& L, const EnsLaunch& a);

// adjoint (kbc_adjoint.hip).  An adjoint step writes its per-workgroup
// dL/dbeta sums as one slice of adjoint_slice_len(L) doubles to `slice`
// (through adjoint_partials(L) doubles of scratch at `partials` on large
// lattices, where they are folded); if `acc` is set the slice is added to
// *acc.  launch_sum_slices adds k consecutive slices, last first, using k
// doubles of scratch at `tot`.
// launch_adjoint_init needs nblocks_cap >= ceil(nx ny / 256).
int64_t adjoint_partials(const Lattice& L);
int64_t adjoint_slice_len(const Lattice& L);
int launch_sum_slices(const double* slices, int64_t len, int k, double* tot, double* acc, hipStream_t stream);
int launch_adjoint_seed(const Lattice& L, const void* state, const double* drho, const double* dux,
                        const double* duy, void* lam);
// fsrc / fdst (both or neither): one forward step between two other state
// buffers, run in the same launch as the adjoint step
int launch_adjoint_step(const Lattice& L, const void* state, const void* lin, void* lout, double* partials,
                        double* slice, double* acc, const void* fsrc = nullptr, void* fdst = nullptr);
int launch_adjoint_init(const Lattice& L, const double* rho, const double* ux, const double* uy, int mode,
                        const void* lam0, double* gux, double* guy, double* P, double* partials,
                        int64_t nblocks_cap, double* acc);

// shell-summed energy and enstrophy spectra of a square lattice
// (kbc_spectra.hip); *plan_slot caches the FFT plan (destroy_spectra_plan);
// work: 2 n^2 + 4 n (n/2 + 1) doubles; ek, zk: kmax + 1 doubles (nullable)
int launch_spectra(const Lattice& L, const void* state, void** plan_slot, double* work, int kmax, double* ek,
                   double* zk);
void destroy_spectra_plan(void* plan);

// kernel-name lookup for profiling output
const char* step_kernel_name(const Lattice& L);

template <typename R>
inline Coef<R> make_coef(const Lattice& L) {
    Coef<R> k;
    k.beta = static_cast<R>(L.beta);
    k.inv_beta = static_cast<R>(1.0 / L.beta);
    k.two_m_inv_beta = static_cast<R>(2.0 - 1.0 / L.beta);
    k.rho0 = static_cast<R>(L.rho0);
    k.guard = static_cast<R>(L.guard);
    k.gamma_fixed = static_cast<R>(L.gamma_fixed);
    return k;
}

// Calls Op<FORM, COLL, VAR, GM>::run(args...) for the lattice's configuration.
// LBGK ignores the variant and the stabiliser mode.  Returns -5 for
// combinations that are not built.
template <template <int, int, int, int> class Op, int F, int V, typename... A>
int dispatch_gm(int gm, A&&... a) {
    switch (gm) {
        case GEST: return Op<F, KBCC, V, GEST>::run(a...);
        case GFIX: return Op<F, KBCC, V, GFIX>::run(a...);
        case GEXACT: return Op<F, KBCC, V, GEXACT>::run(a...);
        default: return -5;
    }
}
template <template <int, int, int, int> class Op, int F, typename... A>
int dispatch_var(int var, int gm, A&&... a) {
    switch (var) {
        case VA: return dispatch_gm<Op, F, VA>(gm, a...);
        case VB: return dispatch_gm<Op, F, VB>(gm, a...);
        case VC: return dispatch_gm<Op, F, VC>(gm, a...);
        case VD: return dispatch_gm<Op, F, VD>(gm, a...);
        default: return -1;
    }
}
template <template <int, int, int, int> class Op, int F, typename... A>
int dispatch_coll(int coll, int var, int gm, A&&... a) {
    if (coll == LBGK) return Op<F, LBGK, VA, GEST>::run(a...);
    return dispatch_var<Op, F>(var, gm, a...);
}
template <template <int, int, int, int> class Op, typename... A>
int dispatch(const Lattice& L, A&&... a) {
    switch (L.form) {
        case F16: return dispatch_coll<Op, F16>(L.collision, L.variant, L.gamma_mode, L, a...);
        case F32: return dispatch_coll<Op, F32>(L.collision, L.variant, L.gamma_mode, L, a...);
        case F64: return dispatch_coll<Op, F64>(L.collision, L.variant, L.gamma_mode, L, a...);
        default: return -1;
    }
}

}  // namespace kbc
