// kbc_ensemble.hip -- many independent lattices of different sizes advanced by
// one kernel.
//
// A device table lists the members (buffers, size, pitch, beta) and the first
// index of each member's tiles in one global tile numbering (members in order,
// row-major tiles within a member); a per-tile index gives each tile's member.
// The tile range is cut into eight equal contiguous bands, one per XCD
// (workgroup b runs on XCD b % 8), and the workgroups of an XCD deal its band
// out round-robin, so x-neighbour tiles of one member meet in the same L2 as in
// the single-lattice step.
//
// Launch modes:
//   * k_ens: one launch per step, one workgroup per tile (tile body of the
//     single-lattice step, kbc_tile.hpp);
//   * k_ens2: one launch per two fused steps, one workgroup per 64 x TH output
//     tile (tile body of the single-lattice fused kernel, kbc_tile2.hpp);
//   * k_ens_persist / k_ens2_persist: ONE launch for many steps (or pairs of
//     steps): as many workgroups as the GPU holds at once, each taking tiles
//     of its XCD's band as it asks for them (BandTiles), with a grid barrier
//     between steps.
// All of them run the per-node code of the single-lattice step on the same
// tiles, so results are bitwise identical to stepping each member alone.
//
// The grid barrier (grid_barrier) counts arrivals in device memory: a
// workgroup finishing a step counts itself in and waits until every workgroup
// of the grid has.  That wait ends only if every workgroup of the grid is
// resident at the same time, so the grid is capped at the resident capacity
// computed from both the runtime's occupancy figure and the kernel's own LDS
// and register use (resident_blocks).  As a safeguard the wait is bounded: a
// workgroup that has polled the counter `spin_limit` times sets a give-up flag,
// after which every wait of the launch returns at once, so the launch always
// ends; the host reads the sticky flag (lbm_ensemble_check) and reports the
// states as invalid.
#include <algorithm>

#include "kbc_launch.hpp"
#include "kbc_tile.hpp"
#include "kbc_tile2.hpp"

namespace kbc {

namespace {

template <typename R>
__device__ __forceinline__ Coef<R> coef_of(const EnsEntry& e) {
    Coef<R> K;
    K.beta = static_cast<R>(e.beta);
    K.inv_beta = static_cast<R>(e.inv_beta);
    K.two_m_inv_beta = static_cast<R>(e.two_m_inv_beta);
    K.rho0 = static_cast<R>(e.rho0);
    K.guard = static_cast<R>(e.guard);
    K.gamma_fixed = static_cast<R>(e.gamma_fixed);
    return K;
}

// Barrier number `b` (1, 2, ...) over the whole grid of a persistent launch.
// Arrival is counted in two levels so that no single counter takes every
// workgroup's atomic: workgroup j of XCD band x adds one to group[x]; the
// last of the band's m workgroups to arrive at barrier b (it reads b m - 1)
// adds one to `count`; everyone waits until `count` reaches 8 b.
// Memory order: every wave first waits until its own stores of the step have
// completed (they are then in the L2 of its XCD); after a workgroup barrier
// one thread makes them visible at device scope (release fence: the L2 is
// written back) and counts the workgroup in; the last arriver of a band
// first acquires what the band released and releases it on with its count
// (acquire-release fence); after the wait, the thread drops cached lines that
// another XCD may have rewritten (acquire fence: the CU's L1 and the
// non-coherent L2 lines are invalidated) before the workgroup goes on.  One
// write-back and one invalidation per workgroup, not per wave: each acts on a
// whole cache.  Counters are read and written with device-scope atomics.
__device__ __forceinline__ void grid_barrier(EnsSync* sy, uint32_t b, uint32_t spin_limit) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t m = gridDim.x >> 3;
        const uint32_t old = __hip_atomic_fetch_add(&sy->group[blockIdx.x & 7u].v, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1u == b * m) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_fetch_add(&sy->count.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const uint32_t target = 8u * b;
        for (uint32_t it = 0;; ++it) {
            if (__hip_atomic_load(&sy->count.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (__hip_atomic_load(&sy->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
            if (it >= spin_limit) {
                __hip_atomic_store(&sy->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&sy->failed.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Clears the group counters, the arrival count and the give-up flag before a
// persistent launch (the sticky `failed` word is left for the host).
__global__ void k_sync_reset(EnsSync* sy) {
    const unsigned t = threadIdx.x;
    if (t < 8) sy->group[t].v = 0u;
    if (t == 8) sy->count.v = 0u;
    if (t == 9) sy->abort.v = 0u;
    if (t >= 16 && t < 24) sy->claim[t - 16].v = 0u;
}

// Tiles of a persistent launch are handed out per band as the workgroups ask
// for them: claim index k of band x is tile start + k mod B of step k / B
// (B tiles in the band), from one counter per band that runs through all the
// launch's steps; every index below steps x B is taken by exactly one
// workgroup.  For single steps a workgroup asks for its next tile as it
// starts one (the counter's round trip overlaps the short tile's loads) and
// ends a step holding one claim of the next step.  For pairs of fused steps
// it asks when it has finished a tile: a tile claimed a whole (long) fused
// tile ahead starts that much later than the tiles claimed next to it, and
// the vertically adjacent tile then no longer finds the two ring rows they
// share in L2 (measured on the 256-member ensemble: 4.40 GB read per launch
// of two steps with the early claim, 3.52 GB with the late one, 3.28 GB
// algorithmic).  The claimed index passes through LDS, double buffered so
// that a value is overwritten only after every wave has read it.
struct BandTiles {
    int start, B;
    uint32_t* ctr;
};
__device__ __forceinline__ BandTiles band_tiles(EnsSync* sy, int ntiles) {
    const int x = static_cast<int>(blockIdx.x & 7u);
    const int band = (ntiles + 7) >> 3;
    BandTiles bt;
    bt.start = x * band;
    const int end = (bt.start + band < ntiles) ? bt.start + band : ntiles;
    bt.B = end > bt.start ? end - bt.start : 0;
    bt.ctr = &sy->claim[x].v;
    return bt;
}
__device__ __forceinline__ int claim_tile(const BandTiles& bt) {
    return static_cast<int>(__hip_atomic_fetch_add(bt.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT>
__global__ __launch_bounds__(256) void k_ens(const EnsEntry* __restrict__ tab,
                                             const int32_t* __restrict__ tile_member, int ntiles, int per_xcd,
                                             int parity) {
    using F = Form<FORM>;
    using S = typename F::S;
    using R = typename F::R;
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    // member holding tile t, from the per-tile index (one scalar load)
    const EnsEntry& e = tab[tile_member[t]];
    const int lt = t - e.tile_start;
    step_tile<FORM, COLL, VAR, GM, TXW, RPT, NT>(static_cast<const S*>(e.buf[parity]),
                                                 static_cast<S*>(e.buf[parity ^ 1]), e.nx, e.ny, e.pitch,
                                                 lt % e.ntx, lt / e.ntx, coef_of<R>(e));
}

// The member of tile t comes from a per-tile index (one scalar load) rather
// than a binary search over the table, whose dependent loads would stall
// every workgroup at its start.
template <int FORM, int COLL, int VAR, int GM, int TH, bool NT>
__global__ __launch_bounds__(256) void k_ens2(const EnsEntry* __restrict__ tab,
                                              const int32_t* __restrict__ tile_member, int ntiles, int per_xcd,
                                              int parity) {
    using F = Form<FORM>;
    using S = typename F::S;
    using R = typename F::R;
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;   // the whole workgroup leaves together
    const EnsEntry& e = tab[tile_member[t]];
    const int lt = t - e.tile_start;
    step2_tile<FORM, COLL, VAR, GM, TH, NT>(static_cast<const S*>(e.buf[parity]), static_cast<S*>(e.buf[parity ^ 1]),
                                            e.nx, e.ny, e.pitch, (lt % e.ntx) * 64, (lt / e.ntx) * TH,
                                            coef_of<R>(e));
}

// Persistent single steps over the band tiles (BandTiles).
template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT>
__global__ __launch_bounds__(256) void k_ens_persist(const EnsEntry* __restrict__ tab,
                                                     const int32_t* __restrict__ tile_member, int ntiles,
                                                     int nsteps, int parity, EnsSync* sync, uint32_t spin_limit) {
    using F = Form<FORM>;
    using S = typename F::S;
    using R = typename F::R;
    __shared__ int s_claim[2];
    const BandTiles bt = band_tiles(sync, ntiles);
    if (threadIdx.x == 0) s_claim[0] = claim_tile(bt);
    __syncthreads();
    int k = s_claim[0], p = 0;
    for (int s = 0; s < nsteps; ++s) {
        const int par = (parity + s) & 1;
        const int base = s * bt.B;
        while (k < base + bt.B) {
            p ^= 1;
            int next = 0;
            if (threadIdx.x == 0) next = claim_tile(bt);
            const int t = bt.start + (k - base);
            const EnsEntry& e = tab[tile_member[t]];
            const int lt = t - e.tile_start;
            step_tile<FORM, COLL, VAR, GM, TXW, RPT, NT>(static_cast<const S*>(e.buf[par]),
                                                         static_cast<S*>(e.buf[par ^ 1]), e.nx, e.ny, e.pitch,
                                                         lt % e.ntx, lt / e.ntx, coef_of<R>(e));
            if (threadIdx.x == 0) s_claim[p] = next;
            __syncthreads();
            k = s_claim[p];
        }
        if (s + 1 < nsteps) grid_barrier(sync, static_cast<uint32_t>(s + 1), spin_limit);
    }
}

// Persistent pairs of fused steps over the band tiles (BandTiles); the tile
// body holds a workgroup barrier and reuses the LDS windows, so consecutive
// tiles of a workgroup are separated by one more barrier.
template <int FORM, int COLL, int VAR, int GM, int TH, bool NT>
__global__ __launch_bounds__(256) void k_ens2_persist(const EnsEntry* __restrict__ tab,
                                                      const int32_t* __restrict__ tile_member, int ntiles,
                                                      int npairs, int parity, EnsSync* sync, uint32_t spin_limit) {
    using F = Form<FORM>;
    using S = typename F::S;
    using R = typename F::R;
    __shared__ int s_claim[2];
    const BandTiles bt = band_tiles(sync, ntiles);
    if (threadIdx.x == 0) s_claim[0] = claim_tile(bt);
    __syncthreads();
    int k = s_claim[0], p = 0;
    for (int s = 0; s < npairs; ++s) {
        const int par = (parity + s) & 1;
        const int base = s * bt.B;
        while (k < base + bt.B) {
            p ^= 1;
            const int t = bt.start + (k - base);
            const EnsEntry& e = tab[tile_member[t]];
            const int lt = t - e.tile_start;
            step2_tile<FORM, COLL, VAR, GM, TH, NT>(static_cast<const S*>(e.buf[par]),
                                                    static_cast<S*>(e.buf[par ^ 1]), e.nx, e.ny, e.pitch,
                                                    (lt % e.ntx) * 64, (lt / e.ntx) * TH, coef_of<R>(e));
            if (threadIdx.x == 0) s_claim[p] = claim_tile(bt);
            __syncthreads();
            k = s_claim[p];
        }
        if (s + 1 < npairs) grid_barrier(sync, static_cast<uint32_t>(s + 1), spin_limit);
    }
}

// Workgroups of 256 threads that the GPU holds at once for `kern`, a multiple
// of 8 (one band per XCD): CUs x the smaller of the runtime's occupancy figure
// and the kernel's own limits -- 8 workgroups of four waves per CU (eight
// waves per SIMD), the LDS of a CU over the workgroup's static LDS, and the
// 512 vector registers of a SIMD lane over the kernel's register count.
// Returns 0 on failure.
int resident_blocks(const void* kern) {
    int dev = 0, cus = 0, lds_cu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, 0) != hipSuccess) return 0;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, kern) != hipSuccess) return 0;
    int own = 8;
    if (fa.sharedSizeBytes > 0) {
        const int granule = 512;
        const int lds = static_cast<int>((fa.sharedSizeBytes + granule - 1) / granule * granule);
        own = std::min(own, lds_cu / lds);
    }
    if (fa.numRegs > 0) own = std::min(own, 512 / ((fa.numRegs + 7) / 8 * 8));
    per_cu = std::min(per_cu, own);
    if (per_cu < 1 || cus < 1) return 0;
    return (per_cu * cus) / 8 * 8;
}

// One persistent launch per chunk of steps: the arrival counter is 32-bit, so
// a chunk holds at most (2^32 - 1) / blocks barriers.
template <typename Kern>
int launch_persistent(Kern kern, const EnsLaunch& a, int blocks) {
    if (!a.sync || blocks < 8 || blocks % 8) return -1;
    // the arrival counters are 32-bit, and a band's tile counter must stay
    // below 2^31 (steps x band tiles plus one claim per workgroup)
    const int64_t band = (a.ntiles + 7) / 8;
    const int64_t max_chunk = std::min<int64_t>(static_cast<int64_t>(0xffffffffu) / blocks,
                                                ((int64_t{1} << 31) - 1 - blocks) / (band + 1));
    const EnsEntry* tab = a.table;
    const int32_t* map = a.tile_member;
    int done = 0;
    while (done < a.nsteps) {
        const int n = static_cast<int>(std::min<int64_t>(a.nsteps - done, max_chunk));
        k_sync_reset<<<1, 64, 0, a.stream>>>(a.sync);
        if (hipGetLastError() != hipSuccess) return -2;
        kern<<<dim3(static_cast<unsigned>(blocks)), dim3(256), 0, a.stream>>>(tab, map, a.ntiles, n,
                                                                            (a.parity + done) & 1, a.sync,
                                                                            a.spin_limit);
        if (hipGetLastError() != hipSuccess) return -2;
        done += n;
    }
    return 0;
}

// a.nsteps launches of two fused steps (or, persistent, one launch for all of them)
template <int FORM, int COLL, int VAR, int GM>
struct Ens2Op {
    template <int TH, bool NT>
    static int go(const EnsLaunch& a) {
        if (a.persistent || a.query_blocks) {
            auto kern = k_ens2_persist<FORM, COLL, VAR, GM, TH, NT>;
            const int blocks = resident_blocks(reinterpret_cast<const void*>(kern));
            if (a.query_blocks) {
                *a.query_blocks = blocks;
                return blocks > 0 ? 0 : -2;
            }
            return launch_persistent(kern, a, blocks);
        }
        const int per_xcd = (a.ntiles + 7) / 8;
        for (int s = 0; s < a.nsteps; ++s) {
            const int par = (a.parity + s) & 1;
            k_ens2<FORM, COLL, VAR, GM, TH, NT><<<dim3(8u * static_cast<unsigned>(per_xcd)), dim3(256), 0, a.stream>>>(
                a.table, a.tile_member, a.ntiles, per_xcd, par);
            if (hipGetLastError() != hipSuccess) return -2;
        }
        return 0;
    }
    static int run(const Lattice& L, const EnsLaunch& a) {
        (void)L;
        if (!a.tile_member && !a.query_blocks) return -1;
        switch (a.rows * 2 + (a.shape.nt ? 1 : 0)) {
            case 8 * 2: return go<8, false>(a);
            case 8 * 2 + 1: return go<8, true>(a);
            case 16 * 2: return go<16, false>(a);
            case 16 * 2 + 1: return go<16, true>(a);
            default: return -1;
        }
    }
};

// a.nsteps single steps: one launch each (or, persistent, one launch for all)
template <int FORM, int COLL, int VAR, int GM>
struct EnsOp {
    template <int TXW, int RPT, bool NT>
    static int go(const EnsLaunch& a) {
        if (a.persistent || a.query_blocks) {
            auto kern = k_ens_persist<FORM, COLL, VAR, GM, TXW, RPT, NT>;
            const int blocks = resident_blocks(reinterpret_cast<const void*>(kern));
            if (a.query_blocks) {
                *a.query_blocks = blocks;
                return blocks > 0 ? 0 : -2;
            }
            return launch_persistent(kern, a, blocks);
        }
        const int per_xcd = (a.ntiles + 7) / 8;
        for (int s = 0; s < a.nsteps; ++s) {
            const int par = (a.parity + s) & 1;
            k_ens<FORM, COLL, VAR, GM, TXW, RPT, NT><<<dim3(8u * static_cast<unsigned>(per_xcd)), dim3(256), 0,
                                                       a.stream>>>(a.table, a.tile_member, a.ntiles, per_xcd, par);
            if (hipGetLastError() != hipSuccess) return -2;
        }
        return 0;
    }
    static int run(const Lattice& L, const EnsLaunch& a) {
        (void)L;
        if (!a.tile_member && !a.query_blocks) return -1;
        const StepShape& sh = a.shape;
        const int key = sh.width * 16 + sh.rpt;
        if (sh.nt) {
            switch (key) {
                case 128 * 16 + 2: return go<2, 2, true>(a);
                case 256 * 16 + 1: return go<4, 1, true>(a);
                case 256 * 16 + 2: return go<4, 2, true>(a);
                default: return -5;
            }
        }
        switch (key) {
            case 128 * 16 + 2: return go<2, 2, false>(a);
            case 256 * 16 + 1: return go<4, 1, false>(a);
            case 256 * 16 + 2: return go<4, 2, false>(a);
            default: return -5;
        }
    }
};

}  // namespace

int launch_ensemble(const Lattice& L, const EnsLaunch& a) { return dispatch<EnsOp>(L, a); }
int launch_ensemble2(const Lattice& L, const EnsLaunch& a) { return dispatch<Ens2Op>(L, a); }

}  // namespace kbc
