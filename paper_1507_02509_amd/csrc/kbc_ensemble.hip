// kbc_ensemble.hip -- many independent lattices of different sizes advanced by
// one kernel.
//
// A device table lists the members (buffers, size, pitch, beta) and the first
// index of each member's tiles in one global tile numbering (members in order,
// row-major tiles within a member); a per-tile index gives each tile's member.  The tile range is cut into eight equal
// contiguous bands, one per XCD (workgroup b runs on XCD b % 8), and the
// workgroups of an XCD deal its band out round-robin, so x-neighbour tiles of
// one member meet in the same L2 as in the single-lattice step.
//
// The same kernel runs in two modes:
//   * one launch per step (nsteps = 1): one workgroup per tile;
//   * one persistent cooperative launch for many steps: as many workgroups as
//     can be resident, looping over their tiles each step, with a grid-wide
//     barrier between steps (cooperative groups; the barrier's device-scope
//     fences make the new states of every XCD visible to all others).
// Both modes run the per-node code of the single-lattice step on the same
// tiles, so results are bitwise identical to stepping each member alone.
//
// k_ens2 advances every member by two fused steps per launch (the tile body
// of the single-lattice fused kernel, 64 x TH output tiles, one workgroup per
// tile), again bitwise identical to single steps.
#include <hip/hip_cooperative_groups.h>

#include "kbc_launch.hpp"
#include "kbc_tile.hpp"
#include "kbc_tile2.hpp"

namespace kbc {

namespace {

template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT>
__global__ __launch_bounds__(256) void k_ens(const EnsEntry* __restrict__ tab,
                                             const int32_t* __restrict__ tile_member, int ntiles, int nsteps,
                                             int parity) {
    using F = Form<FORM>;
    using S = typename F::S;
    using R = typename F::R;
    const int xcd = static_cast<int>(blockIdx.x & 7u), j = static_cast<int>(blockIdx.x >> 3);
    const int m = static_cast<int>(gridDim.x >> 3);
    const int band = (ntiles + 7) >> 3;
    const int start = xcd * band;
    const int end = (start + band < ntiles) ? start + band : ntiles;
    for (int s = 0; s < nsteps; ++s) {
        const int par = (parity + s) & 1;
        for (int t = start + j; t < end; t += m) {
            // member holding tile t, from the per-tile index (one scalar load)
            const EnsEntry& e = tab[tile_member[t]];
            Coef<R> K;
            K.beta = static_cast<R>(e.beta);
            K.inv_beta = static_cast<R>(e.inv_beta);
            K.two_m_inv_beta = static_cast<R>(e.two_m_inv_beta);
            K.rho0 = static_cast<R>(e.rho0);
            K.guard = static_cast<R>(e.guard);
            K.gamma_fixed = static_cast<R>(e.gamma_fixed);
            const int lt = t - e.tile_start;
            step_tile<FORM, COLL, VAR, GM, TXW, RPT, NT>(
                static_cast<const S*>(e.buf[par]), static_cast<S*>(e.buf[par ^ 1]), e.nx, e.ny, e.pitch,
                lt % e.ntx, lt / e.ntx, K);
        }
        if (s + 1 < nsteps) cooperative_groups::this_grid().sync();
    }
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
    Coef<R> K;
    K.beta = static_cast<R>(e.beta);
    K.inv_beta = static_cast<R>(e.inv_beta);
    K.two_m_inv_beta = static_cast<R>(e.two_m_inv_beta);
    K.rho0 = static_cast<R>(e.rho0);
    K.guard = static_cast<R>(e.guard);
    K.gamma_fixed = static_cast<R>(e.gamma_fixed);
    const int lt = t - e.tile_start;
    step2_tile<FORM, COLL, VAR, GM, TH, NT>(static_cast<const S*>(e.buf[parity]), static_cast<S*>(e.buf[parity ^ 1]),
                                            e.nx, e.ny, e.pitch, (lt % e.ntx) * 64, (lt / e.ntx) * TH, K);
}

// one fused launch per two steps: a.nsteps launches, each src -> dst
template <int FORM, int COLL, int VAR, int GM>
struct Ens2Op {
    template <int TH, bool NT>
    static int go(const EnsLaunch& a) {
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
        if (!a.tile_member) return -1;
        switch (a.rows * 2 + (a.shape.nt ? 1 : 0)) {
            case 8 * 2: return go<8, false>(a);
            case 8 * 2 + 1: return go<8, true>(a);
            case 16 * 2: return go<16, false>(a);
            case 16 * 2 + 1: return go<16, true>(a);
            default: return -1;
        }
    }
};

template <int FORM, int COLL, int VAR, int GM>
struct EnsOp {
    template <int TXW, int RPT, bool NT>
    static int go(const EnsLaunch& a) {
        auto kern = k_ens<FORM, COLL, VAR, GM, TXW, RPT, NT>;
        if (a.query_blocks) {
            int per_cu = 0, dev = 0, cus = 0;
            if (hipGetDevice(&dev) != hipSuccess) return -2;
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kern), 256, 0) !=
                hipSuccess)
                return -2;
            *a.query_blocks = (per_cu * cus) / 8 * 8;
            return 0;
        }
        const EnsEntry* tab = a.table;
        const int32_t* map = a.tile_member;
        int ntiles = a.ntiles, nsteps = a.nsteps, parity = a.parity;
        if (!map) return -1;
        if (!a.persistent) {
            const int band = (ntiles + 7) / 8;
            for (int s = 0; s < nsteps; ++s) {
                const int one = 1, par = (parity + s) & 1;
                kern<<<dim3(8u * static_cast<unsigned>(band)), dim3(256), 0, a.stream>>>(tab, map, ntiles, one, par);
                if (hipGetLastError() != hipSuccess) return -2;
            }
            return 0;
        }
        if (a.blocks < 8 || a.blocks % 8) return -1;
        void* args[] = {&tab, &map, &ntiles, &nsteps, &parity};
        if (hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(static_cast<unsigned>(a.blocks)),
                                       dim3(256), args, 0, a.stream) != hipSuccess)
            return -2;
        return 0;
    }
    static int run(const Lattice& L, const EnsLaunch& a) {
        (void)L;
        return shapes(a);
    }
    static int shapes(const EnsLaunch& a) {
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
