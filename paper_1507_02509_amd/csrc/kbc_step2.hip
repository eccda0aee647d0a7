// kbc_step2.hip -- two fused time steps per launch (temporal blocking) on a
// single lattice; the tile body is step2_tile (kbc_tile2.hpp).
//
// Grid: 1-D, one workgroup per 64 x TH output tile.  Tiles are numbered in
// panels of kPanel tile columns (left to right; within a panel row by row,
// top to bottom) and each XCD sweeps one contiguous band of that numbering
// (workgroup b runs on XCD b % 8).  Tiles whose extended regions overlap run
// close together on one XCD, so their shared loads hit in its L2: the
// x-neighbours are consecutive and the tile below, which re-reads the two
// ring rows at the tile's bottom edge, is kPanel tiles later (row-major over
// a 16384-wide lattice it would be 256 tiles later, by which time those rows
// have left the 4 MB L2).  Only the lines at a panel's side edges are
// fetched twice.
#include "kbc_launch.hpp"
#include "kbc_tile2.hpp"

namespace kbc {

namespace {

#ifndef KBC_PANEL
#define KBC_PANEL 32
#endif
constexpr int kPanel = KBC_PANEL;   // tile columns per panel (a power of two)
static_assert(kPanel > 0 && (kPanel & (kPanel - 1)) == 0, "panel width must be a power of two");

// Tile (tx, ty) of panel-order index u: full panels of kPanel columns, then
// one panel of the remaining `last` columns (0 if ntx is a multiple).
// (With no full panel the order is row-major; otherwise kPanel * nty is at
// most the tile count, which the host keeps below 2^24: a launch holds at
// most 2^32 - 1 work-items.)
__device__ __forceinline__ void panel_tile(int u, int ntx, int nty, int& tx, int& ty) {
    const int full = ntx / kPanel;
    if (full == 0) {
        ty = u / ntx;
        tx = u - ty * ntx;
        return;
    }
    const int per_panel = kPanel * nty;
    const int p = u / per_panel;
    if (p < full) {
        const int r = u - p * per_panel;
        ty = r / kPanel;
        tx = p * kPanel + (r & (kPanel - 1));
    } else {
        const int last = ntx - full * kPanel;
        const int r = u - full * per_panel;
        ty = r / last;
        tx = full * kPanel + (r - ty * last);
    }
}

template <int FORM, int COLL, int VAR, int GM, int TH, bool NT, bool SLAB>
__global__ __launch_bounds__(256) void k_step2(const typename Form<FORM>::S* __restrict__ src,
                                               typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                               int64_t pitch, int ntx, int nty, int per_xcd,
                                               Coef<typename Form<FORM>::R> K,
                                               SlabHalo<typename Form<FORM>::S> halo) {
    const int b = blockIdx.x;
    const int u = (b & 7) * per_xcd + (b >> 3);
    if (u >= ntx * nty) return;   // the whole workgroup leaves together
    int tx, ty;
    panel_tile(u, ntx, nty, tx, ty);
    step2_tile<FORM, COLL, VAR, GM, TH, NT, SLAB>(src, dst, nx, ny, pitch, tx * 64, ty * TH, K, halo);
}

template <int FORM, int COLL, int VAR, int GM>
struct Step2Op {
    template <int TH, bool NT, bool SLAB = false>
    static int go(const Lattice& L, const void* src, void* dst) {
        using F = Form<FORM>;
        using S = typename F::S;
        const int ntx = (L.nx + 63) / 64;
        const int nty = (L.ny + TH - 1) / TH;
        const int64_t ntiles64 = static_cast<int64_t>(ntx) * nty;
        if (!grid_fits(8 * ((ntiles64 + 7) / 8), 256)) return kTooLarge;
        const int ntiles = static_cast<int>(ntiles64);
        const int per_xcd = (ntiles + 7) / 8;
        SlabHalo<S> halo;
        halo.lo = static_cast<const S*>(L.halo_lo);
        halo.hi = static_cast<const S*>(L.halo_hi);
        k_step2<FORM, COLL, VAR, GM, TH, NT, SLAB><<<dim3(8u * per_xcd), dim3(256), 0, L.stream>>>(
            static_cast<const S*>(src), static_cast<S*>(dst), L.nx, L.ny, L.pitch, ntx, nty, per_xcd,
            make_coef<typename F::R>(L), halo);
        return hipGetLastError() == hipSuccess ? 0 : -2;
    }
    template <int TH>
    static int nt(const Lattice& L, const void* src, void* dst, int nt_flag) {
        // the LDS tile must fit the 160 KB of a CU
        constexpr size_t lds = 9u * TH * 66u * sizeof(typename Form<FORM>::S);
        if constexpr (lds > 160u * 1024u) {
            return -1;
        } else {
            return nt_flag ? go<TH, true>(L, src, dst) : go<TH, false>(L, src, dst);
        }
    }
    static int run(const Lattice& L, const void* src, void* dst, int rows, int nt_flag) {
        // a slab (halo rows from buffers): 8- and 16-row tiles
        if (L.halo_lo) {
            switch (rows * 2 + (nt_flag ? 1 : 0)) {
                case 8 * 2: return go<8, false, true>(L, src, dst);
                case 8 * 2 + 1: return go<8, true, true>(L, src, dst);
                case 16 * 2: return go<16, false, true>(L, src, dst);
                case 16 * 2 + 1: return go<16, true, true>(L, src, dst);
                default: return -1;
            }
        }
        switch (rows) {
            case 8: return nt<8>(L, src, dst, nt_flag);
            case 16: return nt<16>(L, src, dst, nt_flag);
            case 24: return nt<24>(L, src, dst, nt_flag);
            case 32: return nt<32>(L, src, dst, nt_flag);
            default: return -1;
        }
    }
};

}  // namespace

int launch_step2(const Lattice& L, const void* src, void* dst, int rows, int nt) {
    return dispatch<Step2Op>(L, src, dst, rows, nt);
}

}  // namespace kbc
