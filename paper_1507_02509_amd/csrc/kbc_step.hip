// kbc_step.hip -- fused pull-stream + collide step for gfx950.
//
// Layout: [ny][9][pitch] (x fastest): for every lattice row, the nine
// population rows one after another, deviations g_i = f_i - W_i rho0 in the
// storage form.  Rows of the nine populations are 9 * pitch elements apart
// rather than a whole plane, so a wave's 18 streams fall in three short
// address ranges (rows y - 1, y, y + 1) instead of nine 1 GiB-apart planes;
// on this GPU that raises the sustained rate of the step's access pattern
// from about 5.3 to 6.0 TB/s.  A node gathers population i from
// x - v_i (eq. Egeneral read right to left: the populations that stream into x
// this step left their source node after the previous collision), collides,
// and writes all nine values at x.  Every stored element is read exactly once
// per step (the pull is a bijection per population), so HBM traffic is 9 loads and
// 9 stores per node.  Loads of the six planes with v_x != 0 are shifted by one
// element; the wave's 64 lanes still cover one contiguous 64-element run, so
// the extra cache line per run is shared with the neighbouring wave through
// L2.  Vertical shifts are whole rows.
//
// Workgroup: 256 threads = 4 waves arranged as TXW waves side by side in x
// and 4 / TXW wave rows; each thread walks RPT consecutive rows, so a tile is
// 64 * TXW nodes wide and (4 / TXW) * RPT rows tall.  The grid is 1-D and the
// tiles are renumbered for the eight XCDs: workgroups are dispatched to the
// XCDs round-robin (workgroup b runs on XCD b % 8), so logical tile
// (b % 8) * per_xcd + b / 8 gives every XCD one contiguous band of tiles,
// processed in order.  Tiles that are neighbours in x then meet in the same
// L2, which serves the cache line the x-shifted planes share across a tile
// edge instead of fetching it twice from the fabric.
#include "kbc_launch.hpp"
#include "kbc_tile.hpp"

namespace kbc {

template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT, bool SLAB>
__global__ __launch_bounds__(256) void k_step(const typename Form<FORM>::S* __restrict__ src,
                                              typename Form<FORM>::S* __restrict__ dst, int nx,
                                              int ny, int64_t pitch, int ntx, int ntiles,
                                              int per_xcd, Coef<typename Form<FORM>::R> K,
                                              SlabHalo<typename Form<FORM>::S> halo) {
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    step_tile<FORM, COLL, VAR, GM, TXW, RPT, NT, SLAB>(src, dst, nx, ny, pitch, t % ntx, t / ntx, K, halo);
}

template <int FORM, int COLL, int VAR, int GM>
struct StepOp {
    template <int TXW, int RPT, bool NT, bool SLAB = false>
    static int go(const Lattice& L, const void* src, void* dst) {
        using F = Form<FORM>;
        using S = typename F::S;
        constexpr int TW = 64 * TXW, TH = (4 / TXW) * RPT;
        const int ntx = (L.nx + TW - 1) / TW;
        const int nty = (L.ny + TH - 1) / TH;
        const int64_t ntiles64 = static_cast<int64_t>(ntx) * nty;
        if (!grid_fits(8 * ((ntiles64 + 7) / 8), 256)) return kTooLarge;
        const int ntiles = static_cast<int>(ntiles64);
        const int per_xcd = (ntiles + 7) / 8;
        SlabHalo<S> halo;
        halo.lo = static_cast<const S*>(L.halo_lo);
        halo.hi = static_cast<const S*>(L.halo_hi);
        k_step<FORM, COLL, VAR, GM, TXW, RPT, NT, SLAB><<<dim3(8u * per_xcd), dim3(256), 0, L.stream>>>(
            static_cast<const S*>(src), static_cast<S*>(dst), L.nx, L.ny, L.pitch, ntx, ntiles, per_xcd,
            make_coef<typename F::R>(L), halo);
        return hipGetLastError() == hipSuccess ? 0 : -2;
    }
    template <bool NT>
    static int shape(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        switch (sh.width * 16 + sh.rpt) {
            case 64 * 16 + 1: return go<1, 1, NT>(L, src, dst);
            case 64 * 16 + 2: return go<1, 2, NT>(L, src, dst);
            case 64 * 16 + 4: return go<1, 4, NT>(L, src, dst);
            case 128 * 16 + 1: return go<2, 1, NT>(L, src, dst);
            case 128 * 16 + 2: return go<2, 2, NT>(L, src, dst);
            case 128 * 16 + 4: return go<2, 4, NT>(L, src, dst);
            case 256 * 16 + 1: return go<4, 1, NT>(L, src, dst);
            case 256 * 16 + 2: return go<4, 2, NT>(L, src, dst);
            case 256 * 16 + 4: return go<4, 4, NT>(L, src, dst);
            default: return -1;
        }
    }
    // a slab (halo rows from buffers) runs one of the three default tile
    // shapes: 256 x 4 (FP16), 256 x 1 (FP32) or 128 x 2 (FP64), the
    // requested one if it is among them
    template <bool NT>
    static int slab_shape(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        switch (sh.width * 16 + sh.rpt) {
            case 256 * 16 + 4: return go<4, 4, NT, true>(L, src, dst);
            case 128 * 16 + 2: return go<2, 2, NT, true>(L, src, dst);
            case 256 * 16 + 1: return go<4, 1, NT, true>(L, src, dst);
            default:
                return FORM == F16 ? go<4, 4, NT, true>(L, src, dst)
                                   : (FORM == F64 ? go<2, 2, NT, true>(L, src, dst) : go<4, 1, NT, true>(L, src, dst));
        }
    }
    static int run(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        if (L.halo_lo) return sh.nt ? slab_shape<true>(L, src, dst, sh) : slab_shape<false>(L, src, dst, sh);
        return sh.nt ? shape<true>(L, src, dst, sh) : shape<false>(L, src, dst, sh);
    }
};

bool valid_shape(const StepShape& s) {
    return (s.width == 64 || s.width == 128 || s.width == 256) && (s.rpt == 1 || s.rpt == 2 || s.rpt == 4) &&
           (s.nt == 0 || s.nt == 1);
}

int launch_step(const Lattice& L, const void* src, void* dst, const StepShape& shape) {
    if (!valid_shape(shape)) return -1;
    return dispatch<StepOp>(L, src, dst, shape);
}

const char* step_kernel_name(const Lattice& L) {
    static const char* forms[] = {"f16dev", "f32dev", "f64"};
    static const char* vars[] = {"A", "B", "C", "D"};
    static thread_local char buf[64];
    if (L.collision == LBGK)
        snprintf(buf, sizeof buf, "k_step<%s,LBGK>", forms[L.form]);
    else
        snprintf(buf, sizeof buf, "k_step<%s,KBC-%s>", forms[L.form], vars[L.variant]);
    return buf;
}

}  // namespace kbc
