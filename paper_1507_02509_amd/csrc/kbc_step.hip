// kbc_step.hip -- fused pull-stream + collide step for gfx950.
//
// Layout: 9 planes of ny rows of `pitch` elements (x fastest), deviations
// g_i = f_i - W_i rho0 in the storage form.  A node gathers plane i from
// x - v_i (eq. Egeneral read right to left: the populations that stream into x
// this step left their source node after the previous collision), collides,
// and writes all nine values at x.  Every stored element is read exactly once
// per step (the pull is a bijection per plane), so HBM traffic is 9 loads and
// 9 stores per node.  Loads of the six planes with v_x != 0 are shifted by one
// element; the wave's 64 lanes still cover one contiguous 64-element run, so
// the extra cache line per run is shared with the neighbouring wave through
// L2.  Vertical shifts are whole rows.
//
// Workgroup: 256 threads = 4 waves; a wave covers 64 consecutive x of one row
// and walks `RPT` consecutive rows.  blockIdx.x runs over x tiles fastest so
// that the workgroups a dispatch round places on one XCD cover neighbouring
// tiles of the same rows.
#include "kbc_launch.hpp"

namespace kbc {

template <int FORM, int COLL, int VAR, int GM, int RPT>
__global__ __launch_bounds__(256) void k_step(const typename Form<FORM>::S* __restrict__ src,
                                              typename Form<FORM>::S* __restrict__ dst, int nx,
                                              int ny, int64_t pitch,
                                              Coef<typename Form<FORM>::R> K) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    const int x = blockIdx.x * 64 + threadIdx.x;
    if (x >= nx) return;
    const int y0 = (blockIdx.y * 4 + threadIdx.y) * RPT;
    const int64_t plane = static_cast<int64_t>(ny) * pitch;
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int y = y0 + r;
        if (y >= ny) return;
        const int ym = (y == 0) ? ny - 1 : y - 1;
        const int yp = (y == ny - 1) ? 0 : y + 1;
        const S* r0 = src + static_cast<int64_t>(y) * pitch;
        const S* rm = src + static_cast<int64_t>(ym) * pitch;
        const S* rp = src + static_cast<int64_t>(yp) * pitch;
        R g[9];
        g[0] = F::dec(r0[x], 0);
        g[1] = F::dec(r0[plane + xm], 1);
        g[2] = F::dec(rm[2 * plane + x], 2);
        g[3] = F::dec(r0[3 * plane + xp], 3);
        g[4] = F::dec(rp[4 * plane + x], 4);
        g[5] = F::dec(rm[5 * plane + xm], 5);
        g[6] = F::dec(rm[6 * plane + xp], 6);
        g[7] = F::dec(rp[7 * plane + xp], 7);
        g[8] = F::dec(rp[8 * plane + xm], 8);
        collide<R, COLL, VAR, GM>(g, K);
        S* o = dst + static_cast<int64_t>(y) * pitch + x;
#pragma unroll
        for (int i = 0; i < 9; ++i) o[i * plane] = F::enc(g[i], i);
    }
}

template <int FORM, int COLL, int VAR, int GM>
struct StepOp {
    static int run(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        using F = Form<FORM>;
        using S = typename F::S;
        const auto K = make_coef<typename F::R>(L);
        const dim3 block(64, 4);
        const int rpt = sh.rows / 4;
        const unsigned gx = static_cast<unsigned>((L.nx + 63) / 64);
        const unsigned gy = static_cast<unsigned>((L.ny + sh.rows - 1) / sh.rows);
        const dim3 grid(gx, gy);
        const S* s = static_cast<const S*>(src);
        S* d = static_cast<S*>(dst);
        switch (rpt) {
            case 1: k_step<FORM, COLL, VAR, GM, 1><<<grid, block, 0, L.stream>>>(s, d, L.nx, L.ny, L.pitch, K); break;
            case 2: k_step<FORM, COLL, VAR, GM, 2><<<grid, block, 0, L.stream>>>(s, d, L.nx, L.ny, L.pitch, K); break;
            case 4: k_step<FORM, COLL, VAR, GM, 4><<<grid, block, 0, L.stream>>>(s, d, L.nx, L.ny, L.pitch, K); break;
            default: return -1;
        }
        return hipGetLastError() == hipSuccess ? 0 : -2;
    }
};

int launch_step(const Lattice& L, const void* src, void* dst, const StepShape& shape) {
    if (shape.rows != 4 && shape.rows != 8 && shape.rows != 16) return -1;
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
