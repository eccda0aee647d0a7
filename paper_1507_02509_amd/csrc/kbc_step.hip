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
// Workgroup: 256 threads = 4 waves arranged as TXW waves side by side in x
// and 4 / TXW wave rows; each thread walks RPT consecutive rows, so a tile is
// 64 * TXW nodes wide and (4 / TXW) * RPT rows tall.  The grid is 1-D and the
// tiles are renumbered for the eight XCDs: workgroups are dispatched to the
// XCDs round-robin (workgroup b runs on XCD b % 8), so logical tile
// (b % 8) * per_xcd + b / 8 gives every XCD one contiguous band of tiles,
// processed in order.  Tiles that are neighbours in x then meet in the same
// L2, which serves the cache line the x-shifted planes share across a tile
// edge instead of fetching it twice from the fabric.
// Addressing: the nine plane bases are uniform (scalar registers); a node's
// loads and stores differ from them by byte offsets that fit in 32 bits when a
// plane is below 4 GiB, so the compiler can use the scalar-base + 32-bit vector
// offset form and skip per-access 64-bit address arithmetic.  Larger planes use
// the same code with 64-bit offsets.  NT selects non-temporal stores (the new
// state is not re-read before the next launch).
#include <type_traits>

#include "kbc_launch.hpp"

namespace kbc {

template <typename S, typename O>
__device__ __forceinline__ S ld_at(const S* base, O off) {
    return *reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + off);
}
template <typename S>
using gptr = __attribute__((address_space(1))) S*;

template <bool NT, typename S, typename O>
__device__ __forceinline__ void st_at(gptr<S> base, O off, S v) {
    gptr<S> p = reinterpret_cast<gptr<S>>(reinterpret_cast<__attribute__((address_space(1))) char*>(base) + off);
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// A global-memory pointer that is the same in every lane, kept in scalar
// registers.
template <typename S>
__device__ __forceinline__ gptr<S> uniform_ptr(S* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return reinterpret_cast<gptr<S>>((static_cast<uint64_t>(hi) << 32) | lo);
}

template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT, bool WIDE>
__global__ __launch_bounds__(256) void k_step(const typename Form<FORM>::S* __restrict__ src,
                                              typename Form<FORM>::S* __restrict__ dst, int nx,
                                              int ny, int64_t pitch, int ntx, int ntiles,
                                              int per_xcd, Coef<typename Form<FORM>::R> K) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    using O = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    constexpr int TW = 64 * TXW;            // tile width
    constexpr int WR = 4 / TXW;             // wave rows per tile
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    const int tx = t % ntx, ty = t / ntx;
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int x = tx * TW + lx;
    if (x >= nx) return;
    const int y0 = (ty * WR + ly) * RPT;
    const int64_t plane = static_cast<int64_t>(ny) * pitch;
    const O rowb = static_cast<O>(pitch) * static_cast<O>(sizeof(S));
    const O c0 = static_cast<O>(x) * sizeof(S);
    const O cm = static_cast<O>((x == 0) ? nx - 1 : x - 1) * sizeof(S);
    const O cp = static_cast<O>((x == nx - 1) ? 0 : x + 1) * sizeof(S);
    // plane bases of the destination, uniform across the workgroup
    const gptr<S> d0 = uniform_ptr(dst);
    const gptr<S> d1 = uniform_ptr(dst + plane);
    const gptr<S> d2 = uniform_ptr(dst + 2 * plane);
    const gptr<S> d3 = uniform_ptr(dst + 3 * plane);
    const gptr<S> d4 = uniform_ptr(dst + 4 * plane);
    const gptr<S> d5 = uniform_ptr(dst + 5 * plane);
    const gptr<S> d6 = uniform_ptr(dst + 6 * plane);
    const gptr<S> d7 = uniform_ptr(dst + 7 * plane);
    const gptr<S> d8 = uniform_ptr(dst + 8 * plane);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int y = y0 + r;
        if (y >= ny) return;
        const O r0 = static_cast<O>(y) * rowb;
        const O rm = static_cast<O>((y == 0) ? ny - 1 : y - 1) * rowb;
        const O rp = static_cast<O>((y == ny - 1) ? 0 : y + 1) * rowb;
        R g[9];
        g[0] = F::dec(ld_at(src, r0 + c0), 0);
        g[1] = F::dec(ld_at(src + plane, r0 + cm), 1);
        g[2] = F::dec(ld_at(src + 2 * plane, rm + c0), 2);
        g[3] = F::dec(ld_at(src + 3 * plane, r0 + cp), 3);
        g[4] = F::dec(ld_at(src + 4 * plane, rp + c0), 4);
        g[5] = F::dec(ld_at(src + 5 * plane, rm + cm), 5);
        g[6] = F::dec(ld_at(src + 6 * plane, rm + cp), 6);
        g[7] = F::dec(ld_at(src + 7 * plane, rp + cp), 7);
        g[8] = F::dec(ld_at(src + 8 * plane, rp + cm), 8);
        collide<R, COLL, VAR, GM>(g, K);
        const O o = r0 + c0;
        st_at<NT>(d0, o, F::enc(g[0], 0));
        st_at<NT>(d1, o, F::enc(g[1], 1));
        st_at<NT>(d2, o, F::enc(g[2], 2));
        st_at<NT>(d3, o, F::enc(g[3], 3));
        st_at<NT>(d4, o, F::enc(g[4], 4));
        st_at<NT>(d5, o, F::enc(g[5], 5));
        st_at<NT>(d6, o, F::enc(g[6], 6));
        st_at<NT>(d7, o, F::enc(g[7], 7));
        st_at<NT>(d8, o, F::enc(g[8], 8));
    }
}

template <int FORM, int COLL, int VAR, int GM>
struct StepOp {
    template <int TXW, int RPT, bool NT, bool WIDE>
    static int go(const Lattice& L, const void* src, void* dst) {
        using F = Form<FORM>;
        using S = typename F::S;
        constexpr int TW = 64 * TXW, TH = (4 / TXW) * RPT;
        const int ntx = (L.nx + TW - 1) / TW;
        const int nty = (L.ny + TH - 1) / TH;
        const int64_t ntiles64 = static_cast<int64_t>(ntx) * nty;
        if (ntiles64 > (int64_t{1} << 30)) return -1;
        const int ntiles = static_cast<int>(ntiles64);
        const int per_xcd = (ntiles + 7) / 8;
        k_step<FORM, COLL, VAR, GM, TXW, RPT, NT, WIDE><<<dim3(8u * per_xcd), dim3(256), 0, L.stream>>>(
            static_cast<const S*>(src), static_cast<S*>(dst), L.nx, L.ny, L.pitch, ntx, ntiles, per_xcd,
            make_coef<typename F::R>(L));
        return hipGetLastError() == hipSuccess ? 0 : -2;
    }
    template <bool NT, bool WIDE>
    static int shape(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        switch (sh.width * 16 + sh.rpt) {
            case 64 * 16 + 1: return go<1, 1, NT, WIDE>(L, src, dst);
            case 64 * 16 + 2: return go<1, 2, NT, WIDE>(L, src, dst);
            case 64 * 16 + 4: return go<1, 4, NT, WIDE>(L, src, dst);
            case 128 * 16 + 1: return go<2, 1, NT, WIDE>(L, src, dst);
            case 128 * 16 + 2: return go<2, 2, NT, WIDE>(L, src, dst);
            case 128 * 16 + 4: return go<2, 4, NT, WIDE>(L, src, dst);
            case 256 * 16 + 1: return go<4, 1, NT, WIDE>(L, src, dst);
            case 256 * 16 + 2: return go<4, 2, NT, WIDE>(L, src, dst);
            case 256 * 16 + 4: return go<4, 4, NT, WIDE>(L, src, dst);
            default: return -1;
        }
    }
    static int run(const Lattice& L, const void* src, void* dst, const StepShape& sh) {
        // 32-bit byte offsets need every in-plane offset below 2^32
        const uint64_t plane_bytes = static_cast<uint64_t>(L.ny) * static_cast<uint64_t>(L.pitch) *
                                     sizeof(typename Form<FORM>::S);
        const bool wide = plane_bytes > (uint64_t{1} << 32);
        if (sh.nt) return wide ? shape<true, true>(L, src, dst, sh) : shape<true, false>(L, src, dst, sh);
        return wide ? shape<false, true>(L, src, dst, sh) : shape<false, false>(L, src, dst, sh);
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
