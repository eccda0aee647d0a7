// kbc_tile.hpp -- one workgroup tile of the fused pull-stream + collide step,
// shared by the single-lattice step kernel and the ensemble kernel.
//
// Addressing: the nine plane bases are uniform (scalar registers); a node's
// loads and stores differ from them by byte offsets that fit in 32 bits when a
// plane is below 4 GiB, so the compiler can use the scalar-base + 32-bit vector
// offset form and skip per-access 64-bit address arithmetic.  Larger planes use
// the same code with 64-bit offsets.  NT selects non-temporal stores (the new
// state is not re-read before the next launch).
#pragma once

#include <type_traits>

#include "kbc_device.hpp"

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

// Tile (tx, ty) of a lattice: 64 * TXW nodes wide, (4 / TXW) * RPT rows tall,
// for the 256 threads of the calling workgroup.
template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT, bool WIDE>
__device__ __forceinline__ void step_tile(const typename Form<FORM>::S* __restrict__ src,
                                          typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                          int64_t pitch, int tx, int ty,
                                          const Coef<typename Form<FORM>::R>& K) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    using O = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    constexpr int TW = 64 * TXW;            // tile width
    constexpr int WR = 4 / TXW;             // wave rows per tile
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

}  // namespace kbc
