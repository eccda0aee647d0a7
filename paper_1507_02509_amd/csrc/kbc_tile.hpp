// kbc_tile.hpp -- one workgroup tile of the fused pull-stream + collide step,
// shared by the single-lattice step kernel and the ensemble kernel.
//
// Addressing: row bases are uniform (scalar registers) and a lane adds a
// 32-bit byte offset within the row, so loads and stores use the scalar-base +
// vector-offset form with no per-access 64-bit address arithmetic, for any
// lattice size.  NT selects non-temporal stores (the new state is not re-read
// before the next launch).
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

// A lane's 32-bit byte offset, made opaque where it is used: left alone, the
// compiler hoists its widening to 64 bits out of the row loops, after which
// base + offset no longer matches the scalar-base + 32-bit-offset address
// form and every access pays a 64-bit vector add.  The empty statement emits
// no instruction.
__device__ __forceinline__ uint32_t lane_off(uint32_t off) {
    asm("" : "+v"(off));
    return off;
}

template <bool NT, typename S>
__device__ __forceinline__ void st_at(gptr<S> base, uint32_t off, S v) {
    gptr<S> p = reinterpret_cast<gptr<S>>(reinterpret_cast<__attribute__((address_space(1))) char*>(base) +
                                          lane_off(off));
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

// Pointer to population i of row y: the state is laid out [ny][9][pitch],
// element (i, y, x) at (9 y + i) * pitch + x.  With y uniform across the
// wave this is a scalar base.
template <typename S>
__device__ __forceinline__ gptr<S> row_ptr(S* base, int y, int i, int64_t pitch) {
    return uniform_ptr(base + (static_cast<int64_t>(y) * 9 + i) * pitch);
}
template <typename S>
__device__ __forceinline__ gptr<const S> row_ptr(const S* base, int y, int i, int64_t pitch) {
    return uniform_ptr(base + (static_cast<int64_t>(y) * 9 + i) * pitch);
}

template <typename S>
__device__ __forceinline__ S ld_at(gptr<const S> base, uint32_t off) {
    return *reinterpret_cast<gptr<const S>>(reinterpret_cast<__attribute__((address_space(1))) const char*>(base) +
                                            lane_off(off));
}

// Tile (tx, ty) of a lattice: 64 * TXW nodes wide, (4 / TXW) * RPT rows tall,
// for the 256 threads of the calling workgroup.  Every wave covers 64
// consecutive nodes of one row, so the row index is uniform across the wave:
// the nine source rows (three y values, nine populations) and nine destination
// rows are scalar bases, and a lane's loads and stores differ from them only
// by the 32-bit byte offsets of x - 1, x and x + 1.
template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT>
__device__ __forceinline__ void step_tile(const typename Form<FORM>::S* __restrict__ src,
                                          typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                          int64_t pitch, int tx, int ty,
                                          const Coef<typename Form<FORM>::R>& K) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    constexpr int TW = 64 * TXW;            // tile width
    constexpr int WR = 4 / TXW;             // wave rows per tile
    const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
    const int x = tx * TW + lx;
    if (x >= nx) return;
    const int y0 = __builtin_amdgcn_readfirstlane((ty * WR + ly) * RPT);
    const uint32_t c0 = static_cast<uint32_t>(x) * sizeof(S);
    const uint32_t cm = static_cast<uint32_t>((x == 0) ? nx - 1 : x - 1) * sizeof(S);
    const uint32_t cp = static_cast<uint32_t>((x == nx - 1) ? 0 : x + 1) * sizeof(S);
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int y = y0 + r;
        if (y >= ny) return;
        const int ym = (y == 0) ? ny - 1 : y - 1;
        const int yp = (y == ny - 1) ? 0 : y + 1;
        R g[9];
        g[0] = F::dec(ld_at(row_ptr(src, y, 0, pitch), c0), 0);
        g[1] = F::dec(ld_at(row_ptr(src, y, 1, pitch), cm), 1);
        g[2] = F::dec(ld_at(row_ptr(src, ym, 2, pitch), c0), 2);
        g[3] = F::dec(ld_at(row_ptr(src, y, 3, pitch), cp), 3);
        g[4] = F::dec(ld_at(row_ptr(src, yp, 4, pitch), c0), 4);
        g[5] = F::dec(ld_at(row_ptr(src, ym, 5, pitch), cm), 5);
        g[6] = F::dec(ld_at(row_ptr(src, ym, 6, pitch), cp), 6);
        g[7] = F::dec(ld_at(row_ptr(src, yp, 7, pitch), cp), 7);
        g[8] = F::dec(ld_at(row_ptr(src, yp, 8, pitch), cm), 8);
        collide<R, COLL, VAR, GM>(g, K);
#pragma unroll
        for (int i = 0; i < 9; ++i) st_at<NT>(row_ptr(dst, y, i, pitch), c0, F::enc(g[i], i));
    }
}

}  // namespace kbc
