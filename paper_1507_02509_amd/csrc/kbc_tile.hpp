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

// A slab is a lattice that is one piece of a domain split in y (one piece
// per GPU): it is periodic in x, and its rows -2, -1 and ny, ny + 1 are not
// its own rows wrapped but the neighbouring pieces' edge rows, kept in two
// caller-owned halo buffers laid out [2][9][pitch] like the state (`lo`: rows
// -2, -1; `hi`: rows ny, ny + 1).  Null pointers for a periodic lattice.
template <typename S>
struct SlabHalo {
    const S* lo = nullptr;
    const S* hi = nullptr;
};

// Population-i row y (uniform, -2 <= y <= ny + 1) of a slab's state.
template <typename S>
__device__ __forceinline__ gptr<const S> slab_row(const S* base, const SlabHalo<S>& h, int y, int i, int ny,
                                                  int64_t pitch) {
    const S* b = base;
    int r = y;
    if (y < 0) {
        b = h.lo;
        r = y + 2;
    } else if (y >= ny) {
        b = h.hi;
        r = y - ny;
    }
    return row_ptr(b, r, i, pitch);
}

// Tile (tx, ty) of a lattice: 64 * TXW nodes wide, (4 / TXW) * RPT rows tall,
// for the 256 threads of the calling workgroup.  Every wave covers 64
// consecutive nodes of one row, so the row index is uniform across the wave:
// the nine source rows (three y values, nine populations) and nine destination
// rows are scalar bases, and a lane's loads and stores differ from them only
// by the 32-bit byte offsets of x - 1, x and x + 1.  SLAB: rows -1 and ny
// come from the halo buffers instead of wrapping.
template <int FORM, int COLL, int VAR, int GM, int TXW, int RPT, bool NT, bool SLAB = false>
__device__ __forceinline__ void step_tile(const typename Form<FORM>::S* __restrict__ src,
                                          typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                          int64_t pitch, int tx, int ty,
                                          const Coef<typename Form<FORM>::R>& K,
                                          const SlabHalo<typename Form<FORM>::S>& halo = {}) {
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
        const int ym = SLAB ? y - 1 : ((y == 0) ? ny - 1 : y - 1);
        const int yp = SLAB ? y + 1 : ((y == ny - 1) ? 0 : y + 1);
        auto in = [&](int yy, int i) {
            if constexpr (SLAB)
                return slab_row(src, halo, yy, i, ny, pitch);
            else
                return row_ptr(src, yy, i, pitch);
        };
        R g[9];
        g[0] = F::dec(ld_at(in(y, 0), c0), 0);
        g[1] = F::dec(ld_at(in(y, 1), cm), 1);
        g[2] = F::dec(ld_at(in(ym, 2), c0), 2);
        g[3] = F::dec(ld_at(in(y, 3), cp), 3);
        g[4] = F::dec(ld_at(in(yp, 4), c0), 4);
        g[5] = F::dec(ld_at(in(ym, 5), cm), 5);
        g[6] = F::dec(ld_at(in(ym, 6), cp), 6);
        g[7] = F::dec(ld_at(in(yp, 7), cp), 7);
        g[8] = F::dec(ld_at(in(yp, 8), cm), 8);
        collide<R, COLL, VAR, GM>(g, K);
#pragma unroll
        for (int i = 0; i < 9; ++i) st_at<NT>(row_ptr(dst, y, i, pitch), c0, F::enc(g[i], i));
    }
}

}  // namespace kbc
