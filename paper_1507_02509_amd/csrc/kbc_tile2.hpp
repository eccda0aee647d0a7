// kbc_tile2.hpp -- two fused time steps on one workgroup tile (temporal
// blocking), shared by the single-lattice fused kernel and the ensemble.
//
// A workgroup owns an output tile of 64 x TH nodes (TH = 8, 16, 24 or 32;
// the larger ones only where the LDS tile fits a CU).  Step 1 runs on the
// tile extended by one node on every side (66 x (TH + 2) nodes, periodic):
// each node gathers its populations from the state buffer exactly as the
// single step does (f_i at x - v_i) and collides.  It then pushes each
// post-collision value, in the storage form, to where step 2 will read it:
// population i of node e goes to slot e + v_i of population i's window, which
// covers the 64 x TH output nodes plus one padding column on each side (a
// value whose slot falls outside the window is not needed and not written).
// Step 2 then reads, for every output node x, population i from slot x of
// window i, collides and writes the result to the destination buffer.  The
// windows take 9 x TH x 66 values of LDS instead of the extended tile's
// 9 x (TH + 2) x 66 (FP32, TH = 16: 38.0 KB, four workgroups per CU instead
// of three), and step 2's LDS reads are unshifted.  HBM traffic is the
// single step's 18 values per node for two steps; the ring of extra step-1
// collisions costs (66 (TH + 2)) / (64 TH) - 1 more arithmetic (16 % for
// TH = 16, 8 % for TH = 32).  The values that pass through LDS are rounded to
// the storage form exactly as the single step rounds them on the way to HBM,
// and both steps run the same collision code, so two fused steps are bitwise
// identical to two single steps.
//
// Work split: the 64 interior columns of every extended row are one wave
// (lane = column), so the row is uniform across the wave, its bases are
// scalar, as in the single step, and whether a population's slot row lies in
// the window is a scalar branch; the rows go to the four waves round-robin.
// The two halo columns (2 (TH + 2) nodes) go to the lanes of wave 3 (one
// pass, two for TH = 32), with per-lane addressing.
#pragma once

#include "kbc_tile.hpp"

namespace kbc {

__device__ __forceinline__ int pmod(int v, int n) {
    const int r = v % n;
    return r < 0 ? r + n : r;
}

// v mod n for a wave-uniform v within a few periods of [0, n): scalar loops
// instead of an integer division
__device__ __forceinline__ int wrap_uniform(int v, int n) {
    while (v < 0) v += n;
    while (v >= n) v -= n;
    return v;
}

// v mod n for v in [-1, n]
__device__ __forceinline__ int wrap1(int v, int n) {
    v = (v < 0) ? v + n : v;
    return (v >= n) ? v - n : v;
}

// Two fused steps on the output tile with corner (x0, y0), for the 256
// threads of the calling workgroup (all of which must call it: it holds a
// workgroup barrier).  SLAB: the rows beyond the slab's edges, -2, -1 and
// ny, ny + 1, come from the halo buffers (SlabHalo) instead of wrapping;
// extended rows past row ny (a ragged last tile) only feed output rows the
// tile does not store, and load row ny instead.
template <int FORM, int COLL, int VAR, int GM, int TH, bool NT, bool SLAB = false>
__device__ __forceinline__ void step2_tile(const typename Form<FORM>::S* __restrict__ src,
                                           typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                           int64_t pitch, int x0, int y0, const Coef<typename Form<FORM>::R>& K,
                                           const SlabHalo<typename Form<FORM>::S>& halo = {}) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    constexpr int TW = 64, EW = TW + 2, EH = TH + 2;
    __shared__ S win[9][TH][EW];   // slot (row r, column c) holds output node (c - 1, r)

    const int lane = static_cast<int>(threadIdx.x & 63u);
    const int w = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x >> 6));   // wave index

    // ---- step 1, interior columns x0 .. x0 + 63 (wrapped), extended rows
    // (every fourth for each wave); the next row's loads are issued before
    // the current row collides, into the other of two register sets (the
    // loop is unrolled by two rows so that no row is copied between them)
    {
        const int gx = pmod(x0 + lane, nx);
        const uint32_t c0 = static_cast<uint32_t>(gx) * sizeof(S);
        const uint32_t cm = static_cast<uint32_t>(gx == 0 ? nx - 1 : gx - 1) * sizeof(S);
        const uint32_t cp = static_cast<uint32_t>(gx == nx - 1 ? 0 : gx + 1) * sizeof(S);
        auto load_row = [&](int ey, S (&v)[9]) {
            int y, ym, yp;
            if constexpr (SLAB) {
                y = y0 - 1 + ey < ny ? y0 - 1 + ey : ny;
                ym = y - 1;
                yp = y + 1;
            } else {
                y = wrap_uniform(y0 - 1 + ey, ny);
                ym = (y == 0) ? ny - 1 : y - 1;
                yp = (y == ny - 1) ? 0 : y + 1;
            }
            auto in = [&](int yy, int i) {
                if constexpr (SLAB)
                    return slab_row(src, halo, yy, i, ny, pitch);
                else
                    return row_ptr(src, yy, i, pitch);
            };
            v[0] = ld_at(in(y, 0), c0);
            v[1] = ld_at(in(y, 1), cm);
            v[2] = ld_at(in(ym, 2), c0);
            v[3] = ld_at(in(y, 3), cp);
            v[4] = ld_at(in(yp, 4), c0);
            v[5] = ld_at(in(ym, 5), cm);
            v[6] = ld_at(in(ym, 6), cp);
            v[7] = ld_at(in(yp, 7), cp);
            v[8] = ld_at(in(yp, 8), cm);
        };
        auto row = [&](int ey, const S (&v)[9]) {
            R g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = F::dec(v[i], i);
            collide<R, COLL, VAR, GM>(g, K);
            // node (lane, ey - 1) -> slot (lane + v_x + 1, ey - 1 + v_y); the row test is uniform
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const int r = ey - 1 + kCy[i];
                if (r >= 0 && r < TH) win[i][r][lane + 1 + kCx[i]] = F::enc(g[i], i);
            }
        };
        // steady state: both prefetches exist, so the wait before each row
        // covers only that row's loads (a conditional prefetch makes the
        // compiler wait for all outstanding loads); the last one or two rows
        // are peeled off
        S va[9], vb[9];
        load_row(w, va);
        int ey = w;
        for (; ey + 8 < EH; ey += 8) {
            load_row(ey + 4, vb);
            row(ey, va);
            load_row(ey + 8, va);
            row(ey + 4, vb);
        }
        if (ey + 4 < EH) {
            load_row(ey + 4, vb);
            row(ey, va);
            row(ey + 4, vb);
        } else if (ey < EH) {
            row(ey, va);
        }
    }
    // ---- step 1, halo columns x0 - 1 and x0 + 64 (wrapped), every extended
    // row: 2 (TH + 2) nodes for the lanes of wave 3
    if (w == 3) {
        for (int k = lane; k < 2 * EH; k += 64) {
            const int side = k / EH;
            const int ey = k - side * EH;
            const int gx = pmod(side ? x0 + TW : x0 - 1, nx);
            R g[9];
            if constexpr (SLAB) {
                const int y = y0 - 1 + ey < ny ? y0 - 1 + ey : ny;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int xs = wrap1(gx - kCx[i], nx), ys = y - kCy[i];
                    const S* b = ys < 0 ? halo.lo : (ys >= ny ? halo.hi : src);
                    const int r = ys < 0 ? ys + 2 : (ys >= ny ? ys - ny : ys);
                    g[i] = F::dec(b[(static_cast<int64_t>(r) * 9 + i) * pitch + xs], i);
                }
            } else {
                const int y = pmod(y0 - 1 + ey, ny);
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const int xs = wrap1(gx - kCx[i], nx), ys = wrap1(y - kCy[i], ny);
                    g[i] = F::dec(src[(static_cast<int64_t>(ys) * 9 + i) * pitch + xs], i);
                }
            }
            collide<R, COLL, VAR, GM>(g, K);
            // node (-1 or 64, ey - 1): only the populations that move into
            // the tile land in a column the output nodes read
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                if (kCx[i] != (side ? -1 : 1)) continue;
                const int r = ey - 1 + kCy[i];
                if (r >= 0 && r < TH) win[i][r][side ? EW - 2 : 1] = F::enc(g[i], i);
            }
        }
    }
    __syncthreads();

    // ---- step 2 on the output tile, populations gathered from LDS
    const int gx = x0 + lane;
    const uint32_t c0 = static_cast<uint32_t>(gx) * sizeof(S);
    for (int oy = w; oy < TH; oy += 4) {
        const int y = y0 + oy;
        if (y >= ny) break;
        if (gx < nx) {
            R g[9];
#pragma unroll
            for (int i = 0; i < 9; ++i) g[i] = F::dec(win[i][oy][lane + 1], i);
            collide<R, COLL, VAR, GM>(g, K);
#pragma unroll
            for (int i = 0; i < 9; ++i) st_at<NT>(row_ptr(dst, y, i, pitch), c0, F::enc(g[i], i));
        }
    }
}

}  // namespace kbc
