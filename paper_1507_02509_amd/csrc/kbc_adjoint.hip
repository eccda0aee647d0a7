// kbc_adjoint.hip -- discrete adjoint of the lattice step and of the initial
// state, for gradients of a final-time loss with respect to the initial
// velocity field and beta.
//
// With pull storage the forward step is f^{n+1}_i(x + v_i) = C_i(f^n(x)).
// The adjoint of a loss L(f^N) therefore obeys
//   lam^n_j(x) = sum_i lam^{n+1}_i(x + v_i) dC_i/df_j (f^n(x)),
//   dL/dbeta  += sum_x sum_i lam^{n+1}_i(x + v_i) dC_i/dbeta (f^n(x)).
// An adjoint step reads f^n (nine shifted loads from the state buffer, as the
// forward step does), mu_i(x) = lam^{n+1}_i(x + v_i) (nine loads shifted the
// other way) and writes lam^n at x: 27 accesses per node.  Adjoint fields are
// stored like the state, [ny][9][pitch], in the form's arithmetic type,
// unshifted.
#include <type_traits>

#include "kbc_adjoint.hpp"
#include "kbc_launch.hpp"
#include "kbc_tile.hpp"

namespace kbc {

namespace {

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of one double per thread over the 256-thread block (fixed order).
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[4];
    const double s = wave_sum_d(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// ----------------------------------------------------------------- loss seed
// lam_i(x) = dL/drho + (dL/du_x (c_xi - u_x) + dL/du_y (c_yi - u_y)) / rho
template <int FORM>
__global__ __launch_bounds__(256) void k_adj_seed(const typename Form<FORM>::S* __restrict__ state, int nx,
                                                  int ny, int64_t pitch, double rho0,
                                                  const double* __restrict__ drho,
                                                  const double* __restrict__ dux,
                                                  const double* __restrict__ duy,
                                                  typename Form<FORM>::R* __restrict__ lam) {
    using F = Form<FORM>;
    using R = typename F::R;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    double dr = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int xs = wrapi(x - kCx[i], nx), ys = wrapi(y - kCy[i], ny);
        const double g = F::dec64(state[(static_cast<int64_t>(ys) * 9 + i) * pitch + xs], i);
        dr += g;
        jx += kCx[i] * g;
        jy += kCy[i] * g;
    }
    const double r = rho0 + dr, u = jx / r, v = jy / r;
    const int64_t n = static_cast<int64_t>(y) * nx + x;
    const double a = drho ? drho[n] : 0.0;
    const double bx = dux ? dux[n] : 0.0, by = duy ? duy[n] : 0.0;
    R* o = lam + static_cast<int64_t>(y) * 9 * pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        o[i * pitch] = static_cast<R>(a + (bx * (kCx[i] - u) + by * (kCy[i] - v)) / r);
}

// ----------------------------------------------------------------- adjoint step
// Grid: one workgroup per tile of 128 x (2 RPT) nodes, 8 * rpx * ntx workgroups
// (workgroup b runs on XCD b % 8).  XCD x owns the rpx tile rows from x * rpx
// on; its workgroups, which the hardware dispatches in order, take that band's
// tiles strip by strip (vertical strips of at most kAdjStrip tiles) and
// row-major within a strip.  The resident workgroups then form a compact front
// a few strip rows deep, and a cache line that two vertically adjacent tiles
// share is used again one strip row (under 1 MB of traffic) after its first
// use, while it is still in the XCD's 4 MB L2; with whole-width rows on a
// large lattice that distance is about the L2 size and a fifth of the reads
// miss.  Workgroups left over in a short last band do nothing but write a zero
// partial.  Each workgroup sums its nodes' dL/dbeta terms in a fixed order
// into partials[b]; on large lattices k_fold shortens that array first, and
// k_sum_partials adds it up in a fixed order (no device-scope fence per workgroup: on this GPU such a fence writes
// back the whole L2 of the XCD).
constexpr int kAdjStrip = 32;
// Tile height: 128 x 4 with two nodes per thread (rows r and r + 2) for the
// FP32 and FP16 forms where the lattice has at least kAdjTwoRowTiles such
// tiles, which halves the per-node share of the tile mapping and the
// workgroup reduction (measured 2-3 % on 16384^2); 128 x 2 with one node per
// thread otherwise: smaller lattices are latency-bound and need the
// workgroups (512^2 rollouts ran 1.5 % slower with two rows), and FP64 would
// drop to two waves per SIMD (206 VGPRs).
constexpr int64_t kAdjTwoRowTiles = 8192;
inline int adj_rows_per_thread(const Lattice& L) {
    const int64_t tiles4 = static_cast<int64_t>((L.nx + 127) / 128) * ((L.ny + 3) / 4);
    return (L.form != F64 && tiles4 >= kAdjTwoRowTiles) ? 2 : 1;
}
constexpr int kFold = 2048;   // partials per k_fold workgroup

// The adjoint step of workgroup index bidx (the 256 threads of the calling
// workgroup must all call it: it holds a workgroup barrier).  SLAB: rows -1
// and ny of the state and of the incoming adjoint come from halo buffers
// (SlabHalo, kbc_tile.hpp) instead of wrapping.
template <int FORM, int COLL, int VAR, int GM, bool FROZEN, int RPT, bool SLAB = false>
__device__ __forceinline__ void adj_tile(const typename Form<FORM>::S* __restrict__ state,
                                         const typename Form<FORM>::R* __restrict__ lin,
                                         typename Form<FORM>::R* __restrict__ lout, int nx, int ny,
                                         int64_t pitch, int ntx, int nty, const Coef<typename Form<FORM>::R>& K,
                                         double* __restrict__ partials, unsigned bidx,
                                         const SlabHalo<typename Form<FORM>::S>& sh = {},
                                         const SlabHalo<typename Form<FORM>::R>& lh = {}) {
    using F = Form<FORM>;
    using R = typename F::R;
    using S = typename F::S;
    constexpr int TW = 128, WR = 2 * RPT;
    const int xcd = static_cast<int>(bidx & 7u), u = static_cast<int>(bidx >> 3);
    const int rpx = (nty + 7) >> 3;                            // tile rows per XCD
    const int row0 = xcd * rpx;
    const int rows = (nty - row0 < rpx) ? (nty - row0 > 0 ? nty - row0 : 0) : rpx;
    const int sw = (ntx < kAdjStrip) ? ntx : kAdjStrip;        // strip width in tiles
    const int full = (ntx / sw) * sw * rows;                   // tiles in full-width strips
    const int rw = ntx % sw;                                   // width of the last, narrow strip
    int col = 0, row = 0;
    if (u < full) {
        const int s0 = u / (sw * rows), v = u - s0 * (sw * rows);
        row = v / sw;
        col = s0 * sw + (v - row * sw);
    } else if (u < ntx * rows) {
        const int v = u - full;
        row = v / rw;
        col = full / rows + (v - row * rw);
    }
    row += row0;
    const int x = col * TW + static_cast<int>(threadIdx.x % TW);
    // the wave's first row (a wave covers 64 nodes of one row), then, with two
    // rows per thread, that row + 2
    const int ya = __builtin_amdgcn_readfirstlane(row * WR + static_cast<int>(threadIdx.x / TW));
    const int yb = ya + 2;
    double db = 0.0;
    if (u < ntx * rows && x < nx && ya < ny) {
        const uint32_t xm = static_cast<uint32_t>((x == 0) ? nx - 1 : x - 1);
        const uint32_t xp = static_cast<uint32_t>((x == nx - 1) ? 0 : x + 1);
        const uint32_t sS = sizeof(S), sR = sizeof(R);
        const uint32_t x0 = static_cast<uint32_t>(x);
        auto load = [&](int yu, R (&g)[9], R (&mu)[9]) {
            const int ym = SLAB ? yu - 1 : ((yu == 0) ? ny - 1 : yu - 1);
            const int yp = SLAB ? yu + 1 : ((yu == ny - 1) ? 0 : yu + 1);
            auto st = [&](int yy, int i) {
                if constexpr (SLAB)
                    return slab_row(state, sh, yy, i, ny, pitch);
                else
                    return row_ptr(state, yy, i, pitch);
            };
            auto la = [&](int yy, int i) {
                if constexpr (SLAB)
                    return slab_row(lin, lh, yy, i, ny, pitch);
                else
                    return row_ptr(lin, yy, i, pitch);
            };
            // f^n_i(x) sits at x - v_i
            g[0] = F::dec(ld_at(st(yu, 0), x0 * sS), 0);
            g[1] = F::dec(ld_at(st(yu, 1), xm * sS), 1);
            g[2] = F::dec(ld_at(st(ym, 2), x0 * sS), 2);
            g[3] = F::dec(ld_at(st(yu, 3), xp * sS), 3);
            g[4] = F::dec(ld_at(st(yp, 4), x0 * sS), 4);
            g[5] = F::dec(ld_at(st(ym, 5), xm * sS), 5);
            g[6] = F::dec(ld_at(st(ym, 6), xp * sS), 6);
            g[7] = F::dec(ld_at(st(yp, 7), xp * sS), 7);
            g[8] = F::dec(ld_at(st(yp, 8), xm * sS), 8);
            // mu_i(x) = lam^{n+1}_i(x + v_i)
            mu[0] = ld_at(la(yu, 0), x0 * sR);
            mu[1] = ld_at(la(yu, 1), xp * sR);
            mu[2] = ld_at(la(yp, 2), x0 * sR);
            mu[3] = ld_at(la(yu, 3), xm * sR);
            mu[4] = ld_at(la(ym, 4), x0 * sR);
            mu[5] = ld_at(la(yp, 5), xp * sR);
            mu[6] = ld_at(la(yp, 6), xm * sR);
            mu[7] = ld_at(la(ym, 7), xm * sR);
            mu[8] = ld_at(la(ym, 8), xp * sR);
        };
        auto finish = [&](int yu, const R (&g)[9], const R (&mu)[9]) {
            R lam[9], dbn;
            collide_vjp<R, COLL, VAR, GM, FROZEN>(g, mu, K, lam, dbn);
#pragma unroll
            for (int i = 0; i < 9; ++i) st_at<false>(row_ptr(lout, yu, i, pitch), x0 * sR, lam[i]);
            db += static_cast<double>(dbn);
        };
        R ga[9], ma[9];
        if (RPT == 2 && yb < ny) {
            // both rows: the second row's loads are in flight while the first is differentiated
            R gb[9], mb[9];
            load(ya, ga, ma);
            load(yb, gb, mb);
            finish(ya, ga, ma);
            finish(yb, gb, mb);
        } else {
            load(ya, ga, ma);
            finish(ya, ga, ma);
        }
    }
    const double s = block_sum(db);
    if (threadIdx.x == 0) partials[bidx] = s;
}

template <int FORM, int COLL, int VAR, int GM, bool FROZEN, int RPT, bool SLAB>
__global__ __launch_bounds__(256) void k_adj_step(const typename Form<FORM>::S* __restrict__ state,
                                                  const typename Form<FORM>::R* __restrict__ lin,
                                                  typename Form<FORM>::R* __restrict__ lout, int nx,
                                                  int ny, int64_t pitch, int ntx, int nty,
                                                  Coef<typename Form<FORM>::R> K,
                                                  double* __restrict__ partials,
                                                  SlabHalo<typename Form<FORM>::S> sh,
                                                  SlabHalo<typename Form<FORM>::R> lh) {
    adj_tile<FORM, COLL, VAR, GM, FROZEN, RPT, SLAB>(state, lin, lout, nx, ny, pitch, ntx, nty, K, partials,
                                                     blockIdx.x, sh, lh);
}

// An adjoint step and, in the same grid, one forward step between two other
// state buffers (src -> dst): the backward pass of a checkpointed rollout
// recomputes the next segment's states this way, inside the launches of the
// current segment's adjoint steps, so that the two fill the chip together on
// lattices too small to fill it alone.  Workgroups below nadj (a multiple of
// 8, so both parts keep their XCD banding) run the adjoint tile, the others
// the forward step's 256 x 1 tiles (the per-node code of every tile shape is
// the same, so the recomputed states are those of any forward step).
template <int FORM, int COLL, int VAR, int GM, bool FROZEN, int RPT>
__global__ __launch_bounds__(256) void k_adj_step_fwd(const typename Form<FORM>::S* __restrict__ state,
                                                      const typename Form<FORM>::R* __restrict__ lin,
                                                      typename Form<FORM>::R* __restrict__ lout, int nx,
                                                      int ny, int64_t pitch, int ntx, int nty,
                                                      Coef<typename Form<FORM>::R> K,
                                                      double* __restrict__ partials, unsigned nadj,
                                                      const typename Form<FORM>::S* __restrict__ src,
                                                      typename Form<FORM>::S* __restrict__ dst, int ntx_f,
                                                      int ntiles_f, int per_xcd_f) {
    if (blockIdx.x < nadj) {
        adj_tile<FORM, COLL, VAR, GM, FROZEN, RPT>(state, lin, lout, nx, ny, pitch, ntx, nty, K, partials,
                                                   blockIdx.x);
        return;
    }
    const int b = static_cast<int>(blockIdx.x - nadj);
    const int t = (b & 7) * per_xcd_f + (b >> 3);
    if (t >= ntiles_f) return;
    step_tile<FORM, COLL, VAR, GM, 4, 1, false>(src, dst, nx, ny, pitch, t % ntx_f, t / ntx_f, K);
}

// out[g] = sum of partials[g * kFold .. (g + 1) * kFold), in a fixed order
__global__ __launch_bounds__(256) void k_fold(const double* __restrict__ partials, int64_t n,
                                              double* __restrict__ out) {
    const int64_t lo = static_cast<int64_t>(blockIdx.x) * kFold;
    const int64_t hi = (lo + kFold < n) ? lo + kFold : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += partials[i];
    const double t = block_sum(s);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// acc[0] += sum of n partials, in a fixed order
__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int64_t n,
                                                      double* __restrict__ acc) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += partials[i];
    const double t = block_sum(s);
    if (threadIdx.x == 0) acc[0] += t;
}

// ------------------------------------------------------- adjoint of the initial state
// f0_i - W_i rho0 = W_i [ (rho - rho0) + 3 rho (v.u)
//                         + 4.5 ( rho (v.u)^2 - rho |u|^2 / 3 + Pi1 : v v - tr(Pi1) / 3 ) ],
// Pi1 = k (grad u + grad u^T), k = -rho / (6 beta), gradients by central
// differences.  Pass 1 forms the pointwise derivative in u, the per-node
// beta term and P[ab] = sum_i lam_i dG_i / d(d_a u_b); pass 2 applies the
// transpose of the central-difference stencil.
template <typename R>
__global__ __launch_bounds__(256) void k_adj_init_a(const R* __restrict__ lam, int nx, int ny, int64_t pitch,
                                                    double rho0, double beta, const double* __restrict__ rho,
                                                    const double* __restrict__ ux,
                                                    const double* __restrict__ uy, int mode,
                                                    double* __restrict__ gux, double* __restrict__ guy,
                                                    double* __restrict__ P, double* __restrict__ partials) {
    const int64_t N = static_cast<int64_t>(nx) * ny;
    const int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    double db = 0.0;
    if (n < N) {
        const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<int64_t>(y) * nx);
        const double r = rho ? rho[n] : rho0;
        const double u = ux[n], v = uy[n];
        double l[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) l[i] = static_cast<double>(lam[(static_cast<int64_t>(y) * 9 + i) * pitch + x]);
        double gx = 0.0, gy = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double cx = kCx[i], cy = kCy[i];
            const double cu = cx * u + cy * v;
            const double wl = weight(i) * l[i];
            gx += wl * r * (3.0 * cx + 9.0 * cu * cx - 3.0 * u);
            gy += wl * r * (3.0 * cy + 9.0 * cu * cy - 3.0 * v);
            sxx += wl * 4.5 * (cx * cx - 1.0 / 3.0);
            syy += wl * 4.5 * (cy * cy - 1.0 / 3.0);
            sxy += wl * 9.0 * cx * cy;
        }
        gux[n] = gx;
        guy[n] = gy;
        if (mode == 1) {
            const int64_t xp = static_cast<int64_t>(y) * nx + wrapi(x + 1, nx);
            const int64_t xm = static_cast<int64_t>(y) * nx + wrapi(x - 1, nx);
            const int64_t yp = static_cast<int64_t>(wrapi(y + 1, ny)) * nx + x;
            const int64_t ym = static_cast<int64_t>(wrapi(y - 1, ny)) * nx + x;
            const double dxux = 0.5 * (ux[xp] - ux[xm]), dyux = 0.5 * (ux[yp] - ux[ym]);
            const double dxuy = 0.5 * (uy[xp] - uy[xm]), dyuy = 0.5 * (uy[yp] - uy[ym]);
            const double k = -r / (6.0 * beta);
            // P[0] = d/d(d_x u_x), P[1] = d/d(d_x u_y), P[2] = d/d(d_y u_x), P[3] = d/d(d_y u_y)
            P[n] = 2.0 * k * sxx;
            P[N + n] = k * sxy;
            P[2 * N + n] = k * sxy;
            P[3 * N + n] = 2.0 * k * syy;
            // dk/dbeta = -k / beta
            const double Pxx = 2.0 * k * dxux, Pyy = 2.0 * k * dyuy, Pxy = k * (dyux + dxuy);
            db = -(Pxx * sxx + Pyy * syy + Pxy * sxy) / beta;
        }
    }
    const double s = block_sum(db);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_adj_init_b(int nx, int ny, const double* __restrict__ P,
                                                    double* __restrict__ gux, double* __restrict__ guy) {
    const int64_t N = static_cast<int64_t>(nx) * ny;
    const int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (n >= N) return;
    const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<int64_t>(y) * nx);
    const int64_t xp = static_cast<int64_t>(y) * nx + wrapi(x + 1, nx);
    const int64_t xm = static_cast<int64_t>(y) * nx + wrapi(x - 1, nx);
    const int64_t yp = static_cast<int64_t>(wrapi(y + 1, ny)) * nx + x;
    const int64_t ym = static_cast<int64_t>(wrapi(y - 1, ny)) * nx + x;
    // d_a u_b(x) = (u_b(x + e_a) - u_b(x - e_a)) / 2, transposed
    gux[n] += 0.5 * (P[xm] - P[xp]) + 0.5 * (P[2 * N + ym] - P[2 * N + yp]);
    guy[n] += 0.5 * (P[N + xm] - P[N + xp]) + 0.5 * (P[3 * N + ym] - P[3 * N + yp]);
}

int ok() { return hipGetLastError() == hipSuccess ? 0 : -2; }

// Workgroups of one adjoint step (= per-workgroup partials it writes).
int64_t adj_blocks(const Lattice& L) {
    const int wr = 2 * adj_rows_per_thread(L);
    const int64_t ntx = (L.nx + 127) / 128, nty = (L.ny + wr - 1) / wr;
    return 8 * ((nty + 7) / 8) * ntx;
}

// Up to kDirect workgroups the partials are the step's slice; beyond, they
// are folded by kFold into a shorter slice (one more launch per step, which
// small lattices, limited by launch rate, should not pay).
constexpr int64_t kDirect = 16384;
int64_t adj_slice_len(const Lattice& L) {
    const int64_t nb = adj_blocks(L);
    return nb <= kDirect ? nb : (nb + kFold - 1) / kFold;
}

template <int FORM, int COLL, int VAR, int GM>
struct AdjStepOp {
    static int run(const Lattice& L, const void* state, const void* lin, void* lout, double* partials,
                   double* slice, double* acc, const void* fsrc, void* fdst) {
        return go(L, state, lin, lout, partials, slice, acc, fsrc, fdst);
    }
    template <bool FROZEN, int RPT>
    static void launch(const Lattice& L, const void* state, const void* lin, void* lout, int ntx, int nty,
                       int64_t nb, double* out, const void* fsrc, void* fdst) {
        using F = Form<FORM>;
        using R = typename F::R;
        using S = typename F::S;
        if (L.adj_halo[0]) {   // a slab (no fused forward part: checked by go)
            SlabHalo<S> sh;
            sh.lo = static_cast<const S*>(L.adj_halo[0]);
            sh.hi = static_cast<const S*>(L.adj_halo[1]);
            SlabHalo<R> lh;
            lh.lo = static_cast<const R*>(L.adj_halo[2]);
            lh.hi = static_cast<const R*>(L.adj_halo[3]);
            k_adj_step<FORM, COLL, VAR, GM, FROZEN, RPT, true>
                <<<dim3(static_cast<unsigned>(nb)), dim3(256), 0, L.stream>>>(
                    static_cast<const S*>(state), static_cast<const R*>(lin), static_cast<R*>(lout), L.nx, L.ny,
                    L.pitch, ntx, nty, make_coef<R>(L), out, sh, lh);
            return;
        }
        if (!fsrc) {
            k_adj_step<FORM, COLL, VAR, GM, FROZEN, RPT, false>
                <<<dim3(static_cast<unsigned>(nb)), dim3(256), 0, L.stream>>>(
                    static_cast<const S*>(state), static_cast<const R*>(lin), static_cast<R*>(lout), L.nx, L.ny,
                    L.pitch, ntx, nty, make_coef<R>(L), out, SlabHalo<S>{}, SlabHalo<R>{});
            return;
        }
        // forward part: 256 x 1 tiles, renumbered per XCD as in the step kernel
        const int ntx_f = (L.nx + 255) / 256;
        const int ntiles_f = ntx_f * L.ny;
        const int per_xcd_f = (ntiles_f + 7) / 8;
        const int64_t grid = nb + 8 * static_cast<int64_t>(per_xcd_f);
        k_adj_step_fwd<FORM, COLL, VAR, GM, FROZEN, RPT><<<dim3(static_cast<unsigned>(grid)), dim3(256), 0, L.stream>>>(
            static_cast<const S*>(state), static_cast<const R*>(lin), static_cast<R*>(lout), L.nx, L.ny, L.pitch,
            ntx, nty, make_coef<R>(L), out, static_cast<unsigned>(nb), static_cast<const S*>(fsrc),
            static_cast<S*>(fdst), ntx_f, ntiles_f, per_xcd_f);
    }
    static int go(const Lattice& L, const void* state, const void* lin, void* lout, double* partials,
                  double* slice, double* acc, const void* fsrc, void* fdst) {
        const int rpt = adj_rows_per_thread(L);
        const int ntx = (L.nx + 127) / 128, nty = (L.ny + 2 * rpt - 1) / (2 * rpt);
        const int64_t nb = adj_blocks(L);
        if (!grid_fits(nb, 256)) return kTooLarge;
        if ((fsrc == nullptr) != (fdst == nullptr)) return -1;
        if (L.adj_halo[0] && fsrc) return -1;   // a slab's adjoint step runs alone
        // the fused forward part needs its grid to fit next to the adjoint's
        if (fsrc && !grid_fits(static_cast<int64_t>((L.nx + 255) / 256) * L.ny + 8 + nb, 256)) return kTooLarge;
        const bool direct = nb <= kDirect;
        if (!slice || (!direct && !partials)) return -1;
        double* out = direct ? slice : partials;
        if constexpr (FORM == F64) {
            if (rpt != 1) return -1;
            if (L.adj_frozen)
                launch<true, 1>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
            else
                launch<false, 1>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
        } else {
            if (L.adj_frozen) {
                if (rpt == 2) launch<true, 2>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
                else launch<true, 1>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
            } else {
                if (rpt == 2) launch<false, 2>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
                else launch<false, 1>(L, state, lin, lout, ntx, nty, nb, out, fsrc, fdst);
            }
        }
        if (ok()) return -2;
        const int64_t len = adj_slice_len(L);
        if (!direct) {
            k_fold<<<dim3(static_cast<unsigned>(len)), dim3(256), 0, L.stream>>>(partials, nb, slice);
            if (ok()) return -2;
        }
        if (acc) {
            k_sum_partials<<<1, 256, 0, L.stream>>>(slice, len, acc);
            if (ok()) return -2;
        }
        return 0;
    }
};

// tot[n] = sum of slice n, reduced exactly as k_sum_partials reduces a slice
// (one workgroup per slice)
__global__ __launch_bounds__(256) void k_slice_sums(const double* __restrict__ slices, int64_t len,
                                                    double* __restrict__ tot) {
    const double* p = slices + static_cast<int64_t>(blockIdx.x) * len;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < len; i += 256) s += p[i];
    const double t = block_sum(s);
    if (threadIdx.x == 0) tot[blockIdx.x] = t;
}

// acc[0] += tot[n] for n = k-1 down to 0, the order in which the segment's
// adjoint steps ran: bitwise the same as adding each step's sum after it.
__global__ void k_add_in_order(const double* __restrict__ tot, int k, double* __restrict__ acc) {
    if (threadIdx.x != 0) return;
    double a = acc[0];
    for (int n = k - 1; n >= 0; --n) a += tot[n];
    acc[0] = a;
}

}  // namespace

// scratch doubles for the unfolded partials of one adjoint step (0 when the
// partials are the slice itself), and the length of a step's slice
int64_t adjoint_partials(const Lattice& L) { return adj_blocks(L) <= kDirect ? 0 : adj_blocks(L); }
int64_t adjoint_slice_len(const Lattice& L) { return adj_slice_len(L); }

int launch_sum_slices(const double* slices, int64_t len, int k, double* tot, double* acc, hipStream_t stream) {
    if (!acc || len <= 0 || k <= 0) return 0;
    k_slice_sums<<<dim3(static_cast<unsigned>(k)), dim3(256), 0, stream>>>(slices, len, tot);
    if (ok()) return -2;
    k_add_in_order<<<1, 64, 0, stream>>>(tot, k, acc);
    return ok();
}

int launch_adjoint_seed(const Lattice& L, const void* state, const double* drho, const double* dux,
                        const double* duy, void* lam) {
    const dim3 g(static_cast<unsigned>((L.nx + 63) / 64), static_cast<unsigned>((L.ny + 3) / 4)), b(64, 4);
    switch (L.form) {
        case F16: k_adj_seed<F16><<<g, b, 0, L.stream>>>(static_cast<const _Float16*>(state), L.nx, L.ny, L.pitch, L.rho0, drho, dux, duy, static_cast<float*>(lam)); break;
        case F32: k_adj_seed<F32><<<g, b, 0, L.stream>>>(static_cast<const float*>(state), L.nx, L.ny, L.pitch, L.rho0, drho, dux, duy, static_cast<float*>(lam)); break;
        case F64: k_adj_seed<F64><<<g, b, 0, L.stream>>>(static_cast<const double*>(state), L.nx, L.ny, L.pitch, L.rho0, drho, dux, duy, static_cast<double*>(lam)); break;
        default: return -1;
    }
    return ok();
}

int launch_adjoint_step(const Lattice& L, const void* state, const void* lin, void* lout, double* partials,
                        double* slice, double* acc, const void* fsrc, void* fdst) {
    return dispatch<AdjStepOp>(L, state, lin, lout, partials, slice, acc, fsrc, fdst);
}

int launch_adjoint_init(const Lattice& L, const double* rho, const double* ux, const double* uy, int mode,
                        const void* lam0, double* gux, double* guy, double* P, double* partials,
                        int64_t nblocks_cap, double* acc) {
    const int64_t N = static_cast<int64_t>(L.nx) * L.ny;
    const int64_t nb = (N + 255) / 256;
    if (!grid_fits(nb, 256)) return kTooLarge;
    if (nb > nblocks_cap) return -1;
    const dim3 g(static_cast<unsigned>(nb)), b(256);
    if (L.form == F64)
        k_adj_init_a<double><<<g, b, 0, L.stream>>>(static_cast<const double*>(lam0), L.nx, L.ny, L.pitch, L.rho0, L.beta, rho, ux, uy, mode, gux, guy, P, partials);
    else
        k_adj_init_a<float><<<g, b, 0, L.stream>>>(static_cast<const float*>(lam0), L.nx, L.ny, L.pitch, L.rho0, L.beta, rho, ux, uy, mode, gux, guy, P, partials);
    if (ok()) return -2;
    if (mode == 1) {
        k_adj_init_b<<<g, b, 0, L.stream>>>(L.nx, L.ny, P, gux, guy);
        if (ok()) return -2;
    }
    if (acc) {
        k_sum_partials<<<1, 256, 0, L.stream>>>(partials, nb, acc);
        if (ok()) return -2;
    }
    return 0;
}

}  // namespace kbc
