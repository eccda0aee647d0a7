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
// stored [9][ny][pitch] in the form's arithmetic type, unshifted.
#include <type_traits>

#include "kbc_adjoint.hpp"
#include "kbc_launch.hpp"

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
        const double g = F::dec64(state[(static_cast<int64_t>(i) * ny + ys) * pitch + xs], i);
        dr += g;
        jx += kCx[i] * g;
        jy += kCy[i] * g;
    }
    const double r = rho0 + dr, u = jx / r, v = jy / r;
    const int64_t n = static_cast<int64_t>(y) * nx + x;
    const double a = drho ? drho[n] : 0.0;
    const double bx = dux ? dux[n] : 0.0, by = duy ? duy[n] : 0.0;
    const int64_t plane = static_cast<int64_t>(ny) * pitch;
    R* o = lam + static_cast<int64_t>(y) * pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        o[i * plane] = static_cast<R>(a + (bx * (kCx[i] - u) + by * (kCy[i] - v)) / r);
}

// ----------------------------------------------------------------- adjoint step
template <int FORM, int COLL, int VAR, int GM, bool FROZEN>
__global__ __launch_bounds__(256) void k_adj_step(const typename Form<FORM>::S* __restrict__ state,
                                                  const typename Form<FORM>::R* __restrict__ lin,
                                                  typename Form<FORM>::R* __restrict__ lout, int nx,
                                                  int ny, int64_t pitch, int ntx, int ntiles, int per_xcd,
                                                  Coef<typename Form<FORM>::R> K,
                                                  double* __restrict__ partials) {
    using F = Form<FORM>;
    using R = typename F::R;
    constexpr int TW = 128, WR = 2;   // tile: 128 x 2 nodes, XCD-banded like the forward step
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    double db = 0.0;
    if (t < ntiles) {
        const int tx = t % ntx, ty = t / ntx;
        const int x = tx * TW + static_cast<int>(threadIdx.x % TW);
        const int y = ty * WR + static_cast<int>(threadIdx.x / TW);
        if (x < nx && y < ny) {
            const int64_t plane = static_cast<int64_t>(ny) * pitch;
            const int xm = (x == 0) ? nx - 1 : x - 1, xp = (x == nx - 1) ? 0 : x + 1;
            const int ym = (y == 0) ? ny - 1 : y - 1, yp = (y == ny - 1) ? 0 : y + 1;
            const int64_t r0 = static_cast<int64_t>(y) * pitch, rm = static_cast<int64_t>(ym) * pitch,
                          rp = static_cast<int64_t>(yp) * pitch;
            R g[9], mu[9], lam[9];
            // f^n_i(x) sits at x - v_i
            g[0] = F::dec(state[r0 + x], 0);
            g[1] = F::dec(state[plane + r0 + xm], 1);
            g[2] = F::dec(state[2 * plane + rm + x], 2);
            g[3] = F::dec(state[3 * plane + r0 + xp], 3);
            g[4] = F::dec(state[4 * plane + rp + x], 4);
            g[5] = F::dec(state[5 * plane + rm + xm], 5);
            g[6] = F::dec(state[6 * plane + rm + xp], 6);
            g[7] = F::dec(state[7 * plane + rp + xp], 7);
            g[8] = F::dec(state[8 * plane + rp + xm], 8);
            // mu_i(x) = lam^{n+1}_i(x + v_i)
            mu[0] = lin[r0 + x];
            mu[1] = lin[plane + r0 + xp];
            mu[2] = lin[2 * plane + rp + x];
            mu[3] = lin[3 * plane + r0 + xm];
            mu[4] = lin[4 * plane + rm + x];
            mu[5] = lin[5 * plane + rp + xp];
            mu[6] = lin[6 * plane + rp + xm];
            mu[7] = lin[7 * plane + rm + xm];
            mu[8] = lin[8 * plane + rm + xp];
            R dbn;
            collide_vjp<R, COLL, VAR, GM, FROZEN>(g, mu, K, lam, dbn);
            R* o = lout + r0 + x;
#pragma unroll
            for (int i = 0; i < 9; ++i) o[i * plane] = lam[i];
            db = static_cast<double>(dbn);
        }
    }
    const double s = block_sum(db);
    if (threadIdx.x == 0) partials[b] = s;
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
        const int64_t plane = static_cast<int64_t>(ny) * pitch;
        double l[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) l[i] = static_cast<double>(lam[i * plane + static_cast<int64_t>(y) * pitch + x]);
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

template <int FORM, int COLL, int VAR, int GM>
struct AdjStepOp {
    static int run(const Lattice& L, const void* state, const void* lin, void* lout, double* partials,
                   int64_t nblocks_cap, double* acc) {
        using F = Form<FORM>;
        using R = typename F::R;
        const int ntx = (L.nx + 127) / 128, nty = (L.ny + 1) / 2;
        const int64_t nt64 = static_cast<int64_t>(ntx) * nty;
        if (nt64 > (int64_t{1} << 30)) return -1;
        const int ntiles = static_cast<int>(nt64);
        const int per_xcd = (ntiles + 7) / 8;
        const int64_t nblocks = 8 * static_cast<int64_t>(per_xcd);
        if (nblocks > nblocks_cap) return -1;
        if (L.adj_frozen)
            k_adj_step<FORM, COLL, VAR, GM, true><<<dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, L.stream>>>(
                static_cast<const typename F::S*>(state), static_cast<const R*>(lin), static_cast<R*>(lout), L.nx,
                L.ny, L.pitch, ntx, ntiles, per_xcd, make_coef<R>(L), partials);
        else
            k_adj_step<FORM, COLL, VAR, GM, false><<<dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, L.stream>>>(
                static_cast<const typename F::S*>(state), static_cast<const R*>(lin), static_cast<R*>(lout), L.nx,
                L.ny, L.pitch, ntx, ntiles, per_xcd, make_coef<R>(L), partials);
        if (ok()) return -2;
        if (acc) {
            k_sum_partials<<<1, 256, 0, L.stream>>>(partials, nblocks, acc);
            if (ok()) return -2;
        }
        return 0;
    }
};

}  // namespace

int64_t adjoint_step_blocks(const Lattice& L) {
    const int64_t ntx = (L.nx + 127) / 128, nty = (L.ny + 1) / 2;
    return 8 * ((ntx * nty + 7) / 8);
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
                        int64_t nblocks_cap, double* acc) {
    return dispatch<AdjStepOp>(L, state, lin, lout, partials, nblocks_cap, acc);
}

int launch_adjoint_init(const Lattice& L, const double* rho, const double* ux, const double* uy, int mode,
                        const void* lam0, double* gux, double* guy, double* P, double* partials,
                        int64_t nblocks_cap, double* acc) {
    const int64_t N = static_cast<int64_t>(L.nx) * L.ny;
    const int64_t nb = (N + 255) / 256;
    if (nb > nblocks_cap || nb > (int64_t{1} << 31) - 1) return -1;
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
