// kbc_aux.hip -- kernels around the step: initial state, moments, population
// import/export, diagnostics reductions and the bandwidth reference copy.
//
// All of them address the state the way the step does: the pre-collision
// population f_i(x, t = n) sits in population row i of lattice row y - v_iy,
// at column x - v_ix ([ny][9][pitch] layout).
#include "kbc_launch.hpp"

namespace kbc {

namespace {

__device__ __forceinline__ int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// element offset of f_i(x, y) in a state buffer
__device__ __forceinline__ int64_t src_off(int i, int x, int y, int nx, int ny, int64_t pitch) {
    const int xs = wrap(x - kCx[i], nx), ys = wrap(y - kCy[i], ny);
    return (static_cast<int64_t>(ys) * 9 + i) * pitch + xs;
}

// ------------------------------------------------------------ initial state
// Grad's approximation eq. (Grad) in deviation form:
//   f*_i - W_i rho0 = W_i [ (rho - rho0) + 3 rho (v.u)
//                           + 4.5 ( rho (v.u)^2 - rho |u|^2 / 3 + Pi1 : v v - tr(Pi1) / 3 ) ]
// with Pi1 = -(rho / (6 beta)) (grad u + grad u^T) (eq. P1AC, cs2 = 1/3); the
// equilibrium eq. (Eq) is the case Pi1 = 0.
template <int FORM>
__global__ __launch_bounds__(256) void k_init(typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                              int64_t pitch, double rho0, double beta,
                                              const double* __restrict__ rho,
                                              const double* __restrict__ ux,
                                              const double* __restrict__ uy,
                                              const double* __restrict__ grad, int mode) {
    using F = Form<FORM>;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int64_t N = static_cast<int64_t>(nx) * ny;
    const int64_t n = static_cast<int64_t>(y) * nx + x;
    const double r = rho ? rho[n] : rho0;
    const double u = ux[n], v = uy[n];
    double Pxx = 0.0, Pyy = 0.0, Pxy = 0.0;
    if (mode != 0) {
        double dxux, dyux, dxuy, dyuy;
        if (mode == 2) {
            dxux = grad[n];
            dyux = grad[N + n];
            dxuy = grad[2 * N + n];
            dyuy = grad[3 * N + n];
        } else {
            const int64_t xp = static_cast<int64_t>(y) * nx + wrap(x + 1, nx);
            const int64_t xm = static_cast<int64_t>(y) * nx + wrap(x - 1, nx);
            const int64_t yp = static_cast<int64_t>(wrap(y + 1, ny)) * nx + x;
            const int64_t ym = static_cast<int64_t>(wrap(y - 1, ny)) * nx + x;
            dxux = 0.5 * (ux[xp] - ux[xm]);
            dyux = 0.5 * (ux[yp] - ux[ym]);
            dxuy = 0.5 * (uy[xp] - uy[xm]);
            dyuy = 0.5 * (uy[yp] - uy[ym]);
        }
        const double k = -r / (6.0 * beta);
        Pxx = 2.0 * k * dxux;
        Pyy = 2.0 * k * dyuy;
        Pxy = k * (dyux + dxuy);
    }
    const double dr = r - rho0;
    const double u2 = u * u + v * v;
    const double tr3 = (Pxx + Pyy) / 3.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double cx = kCx[i], cy = kCy[i];
        const double cu = cx * u + cy * v;
        const double pvv = Pxx * cx * cx + 2.0 * Pxy * cx * cy + Pyy * cy * cy;
        const double dev = weight(i) * (dr + 3.0 * r * cu + 4.5 * (r * cu * cu - r * u2 / 3.0 + pvv - tr3));
        const int xs = wrap(x - kCx[i], nx), ys = wrap(y - kCy[i], ny);
        dst[(static_cast<int64_t>(ys) * 9 + i) * pitch + xs] = F::enc64(dev, i);
    }
}

// --------------------------------------------------------------- moments
template <int FORM, int COLL, int VAR, int GM>
__global__ __launch_bounds__(256) void k_moments(const typename Form<FORM>::S* __restrict__ src, int nx,
                                                 int ny, int64_t pitch,
                                                 Coef<typename Form<FORM>::R> K, double rho0,
                                                 double* __restrict__ rho, double* __restrict__ ux,
                                                 double* __restrict__ uy, double* __restrict__ gam) {
    using F = Form<FORM>;
    using R = typename F::R;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    typename F::S s[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = src[src_off(i, x, y, nx, ny, pitch)];
    double dr = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double g = F::dec64(s[i], i);
        dr += g;
        jx += kCx[i] * g;
        jy += kCy[i] * g;
    }
    const int64_t n = static_cast<int64_t>(y) * nx + x;
    const double r = rho0 + dr;
    if (rho) rho[n] = r;
    if (ux) ux[n] = jx / r;
    if (uy) uy[n] = jy / r;
    if (gam) {
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = F::dec(s[i], i);
        gam[n] = static_cast<double>(collide<R, COLL, VAR, GM>(g, K));
    }
}

// ------------------------------------------------------- population import/export
template <int FORM>
__global__ __launch_bounds__(256) void k_get_pop(const typename Form<FORM>::S* __restrict__ src, int nx,
                                                 int ny, int64_t pitch, double rho0,
                                                 double* __restrict__ f) {
    using F = Form<FORM>;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int64_t N = static_cast<int64_t>(nx) * ny;
    const int64_t n = static_cast<int64_t>(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i * N + n] = F::dec64(src[src_off(i, x, y, nx, ny, pitch)], i) + weight(i) * rho0;
}

template <int FORM>
__global__ __launch_bounds__(256) void k_set_pop(typename Form<FORM>::S* __restrict__ dst, int nx, int ny,
                                                 int64_t pitch, double rho0,
                                                 const double* __restrict__ f) {
    using F = Form<FORM>;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int64_t N = static_cast<int64_t>(nx) * ny;
    const int64_t n = static_cast<int64_t>(y) * nx + x;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        dst[src_off(i, x, y, nx, ny, pitch)] = F::enc64(f[i * N + n] - weight(i) * rho0, i);
}

// ----------------------------------------------------------- diagnostics
// Slots of the per-block partials.
enum {
    D_RHO = 0, D_JX, D_JY, D_E, D_E2, D_S, D_G, D_G2, D_NONFIN, D_FEQNEG, D_RHO2,
    D_Z, D_Z2, D_P, D_P2, D_UNUSED
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum `cnt` per-thread values across the 256-thread block and store them at
// partials[blockIdx.x * kDiagSlots + first + k].
template <int CNT>
__device__ __forceinline__ void block_store(double (&acc)[CNT], double* partials, int first) {
    __shared__ double red[4][CNT];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < CNT; ++k) {
        const double s = wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < CNT) {
        const int k = threadIdx.x;
        partials[static_cast<int64_t>(blockIdx.x) * kDiagSlots + first + k] =
            (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
    }
}

template <int FORM, int COLL, int VAR, int GM>
__global__ __launch_bounds__(256) void k_diag_a(const typename Form<FORM>::S* __restrict__ src, int nx,
                                                int ny, int64_t pitch, Coef<typename Form<FORM>::R> K,
                                                double rho0, double* __restrict__ ux_s,
                                                double* __restrict__ uy_s, double* __restrict__ partials) {
    using F = Form<FORM>;
    using R = typename F::R;
    const int64_t N = static_cast<int64_t>(nx) * ny;
    double acc[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * 256) {
        const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<int64_t>(y) * nx);
        typename F::S s[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) s[i] = src[src_off(i, x, y, nx, ny, pitch)];
        double f[9], dr = 0.0, jx = 0.0, jy = 0.0;
        bool finite = true;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double g = F::dec64(s[i], i);
            f[i] = g + weight(i) * rho0;
            finite = finite && isfinite(f[i]);
            dr += g;
            jx += kCx[i] * g;
            jy += kCy[i] * g;
        }
        const double r = rho0 + dr;
        const double u = jx / r, v = jy / r;
        ux_s[n] = u;
        uy_s[n] = v;
        double Sn = 0.0;
        bool neg = false;
        const double u2 = u * u + v * v;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            Sn -= f[i] * log(f[i] / weight(i));
            const double cu = kCx[i] * u + kCy[i] * v;
            const double feq = weight(i) * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * u2);
            neg = neg || !(feq > 0.0);
        }
        R g[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = F::dec(s[i], i);
        const double gm = static_cast<double>(collide<R, COLL, VAR, GM>(g, K));
        const double e = 0.5 * u2;
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += e;
        acc[4] += e * e;
        acc[5] += Sn;
        acc[6] += gm;
        acc[7] += gm * gm;
        acc[8] += finite ? 0.0 : 1.0;
        acc[9] += neg ? 1.0 : 0.0;
        acc[10] += r * r;
    }
    block_store<11>(acc, partials, D_RHO);
}

__global__ __launch_bounds__(256) void k_diag_b(int nx, int ny, const double* __restrict__ ux_s,
                                                const double* __restrict__ uy_s, double* __restrict__ w_s,
                                                double* __restrict__ partials) {
    const int64_t N = static_cast<int64_t>(nx) * ny;
    double acc[2] = {0, 0};
    for (int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * 256) {
        const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<int64_t>(y) * nx);
        const int64_t xp = static_cast<int64_t>(y) * nx + wrap(x + 1, nx);
        const int64_t xm = static_cast<int64_t>(y) * nx + wrap(x - 1, nx);
        const int64_t yp = static_cast<int64_t>(wrap(y + 1, ny)) * nx + x;
        const int64_t ym = static_cast<int64_t>(wrap(y - 1, ny)) * nx + x;
        const double w = 0.5 * (uy_s[xp] - uy_s[xm]) - 0.5 * (ux_s[yp] - ux_s[ym]);
        w_s[n] = w;
        const double z = 0.5 * w * w;
        acc[0] += z;
        acc[1] += z * z;
    }
    block_store<2>(acc, partials, D_Z);
}

__global__ __launch_bounds__(256) void k_diag_c(int nx, int ny, const double* __restrict__ w_s,
                                                double* __restrict__ partials) {
    const int64_t N = static_cast<int64_t>(nx) * ny;
    double acc[2] = {0, 0};
    for (int64_t n = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; n < N;
         n += static_cast<int64_t>(gridDim.x) * 256) {
        const int y = static_cast<int>(n / nx), x = static_cast<int>(n - static_cast<int64_t>(y) * nx);
        const int64_t xp = static_cast<int64_t>(y) * nx + wrap(x + 1, nx);
        const int64_t xm = static_cast<int64_t>(y) * nx + wrap(x - 1, nx);
        const int64_t yp = static_cast<int64_t>(wrap(y + 1, ny)) * nx + x;
        const int64_t ym = static_cast<int64_t>(wrap(y - 1, ny)) * nx + x;
        const double gx = 0.5 * (w_s[xp] - w_s[xm]);
        const double gy = 0.5 * (w_s[yp] - w_s[ym]);
        const double p = 0.5 * (gx * gx + gy * gy);
        acc[0] += p;
        acc[1] += p * p;
    }
    block_store<2>(acc, partials, D_P);
}

// ------------------------------------------------------------ copy reference
// The plainest streaming copy: one 4-byte word per lane, one pass, the same
// access granularity as the step kernel's loads and stores.  It is the
// reference both for achievable bandwidth and for scaling the HBM byte
// counters of the profiler.
__global__ __launch_bounds__(256) void k_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

dim3 node_grid(const Lattice& L) {
    return dim3(static_cast<unsigned>((L.nx + 63) / 64), static_cast<unsigned>((L.ny + 3) / 4));
}

int ok_launch() { return hipGetLastError() == hipSuccess ? 0 : -2; }

template <int FORM, int COLL, int VAR, int GM>
struct MomOp {
    static int run(const Lattice& L, const void* src, double* rho, double* ux, double* uy, double* g) {
        using F = Form<FORM>;
        k_moments<FORM, COLL, VAR, GM><<<node_grid(L), dim3(64, 4), 0, L.stream>>>(
            static_cast<const typename F::S*>(src), L.nx, L.ny, L.pitch, make_coef<typename F::R>(L),
            L.rho0, rho, ux, uy, g);
        return ok_launch();
    }
};

template <int FORM, int COLL, int VAR, int GM>
struct DiagOp {
    static int run(const Lattice& L, const void* src, double* ux_s, double* uy_s, double* w_s,
                   double* partials) {
        using F = Form<FORM>;
        k_diag_a<FORM, COLL, VAR, GM><<<kDiagBlocks, 256, 0, L.stream>>>(
            static_cast<const typename F::S*>(src), L.nx, L.ny, L.pitch, make_coef<typename F::R>(L),
            L.rho0, ux_s, uy_s, partials);
        if (ok_launch()) return -2;
        k_diag_b<<<kDiagBlocks, 256, 0, L.stream>>>(L.nx, L.ny, ux_s, uy_s, w_s, partials);
        if (ok_launch()) return -2;
        k_diag_c<<<kDiagBlocks, 256, 0, L.stream>>>(L.nx, L.ny, w_s, partials);
        return ok_launch();
    }
};

}  // namespace

int launch_init(const Lattice& L, void* dst, const double* rho, const double* ux, const double* uy,
                const double* grad, int mode) {
    const dim3 g = node_grid(L), b(64, 4);
    switch (L.form) {
        case F16: k_init<F16><<<g, b, 0, L.stream>>>(static_cast<_Float16*>(dst), L.nx, L.ny, L.pitch, L.rho0, L.beta, rho, ux, uy, grad, mode); break;
        case F32: k_init<F32><<<g, b, 0, L.stream>>>(static_cast<float*>(dst), L.nx, L.ny, L.pitch, L.rho0, L.beta, rho, ux, uy, grad, mode); break;
        case F64: k_init<F64><<<g, b, 0, L.stream>>>(static_cast<double*>(dst), L.nx, L.ny, L.pitch, L.rho0, L.beta, rho, ux, uy, grad, mode); break;
        default: return -1;
    }
    return ok_launch();
}

int launch_moments(const Lattice& L, const void* src, double* rho, double* ux, double* uy, double* gamma) {
    return dispatch<MomOp>(L, src, rho, ux, uy, gamma);
}

int launch_get_pop(const Lattice& L, const void* src, double* f) {
    const dim3 g = node_grid(L), b(64, 4);
    switch (L.form) {
        case F16: k_get_pop<F16><<<g, b, 0, L.stream>>>(static_cast<const _Float16*>(src), L.nx, L.ny, L.pitch, L.rho0, f); break;
        case F32: k_get_pop<F32><<<g, b, 0, L.stream>>>(static_cast<const float*>(src), L.nx, L.ny, L.pitch, L.rho0, f); break;
        case F64: k_get_pop<F64><<<g, b, 0, L.stream>>>(static_cast<const double*>(src), L.nx, L.ny, L.pitch, L.rho0, f); break;
        default: return -1;
    }
    return ok_launch();
}

int launch_set_pop(const Lattice& L, void* dst, const double* f) {
    const dim3 g = node_grid(L), b(64, 4);
    switch (L.form) {
        case F16: k_set_pop<F16><<<g, b, 0, L.stream>>>(static_cast<_Float16*>(dst), L.nx, L.ny, L.pitch, L.rho0, f); break;
        case F32: k_set_pop<F32><<<g, b, 0, L.stream>>>(static_cast<float*>(dst), L.nx, L.ny, L.pitch, L.rho0, f); break;
        case F64: k_set_pop<F64><<<g, b, 0, L.stream>>>(static_cast<double*>(dst), L.nx, L.ny, L.pitch, L.rho0, f); break;
        default: return -1;
    }
    return ok_launch();
}

int launch_diag(const Lattice& L, const void* src, double* ux_s, double* uy_s, double* w_s,
                double* partials) {
    return dispatch<DiagOp>(L, src, ux_s, uy_s, w_s, partials);
}

int launch_copy(void* dst, const void* src, size_t n_words, hipStream_t stream) {
    const int64_t n = static_cast<int64_t>(n_words);
    if (n == 0) return 0;
    const int64_t blocks = (n + 255) / 256;
    if (!grid_fits(blocks, 256)) return kTooLarge;
    k_copy<<<static_cast<unsigned>(blocks), 256, 0, stream>>>(static_cast<float*>(dst), static_cast<const float*>(src), n);
    return ok_launch();
}

}  // namespace kbc
