// kbc_spectra.hip -- shell-summed kinetic-energy and enstrophy spectra of a
// square periodic lattice (turbulence statistics of section "Decaying
// Two-Dimensional Turbulence").
//
// With u_hat the unnormalised discrete Fourier transform of a velocity
// component on N x N nodes, Parseval gives <|u|^2> = sum_k |u_hat(k)|^2 / N^4,
// so E = (1/2) <|u|^2> splits over wavevectors k (integers, |k_a| <= N/2) as
// e(k) = (|ux_hat|^2 + |uy_hat|^2) / (2 N^4).  E(k) sums e over the shell
// round(|k|) = k; Z(k) sums e(k) (2 pi |k| / N)^2, the spectral enstrophy
// (1/2) <omega^2> with the exact derivative.  The transform is real-to-complex,
// so the stored half plane 0 <= k_x <= N/2 counts twice except the columns
// k_x = 0 and k_x = N/2 (N even).  Shells above kmax are dropped.  Shell sums
// are FP64 atomic adds: results repeat to rounding, not bit for bit.
#include <hipfft/hipfft.h>

#include <cmath>

#include "kbc_launch.hpp"

namespace kbc {

namespace {

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ p, int n) {
    const int i = static_cast<int>(blockIdx.x) * 256 + static_cast<int>(threadIdx.x);
    if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_shells(const double2* __restrict__ fx, const double2* __restrict__ fy,
                                                int n, int nh, int kmax, double scale, double kunit2,
                                                double* __restrict__ ek, double* __restrict__ zk) {
    const int64_t total = static_cast<int64_t>(n) * nh;
    for (int64_t m = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; m < total;
         m += static_cast<int64_t>(gridDim.x) * 256) {
        const int ky = static_cast<int>(m / nh), kx = static_cast<int>(m - static_cast<int64_t>(ky) * nh);
        const int kys = (ky <= n / 2) ? ky : ky - n;
        const double w = (kx == 0 || (2 * kx == n)) ? 1.0 : 2.0;
        const double2 a = fx[m], b = fy[m];
        const double e = w * scale * (a.x * a.x + a.y * a.y + b.x * b.x + b.y * b.y);
        const double k2 = static_cast<double>(kx) * kx + static_cast<double>(kys) * kys;
        const int shell = static_cast<int>(floor(sqrt(k2) + 0.5));
        if (shell > kmax) continue;
        if (ek) atomicAdd(ek + shell, e);
        if (zk) atomicAdd(zk + shell, e * k2 * kunit2);
    }
}

int fft_fail(hipfftResult r) { return r == HIPFFT_SUCCESS ? 0 : -2; }

}  // namespace

// work: 2 n^2 doubles (ux, uy) followed by 2 n (n/2 + 1) complex values
int launch_spectra(const Lattice& L, const void* state, void** plan_slot, double* work, int kmax, double* ek,
                   double* zk) {
    const int n = L.nx;
    if (L.nx != L.ny || kmax < 0) return -1;
    const int nh = n / 2 + 1;
    const int64_t nn = static_cast<int64_t>(n) * n;
    double* ux = work;
    double* uy = work + nn;
    double2* fx = reinterpret_cast<double2*>(work + 2 * nn);
    double2* fy = fx + static_cast<int64_t>(n) * nh;
    int rc = launch_moments(L, state, nullptr, ux, uy, nullptr);
    if (rc) return rc;
    hipfftHandle plan = reinterpret_cast<hipfftHandle>(*plan_slot);
    if (!plan) {
        if (hipfftPlan2d(&plan, n, n, HIPFFT_D2Z) != HIPFFT_SUCCESS) return -2;
        *plan_slot = reinterpret_cast<void*>(plan);
    }
    if (fft_fail(hipfftSetStream(plan, L.stream))) return -2;
    if (fft_fail(hipfftExecD2Z(plan, ux, reinterpret_cast<hipfftDoubleComplex*>(fx)))) return -2;
    if (fft_fail(hipfftExecD2Z(plan, uy, reinterpret_cast<hipfftDoubleComplex*>(fy)))) return -2;
    const int nb = (kmax + 1 + 255) / 256;
    if (ek) k_zero<<<dim3(nb), dim3(256), 0, L.stream>>>(ek, kmax + 1);
    if (zk) k_zero<<<dim3(nb), dim3(256), 0, L.stream>>>(zk, kmax + 1);
    const double scale = 0.5 / (static_cast<double>(nn) * static_cast<double>(nn));
    const double ku = 2.0 * M_PI / n;
    const int64_t total = static_cast<int64_t>(n) * nh;
    const int64_t want = (total + 255) / 256;
    const unsigned grid = static_cast<unsigned>(want < 8192 ? want : 8192);
    k_shells<<<dim3(grid), dim3(256), 0, L.stream>>>(fx, fy, n, nh, kmax, scale, ku * ku, ek, zk);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

void destroy_spectra_plan(void* plan) {
    if (plan) (void)hipfftDestroy(reinterpret_cast<hipfftHandle>(plan));
}

}  // namespace kbc
