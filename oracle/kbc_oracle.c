/*
 * kbc_oracle.c -- FP64 CPU oracle: node functions, lattice step, initial
 * state, moments and diagnostics.
 *
 * TEST INFRASTRUCTURE ONLY (see kbc_oracle.h): loaded by the test suite, the
 * smoke check and the benchmark's CPU-baseline leg, never by the product path.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -fopenmp -fno-fast-math
 *        -ffp-contract=off (oracle/build.py).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "kbc_oracle_internal.h"

#define NODE_T double
#define NODE_FN(name) rnode_##name
#define NODE_LOG log
#include "kbc_oracle_node.inc"
#undef NODE_T
#undef NODE_FN
#undef NODE_LOG

static int nthreads(const orc_params* p) { return p->threads > 0 ? p->threads : 1; }

static int check(const orc_params* p)
{
    if (!p || p->nx < 1 || p->ny < 1) return -1;
    if (!(p->beta > 0.0 && p->beta <= 1.0)) return -1;
    if (p->collision != ORC_LBGK && p->collision != ORC_KBC) return -1;
    if (p->variant < ORC_KBC_A || p->variant > ORC_KBC_D) return -1;
    if (p->gamma_mode < ORC_GAMMA_ESTIMATE || p->gamma_mode > ORC_GAMMA_EXACT) return -1;
    return 0;
}

/* ---------------------------------------------------------------- constants */

double orc_cs2(void) { return ORC_CS2; }

void orc_velocities(int32_t cx[ORC_Q], int32_t cy[ORC_Q])
{
    for (int i = 0; i < ORC_Q; ++i) {
        cx[i] = ORC_CX[i];
        cy[i] = ORC_CY[i];
    }
}

void orc_weights(double W[ORC_Q])
{
    for (int i = 0; i < ORC_Q; ++i) W[i] = orc_weight(i);
}

/* ----------------------------------------------------------- node functions */

void orc_node_equilibrium(double rho, double ux, double uy, double feq[ORC_Q])
{
    rnode_equilibrium(rho, ux, uy, feq);
}

void orc_node_natural(const double f[ORC_Q], double r[ORC_Q]) { rnode_natural_raw(f, r); }

void orc_node_central(const double f[ORC_Q], double ct[6])
{
    double r[ORC_Q];
    rnode_natural_raw(f, r);
    rnode_central(f, r[0], r[1] / r[0], r[2] / r[0], ct);
}

void orc_node_central_to_natural(double ux, double uy, const double ct[6], int32_t kin,
                                 double nat[6])
{
    rnode_central_to_natural(ux, uy, ct, kin, nat);
}

void orc_node_populations(const double r[ORC_Q], double f[ORC_Q]) { rnode_populations(r, f); }

void orc_node_split(int32_t variant, const double f[ORC_Q], double k[ORC_Q], double s[ORC_Q],
                    double h[ORC_Q])
{
    rnode_split(variant, f, k, s, h);
}

void orc_node_deviations(int32_t variant, const double f[ORC_Q], double ds[ORC_Q],
                         double dh[ORC_Q], double out[3])
{
    double r[ORC_Q], feq[ORC_Q];
    rnode_natural_raw(f, r);
    rnode_equilibrium(r[0], r[1] / r[0], r[2] / r[0], feq);
    double k[ORC_Q], s[ORC_Q], h[ORC_Q], keq[ORC_Q], seq[ORC_Q], heq[ORC_Q];
    rnode_split(variant, f, k, s, h);
    rnode_split(variant, feq, keq, seq, heq);
    for (int i = 0; i < ORC_Q; ++i) {
        ds[i] = s[i] - seq[i];
        dh[i] = h[i] - heq[i];
    }
    out[0] = rnode_escalar(ds, dh, feq);
    out[1] = rnode_escalar(dh, dh, feq);
    out[2] = rnode_escalar(ds, ds, feq);
}

double orc_node_collide(const orc_params* p, const double f[ORC_Q], double out[ORC_Q])
{
    return rnode_collide(p, p->beta, f, out);
}

double orc_node_result1(const orc_params* p, const double f[ORC_Q], double gamma)
{
    double ds[ORC_Q], dh[ORC_Q], prod[3], r[ORC_Q], feq[ORC_Q], dF;
    orc_node_deviations(p->variant, f, ds, dh, prod);
    rnode_natural_raw(f, r);
    rnode_equilibrium(r[0], r[1] / r[0], r[2] / r[0], feq);
    return rnode_result1(gamma, p->beta, ds, dh, feq, &dF);
}

void orc_node_grad(double rho, double ux, double uy, const double du[4], double beta,
                   double f[ORC_Q])
{
    /* du = (d_x u_x, d_y u_x, d_x u_y, d_y u_y); g[a][b] = d_a u_b */
    const double g[2][2] = {{du[0], du[2]}, {du[1], du[3]}};
    rnode_grad_populations(rho, ux, uy, g, beta, f);
}

/* --------------------------------------------------------- lattice functions */

/* Initial populations: the equilibrium, or Grad's approximation with
 * Pi = Pi^eq + Pi^(1) (initialisation of the Green-Taylor vortex section)
 * whose velocity gradients come from second-order central differences of the
 * given field (decaying-turbulence section) or from the caller. */
int orc_init(const orc_params* p, const double* rho, double rho0, const double* ux,
             const double* uy, const double* grad, int32_t mode, double* f)
{
    if (check(p) || !ux || !uy || !f) return -1;
    if (mode < ORC_INIT_EQ || mode > ORC_INIT_GRAD_GIVEN) return -1;
    if (mode == ORC_INIT_GRAD_GIVEN && !grad) return -1;
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long n = (long)y * nx + x;
            const double r = rho ? rho[n] : rho0;
            double fl[ORC_Q];
            if (mode == ORC_INIT_EQ) {
                rnode_equilibrium(r, ux[n], uy[n], fl);
            } else {
                double du[4];
                if (mode == ORC_INIT_GRAD_GIVEN) {
                    for (int k = 0; k < 4; ++k) du[k] = grad[k * N + n];
                } else {
                    const long xp = (long)y * nx + orc_wrap(x + 1, nx);
                    const long xm = (long)y * nx + orc_wrap(x - 1, nx);
                    const long yp = (long)orc_wrap(y + 1, ny) * nx + x;
                    const long ym = (long)orc_wrap(y - 1, ny) * nx + x;
                    du[0] = 0.5 * (ux[xp] - ux[xm]);
                    du[1] = 0.5 * (ux[yp] - ux[ym]);
                    du[2] = 0.5 * (uy[xp] - uy[xm]);
                    du[3] = 0.5 * (uy[yp] - uy[ym]);
                }
                orc_node_grad(r, ux[n], uy[n], du, p->beta, fl);
            }
            for (int i = 0; i < ORC_Q; ++i) f[i * N + n] = fl[i];
        }
    }
    return 0;
}

/* One time step of eq. (Egeneral): collide at every node, then push the
 * post-collision population f_i' to x + v_i with periodic wrap-around. */
int orc_step(const orc_params* p, const double* fin, double* fout, double* gamma)
{
    if (check(p) || !fin || !fout || fin == fout) return -1;
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long n = (long)y * nx + x;
            double fl[ORC_Q], out[ORC_Q];
            for (int i = 0; i < ORC_Q; ++i) fl[i] = fin[i * N + n];
            const double g = rnode_collide(p, p->beta, fl, out);
            if (gamma) gamma[n] = g;
            for (int i = 0; i < ORC_Q; ++i) {
                const int xd = orc_wrap(x + ORC_CX[i], nx);
                const int yd = orc_wrap(y + ORC_CY[i], ny);
                fout[i * N + (long)yd * nx + xd] = out[i];
            }
        }
    }
    return 0;
}

int orc_run(const orc_params* p, double* f, double* work, int32_t nsteps)
{
    if (check(p) || !f || !work || nsteps < 0) return -1;
    double *a = f, *b = work;
    for (int s = 0; s < nsteps; ++s) {
        if (orc_step(p, a, b, NULL)) return -1;
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * ORC_Q * (size_t)p->nx * (size_t)p->ny);
    return 0;
}

/* Round to the nearest binary16 value, ties to even, written from the
 * format's definition: 11 significant bits for normal numbers, a fixed
 * spacing of 2^-24 below the smallest normal 2^-14, and overflow to
 * infinity from 65520 (the midpoint above the largest finite value 65504). */
double orc_round_f16(double x)
{
    if (x != x || x == 0.0 || isinf(x)) return x;
    int e;
    (void)frexp(x, &e);                  /* |x| in [2^(e-1), 2^e) */
    int q = e - 11;                      /* spacing of binary16 values there */
    if (q < -24) q = -24;
    const double r = ldexp(rint(ldexp(x, -q)), q);   /* rint: nearest, ties to even */
    return fabs(r) > 65504.0 ? copysign(INFINITY, x) : r;
}

int orc_round_storage(const orc_params* p, double rho0, int32_t storage, double* f)
{
    if (check(p) || !f || storage < ORC_STORE_F64 || storage > ORC_STORE_F16) return -1;
    if (storage == ORC_STORE_F64) return 0;
    const long N = (long)p->nx * p->ny;
    for (int i = 0; i < ORC_Q; ++i) {
        const double w = orc_weight(i) * rho0;
        const int s = (i == 0) ? 1 : (i < 5 ? 3 : 5);
        for (long n = 0; n < N; ++n) {
            const double g = f[i * N + n] - w;
            const double r = (storage == ORC_STORE_F32) ? (double)(float)g
                                                        : ldexp(orc_round_f16(ldexp(g, s)), -s);
            f[i * N + n] = w + r;
        }
    }
    return 0;
}

int orc_run_stored(const orc_params* p, double rho0, int32_t storage, double* f, double* work, int32_t nsteps)
{
    if (check(p) || !f || !work || nsteps < 0) return -1;
    double *a = f, *b = work;
    for (int s = 0; s < nsteps; ++s) {
        if (orc_step(p, a, b, NULL)) return -1;
        if (orc_round_storage(p, rho0, storage, b)) return -1;
        double* t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, sizeof(double) * ORC_Q * (size_t)p->nx * (size_t)p->ny);
    return 0;
}

int orc_moments(const orc_params* p, const double* f, double* rho, double* ux, double* uy)
{
    if (check(p) || !f) return -1;
    const long N = (long)p->nx * p->ny;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double fl[ORC_Q], r[ORC_Q];
        for (int i = 0; i < ORC_Q; ++i) fl[i] = f[i * N + n];
        rnode_natural_raw(fl, r);
        if (rho) rho[n] = r[0];
        if (ux) ux[n] = r[1] / r[0];
        if (uy) uy[n] = r[2] / r[0];
    }
    return 0;
}

/* gamma that the next collision at each node uses (2 for LBGK) */
int orc_gamma_field(const orc_params* p, const double* f, double* gamma)
{
    if (check(p) || !f || !gamma) return -1;
    const long N = (long)p->nx * p->ny;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (long n = 0; n < N; ++n) {
        double fl[ORC_Q], out[ORC_Q];
        for (int i = 0; i < ORC_Q; ++i) fl[i] = f[i * N + n];
        gamma[n] = rnode_collide(p, p->beta, fl, out);
    }
    return 0;
}

/* Mean and spatial standard deviation of a field, in row-major order. */
static void mean_std(const double* v, long N, double* mean, double* sd)
{
    double s = 0.0;
    for (long n = 0; n < N; ++n) s += v[n];
    const double m = s / (double)N;
    double q = 0.0;
    for (long n = 0; n < N; ++n) q += (v[n] - m) * (v[n] - m);
    *mean = m;
    *sd = sqrt(q / (double)N);
}

/* Totals and spatial statistics of a state: mass and momentum; energy
 * e = |u|^2 / 2, enstrophy z = omega^2 / 2 and palinstrophy |grad omega|^2 / 2
 * (means and spatial standard deviations), with omega = d_x u_y - d_y u_x and
 * its gradient from second-order central differences; mean entropy per node
 * from eq. (S); mean and standard deviation of gamma; counts of nodes with a
 * non-finite population and with a non-positive equilibrium population;
 * standard deviation of the density. */
int orc_diagnostics(const orc_params* p, const double* f, double out[ORC_NDIAG])
{
    if (check(p) || !f || !out) return -1;
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    double* rho = malloc(sizeof(double) * N);
    double* ux = malloc(sizeof(double) * N);
    double* uy = malloc(sizeof(double) * N);
    double* w = malloc(sizeof(double) * N);
    double* tmp = malloc(sizeof(double) * N);
    double* gam = malloc(sizeof(double) * N);
    if (!rho || !ux || !uy || !w || !tmp || !gam) {
        free(rho); free(ux); free(uy); free(w); free(tmp); free(gam);
        return -3;
    }
    for (int k = 0; k < ORC_NDIAG; ++k) out[k] = 0.0;
    orc_moments(p, f, rho, ux, uy);
    orc_gamma_field(p, f, gam);

    double mass = 0.0, jx = 0.0, jy = 0.0, S = 0.0;
    long nonfinite = 0, feqneg = 0;
    for (long n = 0; n < N; ++n) {
        double fl[ORC_Q], feq[ORC_Q];
        int finite = 1;
        for (int i = 0; i < ORC_Q; ++i) {
            fl[i] = f[i * N + n];
            if (!isfinite(fl[i])) finite = 0;
        }
        if (!finite) ++nonfinite;
        mass += rho[n];
        jx += rho[n] * ux[n];
        jy += rho[n] * uy[n];
        rnode_equilibrium(rho[n], ux[n], uy[n], feq);
        int neg = 0;
        for (int i = 0; i < ORC_Q; ++i)
            if (!(feq[i] > 0.0)) neg = 1;
        if (neg) ++feqneg;
        double s = 0.0;
        for (int i = 0; i < ORC_Q; ++i) s -= fl[i] * log(fl[i] / orc_weight(i));
        S += s;
    }
    out[ORC_D_MASS] = mass;
    out[ORC_D_JX] = jx;
    out[ORC_D_JY] = jy;
    out[ORC_D_S] = S / (double)N;
    out[ORC_D_NONFINITE] = (double)nonfinite;
    out[ORC_D_FEQ_NONPOS] = (double)feqneg;
    mean_std(rho, N, &out[ORC_D_UNUSED], &out[ORC_D_RHO_STD]);
    out[ORC_D_UNUSED] = 0.0;

    for (long n = 0; n < N; ++n) tmp[n] = 0.5 * (ux[n] * ux[n] + uy[n] * uy[n]);
    mean_std(tmp, N, &out[ORC_D_E], &out[ORC_D_E_STD]);

    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long xp = (long)y * nx + orc_wrap(x + 1, nx);
            const long xm = (long)y * nx + orc_wrap(x - 1, nx);
            const long yp = (long)orc_wrap(y + 1, ny) * nx + x;
            const long ym = (long)orc_wrap(y - 1, ny) * nx + x;
            w[(long)y * nx + x] = 0.5 * (uy[xp] - uy[xm]) - 0.5 * (ux[yp] - ux[ym]);
        }
    for (long n = 0; n < N; ++n) tmp[n] = 0.5 * w[n] * w[n];
    mean_std(tmp, N, &out[ORC_D_Z], &out[ORC_D_Z_STD]);

    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long xp = (long)y * nx + orc_wrap(x + 1, nx);
            const long xm = (long)y * nx + orc_wrap(x - 1, nx);
            const long yp = (long)orc_wrap(y + 1, ny) * nx + x;
            const long ym = (long)orc_wrap(y - 1, ny) * nx + x;
            const double gx = 0.5 * (w[xp] - w[xm]);
            const double gy = 0.5 * (w[yp] - w[ym]);
            tmp[(long)y * nx + x] = 0.5 * (gx * gx + gy * gy);
        }
    mean_std(tmp, N, &out[ORC_D_P], &out[ORC_D_P_STD]);
    mean_std(gam, N, &out[ORC_D_GAMMA], &out[ORC_D_GAMMA_STD]);

    free(rho); free(ux); free(uy); free(w); free(tmp); free(gam);
    return 0;
}
