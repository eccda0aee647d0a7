/*
 * kbc_oracle_adj.c -- FP64 CPU oracle for the discrete adjoint of the lattice
 * step and of the initial state.
 *
 * TEST INFRASTRUCTURE ONLY (see kbc_oracle.h).
 *
 * The adjoint of a step is, by definition, the transpose of its Jacobian
 * applied to the adjoint of the next state.  The oracle forms that Jacobian
 * per node by complex-step differentiation of the very same collision code
 * (kbc_oracle_node.inc compiled with double complex): for a real-analytic
 * map C, Im C(f + i h e_j) / h = dC/df_j + O(h^2), with no subtractive
 * cancellation, so h = 1e-30 gives the derivative to rounding.  The stabiliser
 * gamma(f) is differentiated with the rest of the collision; on the guarded
 * branch (gamma = 2) it is a constant.
 *
 * With push streaming f^{n+1}_i(x + v_i) = C_i(f^n(x)), the adjoint of a loss
 * L(f^{n+1}) with respect to f^n is
 *   lam^n_j(x) = sum_i lam^{n+1}_i(x + v_i) dC_i/df_j(f^n(x)),
 * and the per-node contribution to dL/dbeta is
 *   sum_i lam^{n+1}_i(x + v_i) dC_i/dbeta(f^n(x)).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "kbc_oracle_internal.h"

#define NODE_T double complex
#define NODE_FN(name) cnode_##name
#define NODE_LOG clog
#include "kbc_oracle_node.inc"
#undef NODE_T
#undef NODE_FN
#undef NODE_LOG

static const double CSTEP = 1e-30;

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

/* J[i * 9 + j] = dC_i / df_j and dbeta[i] = dC_i / dbeta at the state f. */
void orc_node_jacobian(const orc_params* p, const double f[ORC_Q], double J[ORC_Q * ORC_Q],
                       double dbeta[ORC_Q])
{
    double complex fc[ORC_Q], out[ORC_Q];
    for (int j = 0; j < ORC_Q; ++j) {
        for (int i = 0; i < ORC_Q; ++i) fc[i] = f[i];
        fc[j] += CSTEP * I;
        cnode_collide(p, p->beta, fc, out);
        for (int i = 0; i < ORC_Q; ++i) J[i * ORC_Q + j] = cimag(out[i]) / CSTEP;
    }
    if (dbeta) {
        for (int i = 0; i < ORC_Q; ++i) fc[i] = f[i];
        cnode_collide(p, p->beta + CSTEP * I, fc, out);
        for (int i = 0; i < ORC_Q; ++i) dbeta[i] = cimag(out[i]) / CSTEP;
    }
}

int orc_adjoint_step(const orc_params* p, const double* f, const double* lam_next,
                     double* lam, double* dbeta)
{
    if (check(p) || !f || !lam_next || !lam || lam == lam_next) return -1;
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long n = (long)y * nx + x;
            double fl[ORC_Q], J[ORC_Q * ORC_Q], db[ORC_Q], mu[ORC_Q];
            for (int i = 0; i < ORC_Q; ++i) {
                fl[i] = f[i * N + n];
                const int xs = orc_wrap(x + ORC_CX[i], nx);
                const int ys = orc_wrap(y + ORC_CY[i], ny);
                mu[i] = lam_next[i * N + (long)ys * nx + xs];
            }
            orc_node_jacobian(p, fl, J, db);
            double sb = 0.0;
            for (int j = 0; j < ORC_Q; ++j) {
                double s = 0.0;
                for (int i = 0; i < ORC_Q; ++i) s += mu[i] * J[i * ORC_Q + j];
                lam[j * N + n] = s;
            }
            for (int i = 0; i < ORC_Q; ++i) sb += mu[i] * db[i];
            if (dbeta) dbeta[n] = sb;
        }
    }
    return 0;
}

/* Adjoint of orc_init (modes ORC_INIT_EQ and ORC_INIT_GRAD_CD, uniform density
 * rho0): given lam0 = dL/df^0, returns dL/du_x, dL/du_y per node and the
 * per-node contribution of the initial state to dL/dbeta (through Pi^(1)).
 * The central-difference stencil d_a u_b(x) = (u_b(x + e_a) - u_b(x - e_a)) / 2
 * is transposed explicitly; the pointwise derivatives of Grad's populations are
 * taken by complex step. */
int orc_init_adjoint(const orc_params* p, double rho0, const double* ux, const double* uy,
                     int32_t mode, const double* lam0, double* gux, double* guy,
                     double* dbeta)
{
    if (check(p) || !ux || !uy || !lam0 || !gux || !guy) return -1;
    if (mode != ORC_INIT_EQ && mode != ORC_INIT_GRAD_CD) return -1;
    const int nx = p->nx, ny = p->ny;
    const long N = (long)nx * ny;
    /* P[ab][n] = sum_i lam0_i(n) dG_i/d(d_a u_b)(n), ab = 2 a + b */
    double* P = calloc((size_t)4 * N, sizeof(double));
    if (!P) return -3;
#pragma omp parallel for num_threads(nthreads(p)) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            const long n = (long)y * nx + x;
            double complex du[2][2] = {{0, 0}, {0, 0}};
            double complex out[ORC_Q];
            if (mode == ORC_INIT_GRAD_CD) {
                const long xp = (long)y * nx + orc_wrap(x + 1, nx);
                const long xm = (long)y * nx + orc_wrap(x - 1, nx);
                const long yp = (long)orc_wrap(y + 1, ny) * nx + x;
                const long ym = (long)orc_wrap(y - 1, ny) * nx + x;
                du[0][0] = 0.5 * (ux[xp] - ux[xm]);
                du[1][0] = 0.5 * (ux[yp] - ux[ym]);
                du[0][1] = 0.5 * (uy[xp] - uy[xm]);
                du[1][1] = 0.5 * (uy[yp] - uy[ym]);
            }
            /* pointwise derivatives in u_x, u_y and beta */
            double d[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k) {
                double complex cux = ux[n], cuy = uy[n], cb = p->beta;
                if (k == 0) cux += CSTEP * I;
                if (k == 1) cuy += CSTEP * I;
                if (k == 2) cb += CSTEP * I;
                if (mode == ORC_INIT_EQ)
                    cnode_equilibrium(rho0, cux, cuy, out);
                else
                    cnode_grad_populations(rho0, cux, cuy, du, cb, out);
                double s = 0.0;
                for (int i = 0; i < ORC_Q; ++i) s += lam0[i * N + n] * cimag(out[i]) / CSTEP;
                d[k] = s;
            }
            gux[n] = d[0];
            guy[n] = d[1];
            if (dbeta) dbeta[n] = d[2];
            if (mode == ORC_INIT_GRAD_CD) {
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        double complex dd[2][2];
                        memcpy(dd, du, sizeof dd);
                        dd[a][b] += CSTEP * I;
                        cnode_grad_populations(rho0, ux[n], uy[n], dd, p->beta, out);
                        double s = 0.0;
                        for (int i = 0; i < ORC_Q; ++i)
                            s += lam0[i * N + n] * cimag(out[i]) / CSTEP;
                        P[(long)(2 * a + b) * N + n] = s;
                    }
            }
        }
    }
    if (mode == ORC_INIT_GRAD_CD) {
        /* transpose of d_a u_b(x) = (u_b(x + e_a) - u_b(x - e_a)) / 2:
         * dL/du_b(y) += (P_ab(y - e_a) - P_ab(y + e_a)) / 2 */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const long n = (long)y * nx + x;
                const long xp = (long)y * nx + orc_wrap(x + 1, nx);
                const long xm = (long)y * nx + orc_wrap(x - 1, nx);
                const long yp = (long)orc_wrap(y + 1, ny) * nx + x;
                const long ym = (long)orc_wrap(y - 1, ny) * nx + x;
                /* a = x (index 0), a = y (index 1); b = x -> gux, b = y -> guy */
                gux[n] += 0.5 * (P[0 * N + xm] - P[0 * N + xp]) + 0.5 * (P[2 * N + ym] - P[2 * N + yp]);
                guy[n] += 0.5 * (P[1 * N + xm] - P[1 * N + xp]) + 0.5 * (P[3 * N + ym] - P[3 * N + yp]);
            }
    }
    free(P);
    return 0;
}
