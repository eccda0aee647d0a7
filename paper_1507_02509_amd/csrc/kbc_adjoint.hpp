// kbc_adjoint.hpp -- reverse-mode derivative (vector-Jacobian product) of the
// per-node collision of kbc_device.hpp.
//
// Given the deviations g of a pre-collision state and the adjoint mu of the
// post-collision deviations, collide_vjp returns lam = J^T mu, J = dg'/dg, and
// the node's contribution mu . dg'/dbeta.  The stabiliser gamma(f) of
// eq. (result21) is by default differentiated with the rest of the collision through
// <ds|dh>, <dh|dh> and the entropic weights 1/feq; where the denominator guard
// selects gamma = 2 it is a constant.  The exact stabiliser (the root of
// eq. (result1), found by Newton's method) is differentiated by the implicit
// function theorem at the root: for F(gamma; ds, dh, 1/feq, beta) = 0,
// d gamma = -(dF at fixed gamma) / F'(gamma).  The forward quantities of the KBC
// collision come from kbc_forward(), the code collide() runs, so both take the
// same guard decisions on the same values; the chain rule then runs through
// them in reverse order.
#pragma once

#include "kbc_device.hpp"

namespace kbc {

// Adjoint of the map from a zero-mass, zero-momentum moment vector (T, N, Pi,
// Q_xyy, Q_yxx, A) to populations, eq. (momentsD2Q9) (the map kbc_forward
// applies to the 1/4-scaled moments): moment adjoints from population
// adjoints pb.
template <typename R>
__device__ __forceinline__ void pop_to_moments_adj(const R (&pb)[9], R& Tb, R& Nb, R& Pb, R& Qxb,
                                                   R& Qyb, R& Ab) {
    const R q = R(0.25), h = R(0.5);
    const R ax = pb[1] + pb[3], ay = pb[2] + pb[4];
    const R dg = (pb[5] + pb[7]) + (pb[6] + pb[8]);
    Tb = q * (ax + ay) - pb[0];
    Nb = q * (ax - ay);
    Pb = q * ((pb[5] + pb[7]) - (pb[6] + pb[8]));
    Qxb = h * (pb[3] - pb[1]) + q * ((pb[5] - pb[7]) - (pb[6] - pb[8]));
    Qyb = h * (pb[4] - pb[2]) + q * ((pb[5] - pb[7]) + (pb[6] - pb[8]));
    Ab = pb[0] - h * (ax + ay) + q * dg;
}

// FROZEN = true holds gamma at its forward value (the derivative of the map
// with the stabiliser treated as a per-node constant).
template <typename R, int COLL, int VAR, int GM, bool FROZEN = false>
__device__ __forceinline__ void collide_vjp(const R (&g)[9], const R (&mu)[9], const Coef<R>& K,
                                            R (&lam)[9], R& dbeta) {
    // adjoints of rho - rho0, j and u collected below
    R drb = R(0), jxb = R(0), jyb = R(0), uxb = R(0), uyb = R(0);
    // adjoints of the raw sums of g: sum c_x^2 g, sum c_y^2 g, sum c_x c_y g,
    // sum c_x c_y^2 g, sum c_x^2 c_y g, sum c_x^2 c_y^2 g
    R Sxxb = R(0), Syyb = R(0), Sxyb = R(0), Qxrb = R(0), Qyrb = R(0), Arb = R(0);
    R ir, ux, uy;

    if constexpr (COLL == LBGK) {
        const R s13 = g[1] + g[3], s24 = g[2] + g[4], s57 = g[5] + g[7], s68 = g[6] + g[8];
        const R d13 = g[1] - g[3], d24 = g[2] - g[4], d57 = g[5] - g[7], d68 = g[6] - g[8];
        const R dr = (g[0] + (s57 + s68)) + (s13 + s24);
        const R jx = d13 + (d57 - d68), jy = d24 + (d57 + d68);
        const R rho = K.rho0 + dr;
        ir = rcpR(rho);
        ux = jx * ir;
        uy = jy * ir;
        const R uxx = ux * ux, uyy = uy * uy, u2 = uxx + uyy;
        const R upv = ux + uy, umv = ux - uy;
        // g' = g - 2 beta (g - feqd); feqd_i = W_i [ (rho - rho0) + rho e_i ]
        const R c0 = R(-1.5) * u2;
        const R bx = fmaR(R(4.5), uxx, c0), by = fmaR(R(4.5), uyy, c0);
        const R bp = fmaR(R(4.5) * upv, upv, c0), bm = fmaR(R(4.5) * umv, umv, c0);
        R e[9];
        e[0] = c0;
        e[1] = fmaR(R(3), ux, bx);
        e[3] = fmaR(R(-3), ux, bx);
        e[2] = fmaR(R(3), uy, by);
        e[4] = fmaR(R(-3), uy, by);
        e[5] = fmaR(R(3), upv, bp);
        e[7] = fmaR(R(-3), upv, bp);
        e[8] = fmaR(R(3), umv, bm);
        e[6] = fmaR(R(-3), umv, bm);
        const R tb = R(2) * K.beta;
        R db = R(0);
        // feqd_i depends on dr (directly and through rho) and on u through e_i:
        // d feqd_i / d dr = W_i (1 + e_i), d e_i / d u = 3 c_i + 9 (c_i.u) c_i - 3 u
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const R feqd = R(weight(i)) * fmaR(rho, e[i], dr);
            db = fmaR(mu[i], g[i] - feqd, db);
            const R fb = tb * mu[i];                 // adjoint of feqd_i
            const R wr = R(weight(i)) * fb;
            drb = fmaR(wr, R(1) + e[i], drb);
            const R cu = R(kCx[i]) * ux + R(kCy[i]) * uy;
            const R eb = wr * rho;                   // adjoint of e_i
            uxb = fmaR(eb, fmaR(R(9) * cu, R(kCx[i]), fmaR(R(-3), ux, R(3) * R(kCx[i]))), uxb);
            uyb = fmaR(eb, fmaR(R(9) * cu, R(kCy[i]), fmaR(R(-3), uy, R(3) * R(kCy[i]))), uyb);
            lam[i] = (R(1) - tb) * mu[i];
        }
        dbeta = R(-2) * db;
    } else {
        KbcNode<R> n;
        kbc_forward<R, VAR, (GM == GEXACT ? GEST : GM)>(g, K, n);
        const R third = R(1.0 / 3.0), ninth = R(1.0 / 9.0);
        ir = n.ir;
        ux = n.ux;
        uy = n.uy;
        const R jx = n.jx, jy = n.jy, uxx = n.uxx, uyy = n.uyy, u2 = n.u2;
        const R dN = n.dN, dP = n.dP, tT = n.tT;
        const R(&ds)[9] = n.ds;
        const R(&dh)[9] = n.dh;
        const R(&w)[9] = n.w;
        const R ratio = n.ratio, bsum = n.b;
        const bool active = n.active;
        R gam = n.gam;
        if constexpr (GM == GEXACT) {
            if (active) gam = exact_gamma<R>(gam, ds, dh, w, ir, K);
        }

        // --------------------------------------------------------- reverse
        // (mul + add pairs below may fuse: nothing else is computed from
        // these values, so there is no bitwise contract to keep)
        {
#pragma clang fp contract(fast)
            // g'_i = g_i - 2 beta ds_i - beta gamma dh_i
            // d g'_i / d beta = -(2 ds_i + gamma dh_i): mu . dg'/dbeta is
            // -(2 mu.ds + gamma mu.dh), and mu.dh also gives gamma's adjoint
            R dsb[9], dhb[9];
            R mdh = R(0), mds = R(0);
            const R tb = R(2) * K.beta, bg = K.beta * gam;
    #pragma unroll
            for (int i = 0; i < 9; ++i) {
                lam[i] = mu[i];
                dsb[i] = -tb * mu[i];
                dhb[i] = -bg * mu[i];
                mdh = fmaR(mu[i], dh[i], mdh);
                mds = fmaR(mu[i], ds[i], mds);
            }
            R gamb = -K.beta * mdh;
            dbeta = -fmaR(gam, mdh, R(2) * mds);
            if constexpr (GM != GFIX && !FROZEN) {
                if (active) {
                    R wd[9];                                   // adjoint of d_i
                    if constexpr (GM == GEXACT) {
                    // F = sum_i dh_i ln(1 + x_i), x_i = y_i wr_i,
                    // y_i = (1 - beta gamma) dh_i - (2 beta - 1) ds_i, wr_i = w_i / rho:
                    // dF/d dh_i = ln(1 + x_i) + (1 - beta gamma) dh_i wr_i / (1 + x_i),
                    // dF/d ds_i = -(2 beta - 1) dh_i wr_i / (1 + x_i),
                    // dF/d wr_i = dh_i y_i / (1 + x_i),
                    // dF/d beta = -sum_i dh_i (gamma dh_i + 2 ds_i) wr_i / (1 + x_i),
                    // F'(gamma) = -beta sum_i dh_i^2 wr_i / (1 + x_i)
                    const R om = R(1) - K.beta * gam, tbm1 = R(2) * K.beta - R(1);
                    R wr[9], y[9], r[9], lg[9];
                    R D = R(0);
                    bool ok = true;
    #pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        wr[i] = w[i] * ir;
                        y[i] = om * dh[i] - tbm1 * ds[i];
                        const R x = y[i] * wr[i];
                        ok = ok && (x > R(-1));
                        r[i] = rcpR(R(1) + x);
                        lg[i] = log1pR(x);
                        D = fmaR(-K.beta * dh[i] * dh[i] * wr[i], r[i], D);
                    }
                    // where the iteration stopped short of a root (an argument
                    // of the logarithm left (0, inf), or F' >= 0) gamma is held
                    const R imp = (ok && D < R(0)) ? -gamb / D : R(0);   // -gamma_bar / F'
                    R irb = R(0), fb = R(0);
    #pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        const R t = dh[i] * wr[i] * r[i];
                        dhb[i] = fmaR(imp, fmaR(om, t, lg[i]), dhb[i]);
                        dsb[i] = fmaR(imp, -tbm1 * t, dsb[i]);
                        const R wrb = imp * dh[i] * y[i] * r[i];
                        irb = fmaR(wrb, w[i], irb);
                        wd[i] = -(wrb * ir) * w[i] * w[i];
                        fb = fmaR(t, fmaR(gam, dh[i], R(2) * ds[i]), fb);
                    }
                    dbeta = fmaR(-imp, fb, dbeta);
                    drb -= irb * ir * ir;                      // ir = 1 / (rho0 + dr)
                    } else {
                    // gamma = 1/beta - (2 - 1/beta) a / b
                    const R ib2 = K.inv_beta * K.inv_beta;
                    dbeta = fmaR(gamb, -(R(1) + ratio) * ib2, dbeta);
                    const R rb = -K.two_m_inv_beta * gamb;     // adjoint of a / b
                    const R ab = rb * rcpR(bsum);              // adjoint of a
                    const R bb = -ab * ratio;                  // adjoint of b = -rb a / b^2
    #pragma unroll
                    for (int i = 0; i < 9; ++i) {
                        // a = sum ds dh w, b = sum dh dh w (c enters the guard only);
                        // the adjoint of w_i is dh_i (ab ds_i + bb dh_i), w_i = 1 / d_i
                        const R hw = dh[i] * w[i];
                        const R bh = bb * dh[i];
                        const R t = fmaR(ab, ds[i], bh);
                        dsb[i] = fmaR(ab, hw, dsb[i]);
                        dhb[i] = fmaR(t + bh, w[i], dhb[i]);
                        wd[i] = -(hw * t) * w[i];
                    }
                    }
                    // d_i in u: 4/9 - 2|u|^2/3; 1/9 - |u|^2/6 + u_a^2/2 +- u_a/3 (axes);
                    // 1/36 + |u|^2/12 +- u_x u_y/4 + (c.u)/12 (diagonals)
                    const R p57 = wd[5] + wd[7], p68 = wd[6] + wd[8];
                    const R e0 = fmaR(R(1.0 / 6.0), p57 + p68, R(-4.0 / 3.0) * wd[0]);
                    const R p13 = wd[1] + wd[3], p24 = wd[2] + wd[4];
                    const R cx = fmaR(R(2.0 / 3.0), p13, fmaR(R(-1.0 / 3.0), p24, e0));
                    const R cy = fmaR(R(-1.0 / 3.0), p13, fmaR(R(2.0 / 3.0), p24, e0));
                    const R dq = R(0.25) * (p57 - p68);
                    const R m57 = wd[5] - wd[7], m86 = wd[8] - wd[6];
                    uxb += fmaR(ux, cx, fmaR(uy, dq, fmaR(R(1.0 / 3.0), wd[1] - wd[3], R(1.0 / 12.0) * (m57 + m86))));
                    uyb += fmaR(uy, cy, fmaR(ux, dq, fmaR(R(1.0 / 3.0), wd[2] - wd[4], R(1.0 / 12.0) * (m57 - m86))));
                }
            }
            // ds = P(Ts, dN, dP, Qxs, Qys, As), dh = P(dT - Ts, 0, 0, dQx - Qxs, dQy - Qys, dA - As)
            R sTb, sNb, sPb, sQxb, sQyb, sAb, hTb, hNb, hPb, hQxb, hQyb, hAb;
            pop_to_moments_adj<R>(dsb, sTb, sNb, sPb, sQxb, sQyb, sAb);
            pop_to_moments_adj<R>(dhb, hTb, hNb, hPb, hQxb, hQyb, hAb);
            R dTb = hTb, dNb = sNb, dPb = sPb, dQxb = hQxb, dQyb = hQyb, dAb = hAb;
            const R Tsb = sTb - hTb, Qxsb = sQxb - hQxb, Qysb = sQyb - hQyb, Asb = sAb - hAb;
            if constexpr (VAR == VC) {
                dTb += Tsb;
            } else if constexpr (VAR == VA || VAR == VB) {
                if constexpr (VAR == VA) dTb += Tsb + R(0.5) * (ux * Qxsb + uy * Qysb + u2 * Asb);
                dNb += R(0.5) * (uy * Qysb - ux * Qxsb - (uxx - uyy) * Asb);
                dPb += R(2) * (uy * Qxsb + ux * Qysb) + R(4) * ux * uy * Asb;
                uxb += R(0.5) * (tT - dN) * Qxsb + R(2) * dP * Qysb + (R(4) * uy * dP + ux * (tT - dN)) * Asb;
                uyb += R(2) * dP * Qxsb + R(0.5) * (tT + dN) * Qysb + (R(4) * ux * dP + uy * (tT + dN)) * Asb;
            }
            // dT = dPxx + dPyy, dN = dPxx - dPyy, dP = dPxy
            const R dPxxb = dTb + dNb, dPyyb = dTb - dNb, dPxyb = dPb;
            // moments of g - feq
            Sxxb = dPxxb;
            Syyb = dPyyb;
            Sxyb = dPxyb;
            Qxrb = dQxb;
            Qyrb = dQyb;
            Arb = dAb;
            drb += -(dPxxb + dPyyb) * third - dAb * ninth;
            jxb += -dPxxb * ux - dPxyb * uy - dQxb * third - dAb * ux * third;
            jyb += -dPyyb * uy - dQyb * third - dAb * uy * third;
            uxb += -dPxxb * jx - dAb * jx * third;
            uyb += -dPyyb * jy - dPxyb * jx - dAb * jy * third;
        }
    }
    // u = j / rho, rho = rho0 + dr
    jxb = fmaR(uxb, ir, jxb);
    jyb = fmaR(uyb, ir, jyb);
    drb -= (uxb * ux + uyb * uy) * ir;
    // dr = sum g, j = sum c g, and the raw sums of g:
    // lam_i += drb + c_x jxb + c_y jyb + c_x^2 Sxxb + c_y^2 Syyb + c_x c_y Sxyb
    //          + c_x c_y^2 Qxrb + c_x^2 c_y Qyrb + c_x^2 c_y^2 Arb
    const R ax = drb + Sxxb, ay = drb + Syyb;
    const R dd = (ax + Syyb) + Arb;               // common to the diagonals
    const R px = jxb + Qxrb, py = jyb + Qyrb;
    lam[0] += drb;
    lam[1] += ax + jxb;
    lam[3] += ax - jxb;
    lam[2] += ay + jyb;
    lam[4] += ay - jyb;
    const R dp = dd + Sxyb, dm = dd - Sxyb;
    lam[5] += dp + (px + py);
    lam[7] += dp - (px + py);
    lam[6] += dm - (px - py);
    lam[8] += dm + (px - py);
}

}  // namespace kbc
