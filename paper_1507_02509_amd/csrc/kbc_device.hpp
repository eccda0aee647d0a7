// kbc_device.hpp -- per-node arithmetic of the D2Q9 KBC / LBGK step for gfx950.
//
// The collision works on deviations g_i = f_i - W_i rho0 (the stored form) and
// never forms full populations.  Everything it needs follows from six
// non-equilibrium moments of df = f - feq, which are cheap in deviation form
// because the second-order polynomial equilibrium (eq. Eq) has closed-form
// moments on D2Q9: rho, rho u, Pi^eq = rho cs2 I + rho u u (eq. Peq),
// Q^eq_xyy = rho u_x / 3, Q^eq_yxx = rho u_y / 3 (eq. Qeq) and
// A^eq = rho / 9 + rho |u|^2 / 3.  With T = P_xx + P_yy, N = P_xx - P_yy,
// Pi = P_xy (eq. natmoments1), the shear part ds and the higher-order part dh
// of Table kbc_moment_grouping are populations of a moment vector
// (T, N, Pi, Q_xyy, Q_yxx, A) through eq. (momentsD2Q9); for the central-moment
// models A and B the shear moments are carried to natural ones by the linear
// part of eq. (cm) (at fixed u the central deviations equal the natural ones).
// gamma follows eq. (result21) with the entropic scalar product weighted by
// 1/feq; the common factor 1/rho cancels in the ratio and in the guard.
//
// All floating-point contractions are written out with fma() and the library
// is compiled with -ffp-contract=off, so every launch shape that runs this
// code produces bitwise identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kbc {

enum Coll { LBGK = 0, KBCC = 1 };
enum Var { VA = 0, VB = 1, VC = 2, VD = 3 };
enum GMode { GEST = 0, GFIX = 1, GEXACT = 2 };
enum FormId { F16 = 0, F32 = 1, F64 = 2 };

// D2Q9 velocities, order (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1)
constexpr int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
// lattice weights 4/9, 1/9, 1/36
__host__ __device__ constexpr double weight(int i) { return i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0); }
// binary16 storage scale exponents: ~1/W_i rounded to a power of two
__host__ __device__ constexpr int f16_shift(int i) { return i == 0 ? 1 : (i < 5 ? 3 : 5); }

// ---------------------------------------------------------------- storage forms
template <int FORM> struct Form;

template <> struct Form<F16> {
    using S = _Float16;
    using R = float;
    static constexpr int bytes = 2;
    // v 2^-s as one mixed-precision FMA (binary16 operand, binary32 result;
    // exact: the scale is a power of two).  The +0 addend keeps the FMA from
    // being rewritten as a conversion and a multiply; it maps a stored -0 to
    // +0, which no later sum can tell apart.
    __device__ static __forceinline__ R dec(S v, int i) {
        return __builtin_fmaf(static_cast<float>(v), 1.0f / static_cast<float>(1 << f16_shift(i)), 0.0f);
    }
    __device__ static __forceinline__ S enc(R v, int i) {
        return static_cast<_Float16>(v * static_cast<float>(1 << f16_shift(i)));
    }
    __device__ static __forceinline__ double dec64(S v, int i) {
        return static_cast<double>(static_cast<float>(v)) / static_cast<double>(1 << f16_shift(i));
    }
    // one rounding, double -> binary16 (not through binary32, which would
    // round twice and can land one unit away)
    __device__ static __forceinline__ S enc64(double v, int i) {
        return static_cast<_Float16>(v * static_cast<double>(1 << f16_shift(i)));
    }
};

template <> struct Form<F32> {
    using S = float;
    using R = float;
    static constexpr int bytes = 4;
    __device__ static __forceinline__ R dec(S v, int) { return v; }
    __device__ static __forceinline__ S enc(R v, int) { return v; }
    __device__ static __forceinline__ double dec64(S v, int) { return static_cast<double>(v); }
    __device__ static __forceinline__ S enc64(double v, int) { return static_cast<float>(v); }
};

template <> struct Form<F64> {
    using S = double;
    using R = double;
    static constexpr int bytes = 8;
    __device__ static __forceinline__ R dec(S v, int) { return v; }
    __device__ static __forceinline__ S enc(R v, int) { return v; }
    __device__ static __forceinline__ double dec64(S v, int) { return v; }
    __device__ static __forceinline__ S enc64(double v, int) { return v; }
};

// ------------------------------------------------------------------- arithmetic
__device__ __forceinline__ float fmaR(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaR(double a, double b, double c) { return __builtin_fma(a, b, c); }
// reciprocal: v_rcp_f32 (1 ulp) in FP32; in FP64 v_rcp_f64 refined by two
// Newton steps r <- r + r (1 - a r) (the refinement of the compiler's own
// division, without its scaling and final correction for exact rounding:
// within about an ulp for the positive normal denominators used here, in
// five instructions instead of eleven)
__device__ __forceinline__ float rcpR(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double rcpR(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = __builtin_fma(r, __builtin_fma(-a, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-a, r, 1.0), r);
}
__device__ __forceinline__ float divR(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double divR(double a, double b) { return a * rcpR(b); }

template <typename R> struct Coef {
    R beta;            // relaxation parameter
    R inv_beta;        // 1 / beta
    R two_m_inv_beta;  // 2 - 1 / beta
    R rho0;            // reference density of the deviation storage
    R guard;           // gamma = 2 where <dh|dh> <= guard <ds|ds>
    R gamma_fixed;     // stabiliser for GFIX
};

// ln(1 + x) for x > -1.  FP32: Goldberg's form (D. Goldberg, "What every
// computer scientist should know about floating-point arithmetic", 1991,
// Theorem 4): with u = fl(1 + x), ln(u) x / (u - 1) is accurate to a few
// units in the last place, because the rounding error of 1 + x cancels
// between ln(u) and u - 1; ln(u) comes from the hardware base-2 logarithm
// (about 10 instructions instead of the library's long compensated form).
// FP64 keeps the library log1p.
__device__ __forceinline__ float log1pR(float x) {
    const float u = 1.0f + x;
    const float d = u - 1.0f;
    return d == 0.0f ? x : (__builtin_amdgcn_logf(u) * 0.693147180559945309f) * (x * __builtin_amdgcn_rcpf(d));
}
__device__ __forceinline__ double log1pR(double x) { return log1p(x); }

// Root of the entropy-maximum condition eq. (result1) in gamma,
//   F(gamma) = sum_i dh_i ln(1 + x_i) = 0,
//   x_i = ((1 - beta gamma) dh_i - (2 beta - 1) ds_i) / feq_i,
// by Newton's method from gamma* (its first-order root, eq. (result21)).
// F decreases strictly in gamma while every 1 + x_i > 0, so the root is
// unique; the iteration stops (keeping the current gamma) if an argument of
// the logarithm leaves (0, inf) or F' is not negative, after a step below
// the tolerance of the arithmetic type, after a step that is not at most half
// the previous one (Newton's steps shrink quadratically until rounding noise
// in F takes over, which at a near-equilibrium node lies above the FP32
// tolerance), or after a fixed number of steps.
// 1 / feq_i = w_i / rho with w_i = 1 / (W_i (1 + e_i)); ln(1 + x) is taken
// as log1pR(x), accurate to rounding for the small x of a near-equilibrium
// node.
//
// While every |x_i| of a node is below 1/32 (FP32) or 1/64 (FP64), i.e. near
// equilibrium, ln(1 + x) is its Taylor polynomial, of degree 6 or 10, by
// Horner's rule: six or ten FMAs against the general form's logarithm,
// reciprocal and guard (FP32) or the library log1p (FP64).  The truncation is
// below 1.4e-10 and 8e-20 relative, the evaluation within 1.2e-7 and an ulp.  The
// choice is the node's own (all nine of its arguments small), so a node's
// result does not depend on which nodes share its wave; a wave skips the
// general form when none of its nodes needs it.  The quantities that do not change
// with gamma (dh_i / feq_i, (2 beta - 1) ds_i / feq_i, -beta dh_i^2 / feq_i)
// are formed once, before the iteration.
__device__ __forceinline__ float log1p_small(float x) {
    float p = fmaR(x, -1.0f / 6.0f, 0.2f);
    p = fmaR(x, p, -0.25f);
    p = fmaR(x, p, 1.0f / 3.0f);
    p = fmaR(x, p, -0.5f);
    p = fmaR(x, p, 1.0f);
    return x * p;
}
// FP64: below 1/64 the Taylor polynomial of degree 10 (truncation below
// 8e-20 relative, evaluation within an ulp) replaces the library log1p
__device__ __forceinline__ double log1p_small(double x) {
    double p = fmaR(x, -1.0 / 10.0, 1.0 / 9.0);
    p = fmaR(x, p, -1.0 / 8.0);
    p = fmaR(x, p, 1.0 / 7.0);
    p = fmaR(x, p, -1.0 / 6.0);
    p = fmaR(x, p, 1.0 / 5.0);
    p = fmaR(x, p, -1.0 / 4.0);
    p = fmaR(x, p, 1.0 / 3.0);
    p = fmaR(x, p, -1.0 / 2.0);
    p = fmaR(x, p, 1.0);
    return x * p;
}
template <typename R> constexpr R log1p_small_limit() { return sizeof(R) == 8 ? R(1.0 / 64.0) : R(1.0 / 32.0); }

template <typename R>
__device__ __forceinline__ R exact_gamma(R gam, const R (&ds)[9], const R (&dh)[9], const R (&w)[9], R ir,
                                         const Coef<R>& K) {
    constexpr int kMaxIt = sizeof(R) == 8 ? 100 : 20;
    const R tol = sizeof(R) == 8 ? R(1e-15) : R(5e-7);
    const R tbm1 = R(2) * K.beta - R(1);
    R hw[9], sw[9], cd[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R wr = w[i] * ir;
        hw[i] = dh[i] * wr;
        sw[i] = tbm1 * ds[i] * wr;
        cd[i] = -K.beta * dh[i] * hw[i];
    }
    R prev = R(1e30);   // size of the previous Newton step
    for (int it = 0; it < kMaxIt; ++it) {
        const R om = R(1) - K.beta * gam;
        R x[9];
        bool ok = true;
        R amax = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            x[i] = fmaR(om, hw[i], -sw[i]);
            ok = ok && (x[i] > R(-1));
            amax = fmax(amax, fabs(x[i]));
        }
        if (!ok) break;
        R F = R(0), D = R(0);
        const bool general = !(amax < log1p_small_limit<R>());
        if (!general) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                F = fmaR(dh[i], log1p_small(x[i]), F);
                D = fmaR(cd[i], rcpR(R(1) + x[i]), D);
            }
        }
        if (general) {
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                F = fmaR(dh[i], log1pR(x[i]), F);
                D = fmaR(cd[i], rcpR(R(1) + x[i]), D);
            }
        }
        if (!(D < R(0))) break;
        const R step = divR(F, D);
        gam -= step;
        const R as = fabs(step);
        if (as <= tol * fabs(gam) || as > R(0.5) * prev) break;
        prev = as;
    }
    return gam;
}

// Forward quantities of one KBC collision at a node, shared by the step
// (collide) and its adjoint (collide_vjp) so that both take the same
// decisions on the same values.
template <typename R> struct KbcNode {
    R dr, rho, ir, jx, jy;              // rho - rho0, rho, 1 / rho, rho u
    R ux, uy, uxx, uyy, u2;
    R dT, dN, dP;                       // non-equilibrium T, N, Pi
    R tT;                               // T of the shear part: dT (A, C) or 0 (B, D)
    R ds[9], dh[9];                     // shear and higher-order parts of f - feq
    R w[9];                             // rho / feq_i (entropic weights)
    R ratio, b;                         // <ds|dh> / <dh|dh> and <dh|dh>
    R gam;                              // stabiliser used (estimate, 2 when guarded, or fixed)
    bool active;                        // gamma follows eq. (result21) (not guarded, not fixed)
};

// Written for instruction count: the kernels that call it issue one vector
// instruction per operation here and are bound by that issue rate, so every
// product-plus-sum is an explicit FMA (contraction is off) and scale factors
// are folded into the moments before they are spread back to populations.
template <typename R, int VAR, int GM>
__device__ __forceinline__ void kbc_forward(const R (&g)[9], const Coef<R>& K, KbcNode<R>& n) {
    // conserved moments, eq. (moments) restricted to the deviations
    const R s13 = g[1] + g[3], s24 = g[2] + g[4], s57 = g[5] + g[7], s68 = g[6] + g[8];
    const R d13 = g[1] - g[3], d24 = g[2] - g[4], d57 = g[5] - g[7], d68 = g[6] - g[8];
    const R sd = s57 + s68, sa = s13 + s24;
    const R dr = (g[0] + sd) + sa;                 // rho - rho0
    const R mq = d57 - d68, pq = d57 + d68;
    const R jx = d13 + mq;                         // rho u_x
    const R jy = d24 + pq;                         // rho u_y
    const R rho = K.rho0 + dr;
    const R ir = rcpR(rho);
    const R ux = jx * ir, uy = jy * ir;
    const R uxx = ux * ux, uyy = uy * uy, u2 = uxx + uyy;
    const R upv = ux + uy, umv = ux - uy;
    n.dr = dr; n.rho = rho; n.ir = ir; n.jx = jx; n.jy = jy;
    n.ux = ux; n.uy = uy; n.uxx = uxx; n.uyy = uyy; n.u2 = u2;

    constexpr bool kCentral = (VAR == VA || VAR == VB);   // s in the co-moving frame, eq. (cm)
    constexpr bool kTrace = (VAR == VA || VAR == VC);     // T belongs to s
    // non-equilibrium moments of df = f - feq (feq of second order, c_s^2 = 1/3)
    const R juy = jy * uy;
    const R jsum = fmaR(jx, ux, juy);          // rho |u|^2
    const R jdif = fmaR(jx, ux, -juy);         // rho (u_x^2 - u_y^2)
    const R dT = fmaR(R(2), sd, sa) - fmaR(R(2.0 / 3.0), dr, jsum);
    const R dN = (s13 - s24) - jdif;
    const R dP = fmaR(-jx, uy, s57 - s68);
    const R dQx = fmaR(R(-1.0 / 3.0), jx, mq);
    const R dQy = fmaR(R(-1.0 / 3.0), jy, pq);
    const R dA = fmaR(R(-1.0 / 3.0), jsum, fmaR(R(-1.0 / 9.0), dr, sd));
    const R uxy = ux * uy;
    n.dT = dT; n.dN = dN; n.dP = dP;
    n.tT = kTrace ? dT : R(0);

    // Shear part s, Table kbc_moment_grouping: (T_s, N, Pi, Q_xyy,s, Q_yxx,s,
    // A_s), all scaled by 1/4 (tq, nq, pq4, xq, yq, aq).  Central variants
    // take the linear part of eq. (cm) at the node's velocity.
    const R nq = R(0.25) * dN, pq4 = R(0.25) * dP;
    R xq = R(0), yq = R(0), aq = R(0);
    if constexpr (kCentral) {
        const R p2 = R(0.5) * dP, n8 = R(0.125) * dN;
        if constexpr (kTrace) {
            const R t8 = R(0.125) * dT;
            xq = fmaR(uy, p2, ux * (t8 - n8));
            yq = fmaR(ux, p2, uy * (t8 + n8));
            aq = fmaR(uxy, dP, fmaR(u2, t8, -((uxx - uyy) * n8)));
        } else {
            xq = fmaR(uy, p2, -(ux * n8));
            yq = fmaR(ux, p2, uy * n8);
            aq = fmaR(uxy, dP, -((uxx - uyy) * n8));
        }
    }
    // populations of s, eq. (momentsD2Q9) without mass and momentum
    R (&ds)[9] = n.ds;
    {
        R tpn, tmn;                              // (T_s +- N) / 4
        if constexpr (kTrace) {
            const R tq = R(0.25) * dT;
            tpn = tq + nq;
            tmn = tq - nq;
        } else {
            tpn = nq;
            tmn = -nq;
        }
        if constexpr (kCentral) {
            ds[0] = kTrace ? fmaR(R(4), aq, -dT) : R(4) * aq;
            ds[1] = fmaR(R(-2), xq + aq, tpn);
            ds[3] = fmaR(R(2), xq - aq, tpn);
            ds[2] = fmaR(R(-2), yq + aq, tmn);
            ds[4] = fmaR(R(2), yq - aq, tmn);
            const R ap = aq + pq4, am = aq - pq4, xp = xq + yq, xm = xq - yq;
            ds[5] = ap + xp;
            ds[7] = ap - xp;
            ds[6] = am - xm;
            ds[8] = am + xm;
        } else {
            ds[0] = kTrace ? -dT : R(0);
            ds[1] = tpn;
            ds[3] = tpn;
            ds[2] = tmn;
            ds[4] = tmn;
            ds[5] = pq4;
            ds[7] = pq4;
            ds[6] = -pq4;
            ds[8] = -pq4;
        }
    }
    // higher-order part h = df - s: moments (T - T_s, 0, 0, dQ - Q_s, dA - A_s) / 4
    R (&dh)[9] = n.dh;
    {
        const R xh = kCentral ? fmaR(R(0.25), dQx, -xq) : R(0.25) * dQx;
        const R yh = kCentral ? fmaR(R(0.25), dQy, -yq) : R(0.25) * dQy;
        const R ah = kCentral ? fmaR(R(0.25), dA, -aq) : R(0.25) * dA;
        const R hp = xh + yh, hm = xh - yh;
        dh[5] = ah + hp;
        dh[7] = ah - hp;
        dh[6] = ah - hm;
        dh[8] = ah + hm;
        if constexpr (kTrace) {
            dh[0] = R(4) * ah;
            dh[1] = R(-2) * (xh + ah);
            dh[3] = R(2) * (xh - ah);
            dh[2] = R(-2) * (yh + ah);
            dh[4] = R(2) * (yh - ah);
        } else {
            const R th = R(0.25) * dT;
            dh[0] = fmaR(R(4), ah, -dT);
            dh[1] = fmaR(R(-2), xh + ah, th);
            dh[3] = fmaR(R(2), xh - ah, th);
            dh[2] = fmaR(R(-2), yh + ah, th);
            dh[4] = fmaR(R(2), yh - ah, th);
        }
    }

    if constexpr (GM == GFIX) {
        n.gam = K.gamma_fixed;
        n.active = false;
        n.ratio = R(0);
        n.b = R(1);
    } else {
        // entropic scalar products, weights 1 / (W_i (1 + e_i)) = rho / feq_i;
        // d_i = W_i (1 + e_i) = W_i (1 - 1.5 |u|^2 + 4.5 (v.u)^2) + 3 W_i (v.u)
        const R a1 = fmaR(R(-1.0 / 6.0), u2, R(1.0 / 9.0));
        const R a5 = fmaR(R(1.0 / 12.0), u2, R(1.0 / 36.0));
        const R dx = fmaR(R(0.5), uxx, a1), dy = fmaR(R(0.5), uyy, a1);
        const R dp = fmaR(R(0.25), uxy, a5), dm = fmaR(R(-0.25), uxy, a5);
        R d[9];
        d[0] = fmaR(R(-2.0 / 3.0), u2, R(4.0 / 9.0));
        d[1] = fmaR(R(1.0 / 3.0), ux, dx);
        d[3] = fmaR(R(-1.0 / 3.0), ux, dx);
        d[2] = fmaR(R(1.0 / 3.0), uy, dy);
        d[4] = fmaR(R(-1.0 / 3.0), uy, dy);
        d[5] = fmaR(R(1.0 / 12.0), upv, dp);
        d[7] = fmaR(R(-1.0 / 12.0), upv, dp);
        d[8] = fmaR(R(1.0 / 12.0), umv, dm);
        d[6] = fmaR(R(-1.0 / 12.0), umv, dm);
        R a = R(0), b = R(0), c = R(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            n.w[i] = rcpR(d[i]);
            const R wh = dh[i] * n.w[i];
            a = fmaR(ds[i], wh, a);
            b = fmaR(dh[i], wh, b);
            c = fmaR(ds[i] * n.w[i], ds[i], c);
        }
        n.ratio = divR(a, b);
        n.b = b;
        const R gs = fmaR(-K.two_m_inv_beta, n.ratio, K.inv_beta);
        n.active = !(b <= K.guard * c);
        n.gam = n.active ? gs : R(2);
    }
}

// One collision on the deviations g (in place).  Returns the gamma used.
template <typename R, int COLL, int VAR, int GM>
__device__ __forceinline__ R collide(R (&g)[9], const Coef<R>& K) {
    if constexpr (COLL == LBGK) {
        const R s13 = g[1] + g[3], s24 = g[2] + g[4], s57 = g[5] + g[7], s68 = g[6] + g[8];
        const R d13 = g[1] - g[3], d24 = g[2] - g[4], d57 = g[5] - g[7], d68 = g[6] - g[8];
        const R dr = (g[0] + (s57 + s68)) + (s13 + s24);
        const R jx = d13 + (d57 - d68), jy = d24 + (d57 + d68);
        const R rho = K.rho0 + dr;
        const R ir = rcpR(rho);
        const R ux = jx * ir, uy = jy * ir;
        const R uxx = ux * ux, uyy = uy * uy, u2 = uxx + uyy;
        const R upv = ux + uy, umv = ux - uy;
        // f' = f - 2 beta (f - feq), eq. (LBGKmirr) in eq. (Egeneral):
        // g' = (1 - 2 beta) g + 2 beta W_i [(rho - rho0) + rho e_i],
        // e_i = 3 (v.u) + 4.5 (v.u)^2 - 1.5 |u|^2
        const R c0 = R(-1.5) * u2;
        const R bx = fmaR(R(4.5), uxx, c0), by = fmaR(R(4.5), uyy, c0);
        const R uxy9 = R(9) * (ux * uy);
        const R b5 = fmaR(R(3), u2, uxy9), b6 = fmaR(R(3), u2, -uxy9);   // 4.5 (u_x +- u_y)^2 - 1.5 |u|^2
        R e[9];
        e[0] = c0;
        e[1] = fmaR(R(3), ux, bx);
        e[3] = fmaR(R(-3), ux, bx);
        e[2] = fmaR(R(3), uy, by);
        e[4] = fmaR(R(-3), uy, by);
        e[5] = fmaR(R(3), upv, b5);
        e[7] = fmaR(R(-3), upv, b5);
        e[8] = fmaR(R(3), umv, b6);
        e[6] = fmaR(R(-3), umv, b6);
        const R tb = R(2) * K.beta, omt = R(1) - tb;
        const R tw[3] = {tb * R(weight(0)), tb * R(weight(1)), tb * R(weight(5))};
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const R twi = tw[i == 0 ? 0 : (i < 5 ? 1 : 2)];
            g[i] = fmaR(omt, g[i], twi * fmaR(rho, e[i], dr));
        }
        return R(2);
    } else {
        KbcNode<R> n;
        kbc_forward<R, VAR, (GM == GEXACT ? GEST : GM)>(g, K, n);
        R gam = n.gam;
        if constexpr (GM == GEXACT) {
            if (n.active) gam = exact_gamma<R>(gam, n.ds, n.dh, n.w, n.ir, K);
        }
        // f' = f - beta (2 ds + gamma dh), eqs. (Egeneral), (ksh-mirror)
        const R tb = R(2) * K.beta, bg = K.beta * gam;
#pragma unroll
        for (int i = 0; i < 9; ++i) g[i] = fmaR(-bg, n.dh[i], fmaR(-tb, n.ds[i], g[i]));
        return gam;
    }
}

}  // namespace kbc
