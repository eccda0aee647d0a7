/*
 * Lattice tables shared by the two translation units of the oracle.
 * TEST INFRASTRUCTURE: see kbc_oracle.h.
 */
#ifndef KBC_ORACLE_INTERNAL_H
#define KBC_ORACLE_INTERNAL_H

#include "kbc_oracle.h"

/* D2Q9 velocities v_(i,j) = (i,j), i,j in {0,+1,-1}, in the documented order. */
static const int ORC_CX[ORC_Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int ORC_CY[ORC_Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Squared sound speed of the three-velocity set {0,+1,-1}: the second moment
 * of its weights, 2 * (1/6) = 1/3. */
#define ORC_CS2 (1.0 / 3.0)

/* The D2Q9 set is the tensor product of the one-dimensional set {0,+1,-1}
 * (section "Moment Representation"), so its weights are products of the
 * one-dimensional weights w(0) = 1 - cs2, w(+-1) = cs2 / 2. */
static inline double orc_w1d(int c) { return c == 0 ? 1.0 - ORC_CS2 : 0.5 * ORC_CS2; }
static inline double orc_weight(int i) { return orc_w1d(ORC_CX[i]) * orc_w1d(ORC_CY[i]); }

static inline double orc_ipow(int c, int p)
{
    double r = 1.0;
    for (int k = 0; k < p; ++k) r *= (double)c;
    return r;
}

static inline int orc_wrap(int v, int n) { return ((v % n) + n) % n; }

#endif
