// Exact line-search step (internal): the positive minimiser of the quartic phi whose derivative is
// phi'(a) = c0 + c1 a + c2 a^2 + c3 a^3 (ADMM solver, X-update: f(theta + a p) is a quartic in a
// because C is quadratic in the factors). Host and device share this code; a CPU test program
// compares it with the oracle's root selection.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace tlr {

using std::fabs;
using std::fmax;
using std::fmin;
using std::isfinite;
using std::sqrt;

__host__ __device__ inline double phi_inc(const double *c, double a) {
    return a * (c[0] + a * (c[1] / 2 + a * (c[2] / 3 + a * c[3] / 4)));
}

__host__ __device__ inline double dphi(const double *c, double a) { return ((c[3] * a + c[2]) * a + c[1]) * a + c[0]; }
__host__ __device__ inline double ddphi(const double *c, double a) { return (3.0 * c[3] * a + 2.0 * c[2]) * a + c[1]; }

// The root of phi' between x1 and x2, where phi' is monotone and phi'(x1), phi'(x2) have opposite
// signs: safeguarded Newton-Raphson (a Newton step is taken while it stays inside the bracket and
// at least halves the step before it; otherwise the bracket is bisected), converging to full
// precision without the cancellation of closed-form cubic roots.
__host__ __device__ inline double bracketed_root(const double *c, double x1, double x2) {
    const double f1 = dphi(c, x1), f2 = dphi(c, x2);
    if (f1 == 0.0) return x1;
    if (f2 == 0.0) return x2;
    double neg = f1 < 0.0 ? x1 : x2, pos = f1 < 0.0 ? x2 : x1;   // phi'(neg) < 0 < phi'(pos)
    double x = 0.5 * (x1 + x2), dx_old = fabs(x2 - x1), dx = dx_old;
    double f = dphi(c, x), fd = ddphi(c, x);
    for (int it = 0; it < 400; ++it) {
        const bool leaves = ((x - pos) * fd - f) * ((x - neg) * fd - f) > 0.0;
        const bool slow = fabs(2.0 * f) > fabs(dx_old * fd);
        dx_old = dx;
        if (leaves || slow) {
            dx = 0.5 * (pos - neg);
            x = neg + dx;
            if (x == neg) return x;
        } else {
            dx = f / fd;
            const double prev = x;
            x -= dx;
            if (x == prev) return x;
        }
        if (fabs(dx) <= 2.220446049250313e-16 * fabs(x)) return x;
        f = dphi(c, x);
        fd = ddphi(c, x);
        if (f == 0.0) return x;
        if (f < 0.0) neg = x;
        else pos = x;
    }
    return x;
}

// Positive minimiser of phi: the positive real root of phi' with the lowest phi (ties: the smaller
// step; none: 0). (0, inf) is split at the positive roots of phi'' into pieces on which phi' is
// monotone; each piece holds at most one root, found by bracketed_root (the last piece's bracket
// by doubling until phi' changes sign). A stationary point of phi' at which phi' vanishes (a double
// root) is a root too.
__host__ __device__ inline double exact_step_dev(const double *c) {
    const double scale = fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);
    if (!(scale > 0.0) || !isfinite(scale)) return 0.0;
    // positive roots of phi''(a) = c1 + 2 c2 a + 3 c3 a^2, ascending (stable quadratic formula)
    double brk[2];
    int nb = 0;
    if (c[3] != 0.0) {
        const double disc = c[2] * c[2] - 3.0 * c[3] * c[1];
        if (disc > 0.0) {
            const double q = -(c[2] + (c[2] >= 0.0 ? sqrt(disc) : -sqrt(disc)));
            const double r1 = q / (3.0 * c[3]), r2 = q != 0.0 ? c[1] / q : r1;
            const double lo = fmin(r1, r2), hi = fmax(r1, r2);
            if (lo > 0.0 && isfinite(lo)) brk[nb++] = lo;
            if (hi > 0.0 && isfinite(hi) && hi != lo) brk[nb++] = hi;
        }
    } else if (c[2] != 0.0) {
        const double r = -c[1] / (2.0 * c[2]);
        if (r > 0.0 && isfinite(r)) brk[nb++] = r;
    }
    // sign of phi' as a -> inf: its leading nonzero coefficient
    const double lead = c[3] != 0.0 ? c[3] : c[2] != 0.0 ? c[2] : c[1] != 0.0 ? c[1] : c[0];
    double cand[3];
    int nc = 0;
    double lo = 0.0;
    for (int k = 0; k <= nb; ++k) {
        const double flo = dphi(c, lo);
        if (k > 0 && flo == 0.0) {   // a root at a stationary point of phi'
            cand[nc++] = lo;
        } else if (k < nb) {
            const double hi = brk[k], fhi = dphi(c, hi);
            if (fhi != 0.0 && (flo < 0.0) != (fhi < 0.0) && flo != 0.0) cand[nc++] = bracketed_root(c, lo, hi);
        } else if (flo != 0.0 && (flo < 0.0) != (lead < 0.0)) {   // last piece [lo, inf)
            double a = lo, b = lo > 0.0 ? 2.0 * lo : 1.0;
            int it = 0;
            while (isfinite(b) && (dphi(c, b) < 0.0) == (flo < 0.0) && dphi(c, b) != 0.0 && it < 2200) {
                a = b;
                b *= 2.0;
                ++it;
            }
            if (isfinite(b) && ((dphi(c, b) < 0.0) != (flo < 0.0) || dphi(c, b) == 0.0))
                cand[nc++] = bracketed_root(c, a, b);
        }
        if (k < nb) lo = brk[k];
    }
    double best = 0.0, bestv = 0.0;
    bool have = false;
    for (int k = 0; k < nc; ++k) {
        const double x = cand[k];
        if (!(x > 0.0) || !isfinite(x)) continue;
        const double v = phi_inc(c, x);
        if (!have || v < bestv || (v == bestv && x < best)) {
            best = x;
            bestv = v;
            have = true;
        }
    }
    return have ? best : 0.0;
}

}  // namespace tlr
