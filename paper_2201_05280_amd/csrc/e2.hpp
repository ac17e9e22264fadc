// e2.hpp -- the E2 equilibrium: the discrete quasi-equilibrium that
// minimises the H function on the 41 velocities under fixed density,
// momentum and pressure tensor (Sec. 2, quasi-equilibria; Sec. 3, the ES
// target as a quasi-equilibrium).  On the lattice it has the exponential form
//   F_i = w_i exp(l . phi_i),  phi_i = (1, c, cx^2, cy^2, cz^2, cxcy, cxcz, cycz),
// with the ten multipliers l fixed by sum_i F_i phi_i = (rho, rho u, rho (uu + lam)).
// The multipliers come from Newton's method on those ten equations, started
// from the continuous Gaussian N(u, lam) / N(0, theta0 I) (or from a nearby
// solution) and damped so that no exponent changes by more than 2 in one
// iteration; a U^T D U factorization of the (symmetric positive definite) Jacobian
// sum_i F_i phi_i phi_i^T gives the step.  It stops once the moments are met
// to 1e-14 and the last step moved no exponent by more than 1e-8, so that the
// result is the constrained minimiser to round-off, not a function of the
// starting point; a full step of at most 1e-8 taken where the moments were
// already met to 1e-8 ends the solve at once (the check after it would pass
// and return the same multipliers).  The same code runs on the host (face
// states) and in the kernels.
//
// The opposite velocities +-c of a pair share the even part of the exponent
// and differ in the sign of the odd part (the three linear multipliers), so
// every sum runs over the rest velocity and 20 pairs.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "lattice.hpp"

namespace pgk {

constexpr int E2_NL = 10;
constexpr int E2_MAXIT = 100;

// index of (k, l), k <= l, in the packed upper triangle of a 10 x 10 matrix
__host__ __device__ constexpr int e2_ij(int k, int l)
{
    return k * E2_NL - k * (k - 1) / 2 + (l - k);
}

// basis values of pair representative P: phi[k] for k = 0..9
template <int P>
struct E2Phi {
    static constexpr double cx = 0.5 * Lattice::REP2[P][0], cy = 0.5 * Lattice::REP2[P][1],
                            cz = 0.5 * Lattice::REP2[P][2];
    __host__ __device__ static constexpr double at(int k)
    {
        return k == 0 ? 1.0 : k == 1 ? cx : k == 2 ? cy : k == 3 ? cz : k == 4 ? cx * cx : k == 5 ? cy * cy
             : k == 6 ? cz * cz : k == 7 ? cx * cy : k == 8 ? cx * cz : cy * cz;
    }
    // phi[k] is odd in c for k = 1..3
    __host__ __device__ static constexpr bool odd(int k) { return k >= 1 && k <= 3; }
};

// even and odd parts of l . phi for pair P
template <int P>
__host__ __device__ __forceinline__ void e2_parts(const double *l, double &ev, double &od)
{
    using F = E2Phi<P>;
    ev = l[0];
    od = 0.0;
    if (F::cx != 0.0) { od += F::cx * l[1]; ev += F::cx * F::cx * l[4]; }
    if (F::cy != 0.0) { od += F::cy * l[2]; ev += F::cy * F::cy * l[5]; }
    if (F::cz != 0.0) { od += F::cz * l[3]; ev += F::cz * F::cz * l[6]; }
    if (F::cx * F::cy != 0.0) ev += F::cx * F::cy * l[7];
    if (F::cx * F::cz != 0.0) ev += F::cx * F::cz * l[8];
    if (F::cy * F::cz != 0.0) ev += F::cy * F::cz * l[9];
}

// The exponentials of l . phi as products of integer powers of ten base
// exponentials.  In doubled coordinates k = 2c every velocity component is 0,
// +-1, +-2 or +-4, so
//   exp(even part) = exp(l0) prod_a exp(l_aa / 4)^(k_a^2) prod_{a<b} exp(l_ab / 4)^(k_a k_b),
//   exp(odd part)  = prod_a exp(l_a / 2)^(k_a),
// with k_a^2 in {1, 4, 16} and k_a k_b in {+-1, +-4}: ten exponentials, six
// reciprocals and squarings instead of 41 exponentials.  The populations
// differ from single exponentials of l . phi by a few ulps; the converged
// multipliers differ from those of single exponentials by no more than a
// restart of the same Newton solve from a nearby point moves them.
// 1 / d for a positive normal d (the base exponentials of the odd powers): on
// the device the hardware reciprocal refined by two Newton-Raphson steps
// r <- r + r (1 - d r), within an ulp of the rounded quotient at a third of
// the instructions of the IEEE division; on the host the division itself.
// The converged multipliers do not depend on it beyond round-off: the moments
// decide when the solve stops.  (In the factorization the refinement's extra
// live values cost the batched kernel more register spills than it saves.)
__host__ __device__ __forceinline__ double e2_rcp(double d)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
#else
    return 1.0 / d;
#endif
}

struct E2Pow {
    double e0;          // exp(l0)
    double d[3][3];     // exp(l_aa / 4) to the powers 1, 4, 16 (a = x, y, z)
    double o[3][4];     // exp(l_ab / 4) to the powers 1, 4, -1, -4 (ab = xy, xz, yz)
    double x[3][6];     // exp(l_a / 2) to the powers 1, 2, 4, -1, -2, -4
};

__host__ __device__ __forceinline__ void e2_pow_bases(const double *l, E2Pow &p)
{
    p.e0 = exp(l[0]);
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double d = exp(0.25 * l[4 + a]), d4 = (d * d) * (d * d), d8 = d4 * d4;
        p.d[a][0] = d;
        p.d[a][1] = d4;
        p.d[a][2] = d8 * d8;
        const double x = exp(0.5 * l[1 + a]), ix = e2_rcp(x), x2 = x * x, ix2 = ix * ix;
        p.x[a][0] = x;
        p.x[a][1] = x2;
        p.x[a][2] = x2 * x2;
        p.x[a][3] = ix;
        p.x[a][4] = ix2;
        p.x[a][5] = ix2 * ix2;
        const double o = exp(0.25 * l[7 + a]), io = e2_rcp(o), o2 = o * o, io2 = io * io;
        p.o[a][0] = o;
        p.o[a][1] = o2 * o2;
        p.o[a][2] = io;
        p.o[a][3] = io2 * io2;
    }
}

// exp(l_aa k^2 / 4), exp(l_ab kk / 4), exp(l_a k / 2) for compile-time k, kk
template <int K>
__host__ __device__ __forceinline__ double e2_dpow(const E2Pow &p, int a)
{
    constexpr int s = K * K;
    static_assert(s == 0 || s == 1 || s == 4 || s == 16, "doubled component");
    return s == 0 ? 1.0 : s == 1 ? p.d[a][0] : s == 4 ? p.d[a][1] : p.d[a][2];
}
template <int KK>
__host__ __device__ __forceinline__ double e2_opow(const E2Pow &p, int b)
{
    static_assert(KK == 0 || KK == 1 || KK == 4 || KK == -1 || KK == -4, "doubled product");
    return KK == 0 ? 1.0 : KK == 1 ? p.o[b][0] : KK == 4 ? p.o[b][1] : KK == -1 ? p.o[b][2] : p.o[b][3];
}
template <int K>
__host__ __device__ __forceinline__ double e2_xpow(const E2Pow &p, int a)
{
    static_assert(K == 0 || K == 1 || K == 2 || K == 4 || K == -1 || K == -2 || K == -4, "doubled component");
    return K == 0 ? 1.0 : K == 1 ? p.x[a][0] : K == 2 ? p.x[a][1] : K == 4 ? p.x[a][2]
         : K == -1 ? p.x[a][3] : K == -2 ? p.x[a][4] : p.x[a][5];
}

// exp(even part) and exp(+-odd part) of l . phi for pair P
template <int P>
__host__ __device__ __forceinline__ void e2_pair_exp(const E2Pow &p, double &ev, double &xp, double &xm)
{
    constexpr int kx = Lattice::REP2[P][0], ky = Lattice::REP2[P][1], kz = Lattice::REP2[P][2];
    ev = ((p.e0 * e2_dpow<kx>(p, 0)) * (e2_dpow<ky>(p, 1) * e2_dpow<kz>(p, 2))) *
         ((e2_opow<kx * ky>(p, 0) * e2_opow<kx * kz>(p, 1)) * e2_opow<ky * kz>(p, 2));
    xp = (e2_xpow<kx>(p, 0) * e2_xpow<ky>(p, 1)) * e2_xpow<kz>(p, 2);
    xm = (e2_xpow<-kx>(p, 0) * e2_xpow<-ky>(p, 1)) * e2_xpow<-kz>(p, 2);
}

// moments and Jacobian contributions of pair P (F+ and F- of weight w)
template <int P = 0>
__host__ __device__ __forceinline__ void e2_accumulate(const E2Pow &pw, const double *w6, double *mom, double *J)
{
    if constexpr (P < NPAIR) {
        using F = E2Phi<P>;
        double ev, xp, xm;
        e2_pair_exp<P>(pw, ev, xp, xm);
        double w = w6[Lattice::SHELL[P]] * ev;
        double fp = w * xp, fm = w * xm;
        double s = fp + fm, d = fp - fm;
#pragma unroll
        for (int k = 0; k < E2_NL; k++) {
            double pk = F::at(k);
            if (pk == 0.0) continue;
            mom[k] += pk * (F::odd(k) ? d : s);
#pragma unroll
            for (int m = k; m < E2_NL; m++) {
                double pm = F::at(m);
                if (pm == 0.0) continue;
                // phi_k phi_m is odd in c exactly when one of the two is
                J[e2_ij(k, m)] += pk * pm * ((F::odd(k) != F::odd(m)) ? d : s);
            }
        }
        e2_accumulate<P + 1>(pw, w6, mom, J);
    }
}

// largest |delta . phi_i| over the velocities (the damping measure)
template <int P = 0>
__host__ __device__ __forceinline__ double e2_maxchange(const double *dl, double acc)
{
    if constexpr (P < NPAIR) {
        double ev, od;
        e2_parts<P>(dl, ev, od);
        double m = fabs(ev) + fabs(od);   // max(|ev + od|, |ev - od|)
        return e2_maxchange<P + 1>(dl, m > acc ? m : acc);
    } else {
        return acc;
    }
}

// In-place solve of the packed SPD system J x = b by the factorization
// J = U^T D U (U unit upper triangular, D diagonal; no square roots, one
// reciprocal per column); false if J is not positive definite (a pivot
// d_j <= 0).  U overwrites the upper triangle of J.
__host__ __device__ __forceinline__ bool e2_cholesky_solve(double *J, double *b)
{
    double dinv[E2_NL], dd[E2_NL];
#pragma unroll
    for (int j = 0; j < E2_NL; j++) {
        double wk[E2_NL];   // U[k][j] d_k, k < j
        double d = J[e2_ij(j, j)];
#pragma unroll
        for (int k = 0; k < j; k++) {
            wk[k] = J[e2_ij(k, j)] * dd[k];
            d -= wk[k] * J[e2_ij(k, j)];
        }
        if (!(d > 0.0)) return false;
        dd[j] = d;
        dinv[j] = 1.0 / d;
#pragma unroll
        for (int i = j + 1; i < E2_NL; i++) {
            double t = J[e2_ij(j, i)];
#pragma unroll
            for (int k = 0; k < j; k++) t -= wk[k] * J[e2_ij(k, i)];
            J[e2_ij(j, i)] = t * dinv[j];   // U[j][i]
        }
    }
    // U^T y = b, then z = y / d, then U x = z
#pragma unroll
    for (int i = 0; i < E2_NL; i++) {
        double t = b[i];
#pragma unroll
        for (int k = 0; k < i; k++) t -= J[e2_ij(k, i)] * b[k];
        b[i] = t;
    }
#pragma unroll
    for (int i = 0; i < E2_NL; i++) b[i] *= dinv[i];
#pragma unroll
    for (int i = E2_NL - 1; i >= 0; i--) {
        double t = b[i];
#pragma unroll
        for (int k = i + 1; k < E2_NL; k++) t -= J[e2_ij(i, k)] * b[k];
        b[i] = t;
    }
    return true;
}

// Moment targets (rho, rho u, rho (uu + lam)) of density rho, velocity u and
// covariance lam (xx yy zz xy xz yz).
__host__ __device__ __forceinline__ void e2_targets(double rho, const double *u, const double *lam, double *tg)
{
    tg[0] = rho;
    tg[1] = rho * u[0];
    tg[2] = rho * u[1];
    tg[3] = rho * u[2];
    tg[4] = rho * (u[0] * u[0] + lam[0]);
    tg[5] = rho * (u[1] * u[1] + lam[1]);
    tg[6] = rho * (u[2] * u[2] + lam[2]);
    tg[7] = rho * (u[0] * u[1] + lam[3]);
    tg[8] = rho * (u[0] * u[2] + lam[4]);
    tg[9] = rho * (u[1] * u[2] + lam[5]);
}

// Newton start: the continuous Gaussian N(u, lam) over the reference
// Gaussian N(0, theta0 I); false if lam is not positive definite
__host__ __device__ __forceinline__ bool e2_gaussian_start(double th0, double rho, const double *u, const double *lam,
                                                           double *l)
{
    double a = lam[0], b = lam[1], c = lam[2], d = lam[3], e = lam[4], f = lam[5];
    double c00 = b * c - f * f, c01 = e * f - d * c, c02 = d * f - b * e;
    double det = a * c00 + d * c01 + e * c02;
    if (!(det > 0.0) || !(rho > 0.0)) return false;
    double id = 1.0 / det;
    double i00 = c00 * id, i01 = c01 * id, i02 = c02 * id;
    double i11 = (a * c - e * e) * id, i12 = (d * e - a * f) * id, i22 = (a * b - d * d) * id;
    double v0 = i00 * u[0] + i01 * u[1] + i02 * u[2];
    double v1 = i01 * u[0] + i11 * u[1] + i12 * u[2];
    double v2 = i02 * u[0] + i12 * u[1] + i22 * u[2];
    l[0] = log(rho) - 0.5 * log(det / (th0 * th0 * th0)) - 0.5 * (u[0] * v0 + u[1] * v1 + u[2] * v2);
    l[1] = v0;
    l[2] = v1;
    l[3] = v2;
    l[4] = -0.5 * (i00 - 1.0 / th0);
    l[5] = -0.5 * (i11 - 1.0 / th0);
    l[6] = -0.5 * (i22 - 1.0 / th0);
    l[7] = -i01;
    l[8] = -i02;
    l[9] = -i12;
    return true;
}

// Damped Newton from the multipliers in l toward the targets tg; returns the
// iteration count (> 0) or -1 (Jacobian not positive definite, no
// convergence in E2_MAXIT iterations, or a non-finite step).
__host__ __device__ __forceinline__ int e2_newton(const double *w6, const double *tg, double *l)
{
    double scale = 0.0;
#pragma unroll
    for (int k = 0; k < E2_NL; k++) scale += fabs(tg[k]);
    double last = 1e300;   // largest exponent change of the last step
    for (int it = 1; it <= E2_MAXIT; it++) {
        double mom[E2_NL], J[E2_NL * (E2_NL + 1) / 2];
#pragma unroll
        for (int k = 0; k < E2_NL; k++) mom[k] = 0.0;
#pragma unroll
        for (int k = 0; k < E2_NL * (E2_NL + 1) / 2; k++) J[k] = 0.0;
        E2Pow pw;
        e2_pow_bases(l, pw);
        double f0 = w6[0] * pw.e0;   // rest velocity: phi = (1, 0, ...)
        mom[0] = f0;
        J[0] = f0;
        e2_accumulate(pw, w6, mom, J);
        double rhs[E2_NL], res = 0.0;
#pragma unroll
        for (int k = 0; k < E2_NL; k++) {
            rhs[k] = tg[k] - mom[k];
            res += fabs(rhs[k]);
        }
        // converged: moments within 1e-14 and the last step so small that the
        // next would change nothing (the multipliers then sit at the
        // round-off floor whatever the starting point)
        if (res <= 1e-14 * scale && last <= 1e-8) return it;
        if (!e2_cholesky_solve(J, rhs)) return -1;
        double maxd = e2_maxchange(rhs, fabs(rhs[0]));
        last = maxd;
        double damp = maxd > 2.0 ? 2.0 / maxd : 1.0;
#pragma unroll
        for (int k = 0; k < E2_NL; k++) l[k] += damp * rhs[k];
        if (!(fabs(l[0]) < 1e300)) return -1;   // NaN or overflow
        // a full step this small from a point this close leaves an error of
        // the order of its square (Newton's quadratic convergence), below
        // round-off: the confirming pass would find the moments met and return
        // these same multipliers, so return them now
        if (maxd <= 1e-8 && res <= 1e-8 * scale) return it;
    }
    return -1;
}

// Multipliers of the E2 equilibrium with density rho, velocity u and
// covariance lam (xx yy zz xy xz yz), Newton started from the Gaussian.
// Returns the Newton iteration count (> 0), or -1 when the moments cannot be
// reached (covariance not positive definite, Jacobian singular, no
// convergence); the moments then lie outside what a positive distribution on
// the 41 velocities can carry.
__host__ __device__ __forceinline__ int e2_solve(double th0, const double *w6, double rho, const double *u,
                                                 const double *lam, double *l)
{
    double tg[E2_NL];
    e2_targets(rho, u, lam, tg);
    if (!e2_gaussian_start(th0, rho, u, lam, l)) return -1;
    return e2_newton(w6, tg, l);
}

// The same, started from the multipliers already in l when they are finite
// (a neighbouring state, e.g. the site's previous step), falling back to the
// Gaussian start if that Newton run fails.
__host__ __device__ __forceinline__ int e2_solve_from(double th0, const double *w6, double rho, const double *u,
                                                      const double *lam, double *l)
{
    double tg[E2_NL];
    e2_targets(rho, u, lam, tg);
    bool warm = true;
#pragma unroll
    for (int k = 0; k < E2_NL; k++) warm = warm && fabs(l[k]) < 1e300;
    if (warm) {
        int it = e2_newton(w6, tg, l);
        if (it > 0) return it;
    }
    if (!e2_gaussian_start(th0, rho, u, lam, l)) return -1;
    return e2_newton(w6, tg, l);
}

// F_q of the multipliers l (any q, host side)
__host__ inline double e2_population(const double *l, const double *w6, int q)
{
    double cx = 0.5 * c2(q, 0), cy = 0.5 * c2(q, 1), cz = 0.5 * c2(q, 2);
    double ex = l[0] + cx * l[1] + cy * l[2] + cz * l[3] + cx * cx * l[4] + cy * cy * l[5] + cz * cz * l[6] +
                cx * cy * l[7] + cx * cz * l[8] + cy * cz * l[9];
    return w6[shell_of(q)] * exp(ex);
}

}  // namespace pgk
