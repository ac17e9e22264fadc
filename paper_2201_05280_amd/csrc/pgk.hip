// pgk.hip -- HIP kernels (gfx950) and the C ABI for the reduced polyatomic
// ES-BGK lattice-Boltzmann step (Kolluru, Atif & Ansumali, arXiv:2201.05280).
//
// One time step is three launches (plus a boundary launch when an x face is
// not periodic):
//   k_lb   pull 41 populations, moments (double), g->f map with the first
//          half relaxation of theta_R (Sec. 5 g-f relations and step 1),
//          ES + BGK target (Sec. 4), F3 equilibrium, trapezoid collide
//          (Sec. 5), write the own site; hand rho, u, rho*theta, the
//          half-relaxed theta_R and its increment to the transport.
//   k_mc   MacCormack advection of theta_R (Sec. 5, step 2).
//   k_dif  FTCS diffusion and the second relaxation half (Sec. 5, steps 3-4).
//   k_bc   fill the x ghost populations (diffuse wall / Dirichlet).
// Populations are stored after the collision of the previous step, at their
// own site, structure-of-arrays [q][sub][z][y][x]; the next step pulls.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pgk.h"
#include "lattice.hpp"

namespace pgk {

constexpr int WG = 256;
constexpr int NSLOT = 4;  // ghost slots per x face: doubled x offsets 1..4 beyond the face

struct Consts {
    int nx, ny, nz, ns;
    int bc[2];
    double th0;
    double w[6];            // shell weights
    float whi[6], wlo[6];   // the same as float hi + lo parts (w = whi + wlo to ~1e-15)
    double tau, tau1, b, delta;
    double X, Y, ssig, beta, kfac;
    double thbc[2], rhobc[2];
    double Fbc[2][NQ];      // wall equilibrium at unit density / Dirichlet equilibrium
    double in_col[2];       // re-emitted mass per ghost column at unit wall density
    // division by nx, ny, nz: q = (umulhi(n, m) + n) >> sh for n < 2^31
    unsigned mx, my, mz;
    int shx, shy, shz;
    // per-step constants computed once on the host
    double inv1X, inv1XY, inv3d;  // 1/(1+X), 1/(1+X+Y), 1/(3+delta)
    double wt1, wt, bs;           // tau1/(tau+tau1), tau/(tau+tau1), b/s_sigma
    double it, i2t, ih2, i6t3, i2t3, it2;  // 1/t, 1/(2t), 1/(2t^2), 1/(6t^3), 1/(2t^3), 1/t^2 with t = theta0
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned fdiv(unsigned n, unsigned m, int sh)
{
    return (__umulhi(n, m) + n) >> sh;
}

__device__ __forceinline__ void decode(int s, const Consts &k, int &x, int &y, int &z, int &sub)
{
    unsigned t = fdiv((unsigned)s, k.mx, k.shx);
    x = s - (int)t * k.nx;
    unsigned t2 = fdiv(t, k.my, k.shy);
    y = (int)t - (int)t2 * k.ny;
    unsigned t3 = fdiv(t2, k.mz, k.shz);
    z = (int)t2 - (int)t3 * k.nz;
    sub = (int)t3;
}

// wrap x + d into [0, n) for |d| <= 2 and any n >= 1
__device__ __forceinline__ int wrap2(int v, int n)
{
    v += (v < 0) ? n : 0;
    v += (v < 0) ? n : 0;
    v -= (v >= n) ? n : 0;
    v -= (v >= n) ? n : 0;
    return v;
}

// Offsets of the pull sources of one site on a periodic grid.  Integer
// velocities stay on the own sublattice at coordinate offsets -c (|c| <= 2);
// half velocities come from the other sublattice, at offset -1 or 0 along an
// axis for corner sites and 0 or +1 for body-centre sites.
struct Off5 {
    int m2, m1, z0, p1, p2;
    template <int D> __device__ __forceinline__ int at() const
    {
        if constexpr (D == -2) return m2;
        else if constexpr (D == -1) return m1;
        else if constexpr (D == 0) return z0;
        else if constexpr (D == 1) return p1;
        else return p2;
    }
};

struct PullMap {
    int own, oth;                 // offsets of the own and the other sublattice
    Off5 X, Y, Z;                 // wrapped x, y*nx, z*nx*ny for offsets -2..2
    int hx[2], hy[2], hz[2];      // half velocities: [0] for c > 0, [1] for c < 0
};

__device__ __forceinline__ PullMap pull_map(int x, int y, int z, int sub, const Consts &k)
{
    PullMap p;
    int plane = k.nx * k.ny, subsz = plane * k.nz;
    p.own = sub * subsz;
    p.oth = (1 - sub) * subsz;
    p.X = {wrap2(x - 2, k.nx), wrap2(x - 1, k.nx), x, wrap2(x + 1, k.nx), wrap2(x + 2, k.nx)};
    p.Y = {wrap2(y - 2, k.ny) * k.nx, wrap2(y - 1, k.ny) * k.nx, y * k.nx, wrap2(y + 1, k.ny) * k.nx,
           wrap2(y + 2, k.ny) * k.nx};
    p.Z = {wrap2(z - 2, k.nz) * plane, wrap2(z - 1, k.nz) * plane, z * plane, wrap2(z + 1, k.nz) * plane,
           wrap2(z + 2, k.nz) * plane};
    bool b = sub != 0;
    p.hx[0] = b ? p.X.z0 : p.X.m1; p.hx[1] = b ? p.X.p1 : p.X.z0;
    p.hy[0] = b ? p.Y.z0 : p.Y.m1; p.hy[1] = b ? p.Y.p1 : p.Y.z0;
    p.hz[0] = b ? p.Z.z0 : p.Z.m1; p.hz[1] = b ? p.Z.p1 : p.Z.z0;
    return p;
}

template <int Q>
__device__ __forceinline__ unsigned pull_off(const PullMap &p)
{
    constexpr int cx = c2(Q, 0), cy = c2(Q, 1), cz = c2(Q, 2);
    if constexpr ((cx & 1) == 0) {
        return (unsigned)(p.own + p.Z.template at<-cz / 2>() + p.Y.template at<-cy / 2>() + p.X.template at<-cx / 2>());
    } else {
        return (unsigned)(p.oth + p.hz[cz > 0 ? 0 : 1] + p.hy[cy > 0 ? 0 : 1] + p.hx[cx > 0 ? 0 : 1]);
    }
}

template <typename S, int Q = 0>
__device__ __forceinline__ void load_periodic(const S *__restrict__ src, const PullMap &p, int ns, S *v)
{
    if constexpr (Q < NQ) {
        const S *__restrict__ base = src + (size_t)Q * ns;
        v[Q] = base[pull_off<Q>(p)];
        load_periodic<S, Q + 1>(src, p, ns, v);
    }
}

__device__ __forceinline__ int wrapc(int i, int n)
{
    // offsets are at most 2 cells: one correction suffices for n >= 2; n == 1 maps to 0
    if (n == 1) return 0;
    i += (i < 0) ? n : 0;
    i -= (i >= n) ? n : 0;
    if (i < 0) i += n;      // n == 2 with offset -2
    if (i >= n) i -= n;
    return i;
}

template <typename S> __device__ __forceinline__ double ref_of(int q, const Consts &k);
template <> __device__ __forceinline__ double ref_of<double>(int, const Consts &) { return 0.0; }
template <> __device__ __forceinline__ double ref_of<float>(int q, const Consts &k) { return k.w[shell_of(q)]; }

// Index of the population q pulled by site (x,y,z,sub): returns the array
// index and sets `ghost` (0 = interior, 1 = low-x ghost, 2 = high-x ghost).
template <int Q, bool BOUNDED>
__device__ __forceinline__ int pull_index(int x, int y, int z, int sub, const Consts &k, int &ghost)
{
    constexpr int cx = c2(Q, 0), cy = c2(Q, 1), cz = c2(Q, 2);
    int qx = 2 * x + sub - cx, qy = 2 * y + sub - cy, qz = 2 * z + sub - cz;
    int ssub = qx & 1;
    int sx = (qx - ssub) >> 1, sy = wrapc((qy - ssub) >> 1, k.ny), sz = wrapc((qz - ssub) >> 1, k.nz);
    ghost = 0;
    if (BOUNDED) {
        if (qx < 0 && k.bc[0] != PGK_PERIODIC) {
            ghost = 1;
            int slot = -qx - 1;
            return ((0 * NQ + Q) * NSLOT + slot) * k.nz * k.ny + sz * k.ny + sy;
        }
        if (qx > 2 * k.nx - 1 && k.bc[1] != PGK_PERIODIC) {
            ghost = 2;
            int slot = qx - 2 * k.nx;
            return ((1 * NQ + Q) * NSLOT + slot) * k.nz * k.ny + sz * k.ny + sy;
        }
    }
    sx = wrapc(sx, k.nx);
    return ((ssub * k.nz + sz) * k.ny + sy) * k.nx + sx;
}

template <typename S, bool BOUNDED, int Q>
__device__ __forceinline__ void load_one(const S *__restrict__ src, const S *__restrict__ gh,
                                         int x, int y, int z, int sub, const Consts &k, S *v)
{
    int ghost;
    int idx = pull_index<Q, BOUNDED>(x, y, z, sub, k, ghost);
    if (BOUNDED && ghost) v[Q] = gh[idx];
    else v[Q] = src[(size_t)Q * k.ns + idx];
}

template <typename S, bool BOUNDED, int Q = 0>
__device__ __forceinline__ void load_all(const S *__restrict__ src, const S *__restrict__ gh,
                                         int x, int y, int z, int sub, const Consts &k, S *v)
{
    if constexpr (Q < NQ) {
        load_one<S, BOUNDED, Q>(src, gh, x, y, z, sub, k, v);
        load_all<S, BOUNDED, Q + 1>(src, gh, x, y, z, sub, k, v);
    }
}

// Sums over the stored values v (g, or h = g - w): rho, j, Pi.
struct Mom {
    double rho, j[3], P[6];  // P: xx yy zz xy xz yz
};

template <typename S, int P = 0>
__device__ __forceinline__ void accumulate(const S *v, Mom &m)
{
    if constexpr (P < NPAIR) {
        constexpr int cx = Lattice::REP2[P][0], cy = Lattice::REP2[P][1], cz = Lattice::REP2[P][2];
        double a = (double)v[1 + P], b = (double)v[1 + NPAIR + P];
        double s = a + b, d = a - b;
        m.rho += s;
        if (cx) m.j[0] += (0.5 * cx) * d;
        if (cy) m.j[1] += (0.5 * cy) * d;
        if (cz) m.j[2] += (0.5 * cz) * d;
        if (cx) m.P[0] += (0.25 * cx * cx) * s;
        if (cy) m.P[1] += (0.25 * cy * cy) * s;
        if (cz) m.P[2] += (0.25 * cz * cz) * s;
        if (cx * cy) m.P[3] += (0.25 * cx * cy) * s;
        if (cx * cz) m.P[4] += (0.25 * cx * cz) * s;
        if (cy * cz) m.P[5] += (0.25 * cy * cz) * s;
        accumulate<S, P + 1>(v, m);
    }
}

template <typename S>
__device__ __forceinline__ Mom moments(const S *v, const Consts &k)
{
    Mom m;
    m.rho = (double)v[0];
    m.j[0] = m.j[1] = m.j[2] = 0.0;
    for (int i = 0; i < 6; i++) m.P[i] = 0.0;
    accumulate<S>(v, m);
    if (sizeof(S) == 4) {
        // deviations from w_i (rho0 = 1): add the moments of the weights
        m.rho += 1.0;
        m.P[0] += k.th0;
        m.P[1] += k.th0;
        m.P[2] += k.th0;
    }
    return m;
}

// Per-site solve (Sec. 5): g->f temperature map with the backward-Euler half
// relaxation, stress rescale, ES and BGK targets.  Everything in double.
struct Solve {
    double rho, u[3], a, r, T, R, theta;
    double sg[6];   // sigma(g)
    double lamF[6]; // covariance of the gain term F
};

__device__ __forceinline__ Solve site_solve(const Mom &m, double r, const Consts &k)
{
    Solve s;
    s.rho = m.rho;
    double ir = 1.0 / m.rho;
    for (int a = 0; a < 3; a++) s.u[a] = m.j[a] * ir;
    double uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    s.a = (m.P[0] + m.P[1] + m.P[2] - m.rho * uu) * ir * (1.0 / 3.0);
    s.sg[0] = m.P[0] - m.rho * s.u[0] * s.u[0] - m.rho * s.a;
    s.sg[1] = m.P[1] - m.rho * s.u[1] * s.u[1] - m.rho * s.a;
    s.sg[2] = m.P[2] - m.rho * s.u[2] * s.u[2] - m.rho * s.a;
    s.sg[3] = m.P[3] - m.rho * s.u[0] * s.u[1];
    s.sg[4] = m.P[4] - m.rho * s.u[0] * s.u[2];
    s.sg[5] = m.P[5] - m.rho * s.u[1] * s.u[2];
    s.r = r;
    // a = T + Y (T - R),  R = (r + X T)/(1 + X)
    s.T = (s.a * (1.0 + k.X) + k.Y * r) * k.inv1XY;
    s.R = (r + k.X * s.T) * k.inv1X;
    s.theta = (3.0 * s.T + k.delta * s.R) * k.inv3d;
    // lam_ES = T I + b sigma(f)/rho, sigma(f) = sigma(g)/s_sigma;
    // lam_F = (tau1 lam_ES + tau theta I)/(tau + tau1)
    double cb = k.wt1 * k.bs * ir;
    double iso = k.wt1 * s.T + k.wt * s.theta;
    for (int i = 0; i < 6; i++) s.lamF[i] = (i < 3 ? iso : 0.0) + cb * s.sg[i];
    return s;
}

// F3 coefficients in compute precision R.
template <typename R>
struct Eq {
    R u0, u1, u2;       // velocity
    R Du0, Du1, Du2;    // (lam - theta0 I) u
    R D0, D1, D2, D3, D4, D5;
    R k0;               // (u^2 + tr D)/(2 theta0)
    R A1;               // 1/theta0 - (u^2 + tr D)/(2 theta0^2)
    R k2;               // 1/(2 theta0^2)
    R k3;               // 1/(6 theta0^3)
    R k4;               // 1/(2 theta0^3)
    R k5;               // 1/theta0^2
    R rho, drho;        // rho, rho - 1
    R omb, tb;          // 1 - 2 beta, 2 beta
};

template <typename R>
__device__ __forceinline__ Eq<R> make_eq(const Solve &s, const Consts &k)
{
    double t = k.th0;
    double D[6];
    for (int i = 0; i < 6; i++) D[i] = s.lamF[i] - (i < 3 ? t : 0.0);
    double uu = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
    double trD = D[0] + D[1] + D[2];
    Eq<R> e;
    e.u0 = (R)s.u[0]; e.u1 = (R)s.u[1]; e.u2 = (R)s.u[2];
    e.Du0 = (R)(D[0] * s.u[0] + D[3] * s.u[1] + D[4] * s.u[2]);
    e.Du1 = (R)(D[3] * s.u[0] + D[1] * s.u[1] + D[5] * s.u[2]);
    e.Du2 = (R)(D[4] * s.u[0] + D[5] * s.u[1] + D[2] * s.u[2]);
    e.D0 = (R)D[0]; e.D1 = (R)D[1]; e.D2 = (R)D[2]; e.D3 = (R)D[3]; e.D4 = (R)D[4]; e.D5 = (R)D[5];
    e.k0 = (R)((uu + trD) * k.i2t);
    e.A1 = (R)(k.it - (uu + trD) * k.ih2);
    e.k2 = (R)k.ih2;
    e.k3 = (R)k.i6t3;
    e.k4 = (R)k.i2t3;
    e.k5 = (R)k.it2;
    e.rho = (R)s.rho;
    e.drho = (R)(s.rho - 1.0);
    e.omb = (R)(1.0 - 2.0 * k.beta);
    e.tb = (R)(2.0 * k.beta);
    return e;
}

// Collide the pair (+c_P, -c_P) and the rest population, write the own site.
template <typename S, int P = 0>
__device__ __forceinline__ void collide_store(S *v, const Eq<S> &e, const Consts &k, S *__restrict__ dst, int s)
{
    if constexpr (P < NPAIR) {
        constexpr int cx = Lattice::REP2[P][0], cy = Lattice::REP2[P][1], cz = Lattice::REP2[P][2];
        constexpr S hx = (S)(0.5 * cx), hy = (S)(0.5 * cy), hz = (S)(0.5 * cz);
        S cu = hx * e.u0 + hy * e.u1 + hz * e.u2;
        S cDc = hx * hx * e.D0 + hy * hy * e.D1 + hz * hz * e.D2
              + (S)2 * (hx * hy * e.D3 + hx * hz * e.D4 + hy * hz * e.D5);
        S cDu = hx * e.Du0 + hy * e.Du1 + hz * e.Du2;
        S even = (cu * cu + cDc) * e.k2 - e.k0;
        S odd = cu * e.A1 + cu * cu * cu * e.k3 + cDc * cu * e.k4 - cDu * e.k5;
        if constexpr (sizeof(S) == 4) {
            // deviation form: F - w = w [(rho - 1) + rho (even +- odd)], with w
            // carried as hi + lo floats so the rounding of w adds no bias to the
            // moments of F; h* = h + 2 beta (F - w - h) conserves the moments of
            // the collision whatever the rounding of 2 beta
            S wh = k.whi[Lattice::SHELL[P]], wl = k.wlo[Lattice::SHELL[P]];
            S Xp = e.drho + e.rho * (even + odd), Xm = e.drho + e.rho * (even - odd);
            S Fp = wh * Xp + wl * Xp, Fm = wh * Xm + wl * Xm;
            // the next read of these values is a step away: stream them past the caches
            __builtin_nontemporal_store(v[1 + P] + e.tb * (Fp - v[1 + P]), &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(v[1 + NPAIR + P] + e.tb * (Fm - v[1 + NPAIR + P]),
                                        &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        } else {
            S w = (S)k.w[Lattice::SHELL[P]];
            S Fp = w * e.rho * ((S)1 + even + odd);
            S Fm = w * e.rho * ((S)1 + even - odd);
            __builtin_nontemporal_store(e.omb * v[1 + P] + e.tb * Fp, &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(e.omb * v[1 + NPAIR + P] + e.tb * Fm, &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        }
        collide_store<S, P + 1>(v, e, k, dst, s);
    } else {
        if constexpr (sizeof(S) == 4) {
            S X0 = e.drho - e.rho * e.k0;
            S F0 = k.whi[0] * X0 + k.wlo[0] * X0;
            __builtin_nontemporal_store(v[0] + e.tb * (F0 - v[0]), &dst[s]);
        } else {
            S w0 = (S)k.w[0];
            __builtin_nontemporal_store(e.omb * v[0] + e.tb * (w0 * e.rho * ((S)1 - e.k0)), &dst[s]);
        }
    }
}

// block-wide sum of NV doubles; thread 0 of the block gets the result
template <int NV>
__device__ __forceinline__ void block_sum(double *val, double *out)
{
    __shared__ double red[WG / 64][NV];
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < NV; c++) val[c] += __shfl_xor(val[c], off, 64);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < NV; c++) red[wv][c] = val[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int c = 0; c < NV; c++) {
            double t = 0.0;
            for (int i = 0; i < WG / 64; i++) t += red[i][c];
            out[c] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// k_lb: fused pull - moments - solve - equilibrium - collide
// ---------------------------------------------------------------------------
template <typename S, typename A, int VAR, bool BOUNDED, bool REDUCE>
__global__ __launch_bounds__(WG) void k_lb(const S *__restrict__ src, S *__restrict__ dst,
                                           const S *__restrict__ gh, double *__restrict__ thR,
                                           double *__restrict__ that_, A *__restrict__ aux,
                                           double *__restrict__ partial, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    double red[5] = {0, 0, 0, 0, 0};
    if (s < k.ns) {
        int x, y, z, sub;
        decode(s, k, x, y, z, sub);
        S v[NQ];
        if constexpr (BOUNDED) load_all<S, true>(src, gh, x, y, z, sub, k, v);
        else load_periodic<S>(src, pull_map(x, y, z, sub, k), k.ns, v);
        double r = thR[s];
        Mom m = moments<S>(v, k);
        Solve so = site_solve(m, r, k);
        Eq<S> e = make_eq<S>(so, k);
        collide_store<S>(v, e, k, dst, s);
        that_[s] = so.R;                                  // theta_R after step 1
        if (VAR == PGK_LIT) thR[s] = so.T;                // the printed second half needs theta_T
        aux[s] = (A)so.u[0];
        aux[(size_t)k.ns + s] = (A)so.u[1];
        aux[(size_t)2 * k.ns + s] = (A)so.u[2];
        aux[(size_t)3 * k.ns + s] = (A)so.rho;
        aux[(size_t)4 * k.ns + s] = (A)(so.rho * so.theta);
        if (REDUCE) {
            red[0] = m.rho;
            red[1] = m.j[0];
            red[2] = m.j[1];
            red[3] = m.j[2];
            red[4] = 0.5 * (m.P[0] + m.P[1] + m.P[2]) + 0.5 * k.delta * m.rho * r;
        }
    }
    if (REDUCE) block_sum<5>(red, partial + (size_t)blockIdx.x * 5);
}

// ---------------------------------------------------------------------------
// theta_R transport
// ---------------------------------------------------------------------------
// same-sublattice neighbour along axis a (0,1,2) by dir (+-1); returns -1 / -2
// for the low / high x ghost of a bounded face
template <bool BOUNDED>
__device__ __forceinline__ int nbr(int x, int y, int z, int sub, int a, int dir, const Consts &k)
{
    int c[3] = {x, y, z};
    int n[3] = {k.nx, k.ny, k.nz};
    c[a] += dir;
    if (BOUNDED && a == 0) {
        if (c[0] < 0 && k.bc[0] != PGK_PERIODIC) return -1;
        if (c[0] >= k.nx && k.bc[1] != PGK_PERIODIC) return -2;
    }
    c[a] = wrapc(c[a], n[a]);
    return ((sub * k.nz + c[2]) * k.ny + c[1]) * k.nx + c[0];
}

template <typename A, bool BOUNDED>
__device__ __forceinline__ double theta_star(const double *__restrict__ th, const A *__restrict__ aux,
                                             int idx, const Consts &k)
{
    // predictor at site idx (forward differences); ghosts keep their value
    if (BOUNDED && idx < 0) return k.thbc[idx == -1 ? 0 : 1];
    int x, y, z, sub;
    decode(idx, k, x, y, z, sub);
    double t = th[idx], adv = 0.0;
    for (int a = 0; a < 3; a++) {
        int p = nbr<BOUNDED>(x, y, z, sub, a, +1, k);
        double tp = (BOUNDED && p < 0) ? k.thbc[p == -1 ? 0 : 1] : th[p];
        adv += (double)aux[(size_t)a * k.ns + idx] * (tp - t);
    }
    return t - adv;
}

template <typename A, bool BOUNDED>
__global__ __launch_bounds__(WG) void k_mc(const double *__restrict__ that_, const A *__restrict__ aux,
                                           double *__restrict__ tmc, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s >= k.ns) return;
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    double ts = theta_star<A, BOUNDED>(that_, aux, s, k);
    double adv = 0.0;
    for (int a = 0; a < 3; a++) {
        int m = nbr<BOUNDED>(x, y, z, sub, a, -1, k);
        double tm = theta_star<A, BOUNDED>(that_, aux, m, k);
        adv += (double)aux[(size_t)a * k.ns + s] * (ts - tm);
    }
    tmc[s] = 0.5 * (that_[s] + ts - adv);
}

template <typename A, int VAR, bool BOUNDED>
__global__ __launch_bounds__(WG) void k_dif(const double *__restrict__ tmc, const double *__restrict__ that_,
                                            const A *__restrict__ aux, double *__restrict__ thR, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s >= k.ns) return;
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    double rho = (double)aux[(size_t)3 * k.ns + s];
    double ks = k.kfac * (double)aux[(size_t)4 * k.ns + s];
    double t = tmc[s];
    double flux = 0.0, lap = 0.0;
    for (int a = 0; a < 3; a++)
        for (int dir = -1; dir <= 1; dir += 2) {
            int q = nbr<BOUNDED>(x, y, z, sub, a, dir, k);
            double tq, kq;
            if (BOUNDED && q < 0) {
                int side = q == -1 ? 0 : 1;
                tq = k.thbc[side];
                double rg = k.bc[side] == PGK_WALL ? rho : k.rhobc[side];
                kq = k.kfac * rg * tq;
            } else {
                tq = tmc[q];
                kq = k.kfac * (double)aux[(size_t)4 * k.ns + q];
            }
            flux += 0.5 * (ks + kq) * (tq - t);
            lap += tq - t;
        }
    double v = thR[s];
    if (VAR == PGK_CN) {
        // second half: repeat the first-half increment R - r
        thR[s] = t + 2.0 * flux / (rho * k.delta) + (that_[s] - v);
    } else {
        double DR = 2.0 * ks / (rho * k.delta);
        thR[s] = (t + DR * lap + k.X * v) / (1.0 + k.X);
    }
}

// ---------------------------------------------------------------------------
// k_tr: fused theta_R transport on periodic grids (steps 2-4 in one pass).
// A work-group owns a TX x TY tile of one sublattice and marches through TZ
// z-planes.  Rolling LDS rings hold the planes each stage needs:
//   theta_hat  (planes z, z+1)   region [-2, TX+2) x [-2, TY+2)
//   theta*     (planes z-1, z)   region [-2, TX+1) x [-2, TY+1)
//   theta^mc   (planes z-2..z)   region [-1, TX+1) x [-1, TY+1)
//   rho*theta  (planes z-2..z)   region [-1, TX+1) x [-1, TY+1)
//   u          (plane z)         region [-2, TX+1) x [-2, TY+1)
// At plane z the group computes theta*(z), theta^mc(z) and the diffused,
// fully relaxed theta_R at plane z-1.  Every value entering a stencil is
// staged once per group; HBM sees each field about once.
// ---------------------------------------------------------------------------
constexpr int TX = 64, TY = 4, TZ = 32;
constexpr int HX = TX + 4, HY = TY + 4;     // theta_hat plane (origin -2)
constexpr int SX = TX + 3, SY = TY + 3;     // theta* and u plane (origin -2)
constexpr int MX = TX + 2, MY = TY + 2;     // theta^mc and rho*theta plane (origin -1)
constexpr int NH = (HX * HY + WG - 1) / WG; // staged points per thread
constexpr int NS = (SX * SY + WG - 1) / WG;
constexpr int NM = (MX * MY + WG - 1) / WG;

__device__ __forceinline__ int wrapn(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename A, int VAR>
__global__ __launch_bounds__(WG) void k_tr(const double *__restrict__ that_, const A *__restrict__ aux,
                                           double *__restrict__ thR, Consts k)
{
    __shared__ double l_th[2][HY * HX];
    __shared__ double l_ts[2][SY * SX];
    __shared__ double l_mc[3][MY * MX];
    __shared__ A l_pt[3][MY * MX];
    __shared__ A l_u[3][SY * SX];

    const int nbx = (k.nx + TX - 1) / TX, nby = (k.ny + TY - 1) / TY, nbz = (k.nz + TZ - 1) / TZ;
    // work-groups are dispatched round-robin over the 8 XCDs (each with its own
    // L2); give every XCD a contiguous run of tiles so that the halos shared by
    // neighbouring tiles are fetched into one L2
    int b;
    {
        const int n = gridDim.x, q = n / 8, r = n % 8, i = blockIdx.x, xcd = i % 8, kk = i / 8;
        b = xcd < r ? xcd * (q + 1) + kk : r * (q + 1) + (xcd - r) * q + kk;
    }
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nby;
    b /= nby;
    const int bz = b % nbz;
    const int sub = b / nbz;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int zend = min(z0 + TZ, k.nz);   // planes [z0, zend) are produced
    const int plane = k.nx * k.ny;
    const int subo = sub * plane * k.nz;
    const int tid = threadIdx.x;

    // plane-invariant (x, y) offsets of the points this thread stages
    int oh[NH], os[NS], om[NM];
#pragma unroll
    for (int j = 0; j < NH; j++) {
        int i = min(tid + j * WG, HX * HY - 1);
        int ly = i / HX, lx = i - ly * HX;
        oh[j] = wrapn(y0 + ly - 2, k.ny) * k.nx + wrapn(x0 + lx - 2, k.nx);
    }
#pragma unroll
    for (int j = 0; j < NS; j++) {
        int i = min(tid + j * WG, SX * SY - 1);
        int ly = i / SX, lx = i - ly * SX;
        os[j] = wrapn(y0 + ly - 2, k.ny) * k.nx + wrapn(x0 + lx - 2, k.nx);
    }
#pragma unroll
    for (int j = 0; j < NM; j++) {
        int i = min(tid + j * WG, MX * MY - 1);
        int ly = i / MX, lx = i - ly * MX;
        om[j] = wrapn(y0 + ly - 1, k.ny) * k.nx + wrapn(x0 + lx - 1, k.nx);
    }
    const int lxo = tid % TX, lyo = tid / TX;
    const bool outv = (x0 + lxo < k.nx) && (y0 + lyo < k.ny);
    const int oo = outv ? (y0 + lyo) * k.nx + (x0 + lxo) : 0;
    auto zoff = [&](int z) { return subo + wrapn(z, k.nz) * plane; };

    // registers carrying the next plane's data
    double r_th[NH];
    A r_u[3][NS], r_pt[NM];
    auto fetch = [&](int zth, int zu) {
        int zt = zoff(zth), zuo = zoff(zu);
#pragma unroll
        for (int j = 0; j < NH; j++) r_th[j] = that_[zt + oh[j]];
#pragma unroll
        for (int j = 0; j < NS; j++) {
            r_u[0][j] = aux[zuo + os[j]];
            r_u[1][j] = aux[(size_t)k.ns + zuo + os[j]];
            r_u[2][j] = aux[(size_t)2 * k.ns + zuo + os[j]];
        }
#pragma unroll
        for (int j = 0; j < NM; j++) r_pt[j] = aux[(size_t)4 * k.ns + zuo + om[j]];
    };
    auto stash = [&](int slot_th, int slot3) {
#pragma unroll
        for (int j = 0; j < NH; j++)
            if (tid + j * WG < HX * HY) l_th[slot_th][tid + j * WG] = r_th[j];
#pragma unroll
        for (int j = 0; j < NS; j++)
            if (tid + j * WG < SX * SY) {
                l_u[0][tid + j * WG] = r_u[0][j];
                l_u[1][tid + j * WG] = r_u[1][j];
                l_u[2][tid + j * WG] = r_u[2][j];
            }
#pragma unroll
        for (int j = 0; j < NM; j++)
            if (tid + j * WG < MX * MY) l_pt[slot3][tid + j * WG] = r_pt[j];
    };

    // prologue: theta_hat(z0-2) straight into its slot, then the data of plane z0-2
    {
        int zt = zoff(z0 - 2);
#pragma unroll
        for (int j = 0; j < NH; j++)
            if (tid + j * WG < HX * HY) l_th[(z0 + 2) & 1][tid + j * WG] = that_[zt + oh[j]];
    }
    fetch(z0 - 1, z0 - 2);
    double o_rho = 0.0, o_v = 0.0, o_th = 0.0;

    for (int zz = z0 - 2; zz <= zend; zz++) {
        const int rz = zz + 4;                          // non-negative ring index
        stash((rz + 1) & 1, rz % 3);                   // theta_hat(zz+1), u(zz), rho theta(zz)
        if (zz < zend) fetch(zz + 2, zz + 1);          // in flight during this plane
        const int zo = zz - 1;                          // output plane of this iteration
        if (zz >= z0 + 1 && outv) {
            int g = zoff(zo) + oo;
            o_rho = (double)aux[(size_t)3 * k.ns + g];
            o_v = thR[g];
            o_th = that_[g];
        }
        __syncthreads();
        // predictor theta*(zz) = th - sum_a u_a (th(+e_a) - th), region origin -2
        for (int i = tid; i < SY * SX; i += WG) {
            int ly = i / SX, lx = i - ly * SX;
            int h = ly * HX + lx;
            double t = l_th[rz & 1][h];
            double adv = (double)l_u[0][i] * (l_th[rz & 1][h + 1] - t)
                       + (double)l_u[1][i] * (l_th[rz & 1][h + HX] - t)
                       + (double)l_u[2][i] * (l_th[(rz + 1) & 1][h] - t);
            l_ts[rz & 1][i] = t - adv;
        }
        __syncthreads();
        // corrector theta^mc(zz) = 1/2 [th + th* - sum_a u_a (th* - th*(-e_a))], origin -1
        if (zz > z0 - 2) {
            for (int i = tid; i < MY * MX; i += WG) {
                int ly = i / MX, lx = i - ly * MX;
                int sI = (ly + 1) * SX + lx + 1, hI = (ly + 1) * HX + lx + 1;
                double ts = l_ts[rz & 1][sI];
                double adv = (double)l_u[0][sI] * (ts - l_ts[rz & 1][sI - 1])
                           + (double)l_u[1][sI] * (ts - l_ts[rz & 1][sI - SX])
                           + (double)l_u[2][sI] * (ts - l_ts[(rz + 1) & 1][sI]);
                l_mc[rz % 3][i] = 0.5 * (l_th[rz & 1][hI] + ts - adv);
            }
        }
        __syncthreads();
        // diffusion and second half at plane zz-1
        if (zz >= z0 + 1 && outv) {
            const int rc = (rz + 2) % 3, rm = (rz + 1) % 3, rp = rz % 3;
            int c = (lyo + 1) * MX + lxo + 1;
            double t = l_mc[rc][c];
            double ks = k.kfac * (double)l_pt[rc][c];
            double tq[6] = {l_mc[rc][c - 1], l_mc[rc][c + 1], l_mc[rc][c - MX], l_mc[rc][c + MX],
                            l_mc[rm][c], l_mc[rp][c]};
            double kq[6] = {(double)l_pt[rc][c - 1], (double)l_pt[rc][c + 1], (double)l_pt[rc][c - MX],
                            (double)l_pt[rc][c + MX], (double)l_pt[rm][c], (double)l_pt[rp][c]};
            double flux = 0.0, lap = 0.0;
#pragma unroll
            for (int q = 0; q < 6; q++) {
                flux += 0.5 * (ks + k.kfac * kq[q]) * (tq[q] - t);
                lap += tq[q] - t;
            }
            int g = zoff(zo) + oo;
            if (VAR == PGK_CN) {
                thR[g] = t + 2.0 * flux / (o_rho * k.delta) + (o_th - o_v);
            } else {
                double DR = 2.0 * ks / (o_rho * k.delta);
                thR[g] = (t + DR * lap + k.X * o_v) * k.inv1X;
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// boundaries: x ghost populations
// ---------------------------------------------------------------------------
// One thread per (side, ghost column gz*ny+gy).  Diffuse wall: the density of
// the re-emitted populations balances the mass that left through the face in
// the last collision (zero net mass flux per column); Dirichlet: equilibrium.
template <typename S>
__global__ void k_bc(const S *__restrict__ src, S *__restrict__ gh, Consts k)
{
    int col = blockIdx.x * blockDim.x + threadIdx.x;
    int ncol = k.ny * k.nz;
    if (col >= 2 * ncol) return;
    int side = col / ncol;
    col -= side * ncol;
    if (k.bc[side] == PGK_PERIODIC) return;
    int gy = col % k.ny, gz = col / k.ny;
    double scale = 1.0;
    if (k.bc[side] == PGK_WALL) {
        double out = 0.0;
        for (int q = 1; q < NQ; q++) {
            int cx = c2(q, 0), cy = c2(q, 1), cz = c2(q, 2);
            if ((side == 0 && cx >= 0) || (side == 1 && cx <= 0)) continue;
            for (int sub = 0; sub < 2; sub++)
                for (int xi = 0; xi < 2; xi++) {
                    int x = side == 0 ? xi : k.nx - 1 - xi;
                    if (x < 0 || x >= k.nx) continue;
                    if (xi == 1 && k.nx == 1) continue;
                    int dx = 2 * x + sub + cx;
                    bool crosses = side == 0 ? dx < 0 : dx > 2 * k.nx - 1;
                    if (!crosses) continue;
                    // ghost column of the destination: floor((2y + sub + cy)/2) = y + floor((sub + cy)/2)
                    int ky = (sub + cy) >= 0 ? (sub + cy) / 2 : -((-(sub + cy) + 1) / 2);
                    int kz = (sub + cz) >= 0 ? (sub + cz) / 2 : -((-(sub + cz) + 1) / 2);
                    int y = wrapc(gy - ky, k.ny), z = wrapc(gz - kz, k.nz);
                    if (k.ny == 1) y = 0;
                    if (k.nz == 1) z = 0;
                    int s = ((sub * k.nz + z) * k.ny + y) * k.nx + x;
                    out += (double)src[(size_t)q * k.ns + s] + (sizeof(S) == 4 ? k.w[shell_of(q)] : 0.0);
                }
        }
        scale = out / k.in_col[side];
    }
    for (int q = 0; q < NQ; q++) {
        double val = scale * k.Fbc[side][q] - (sizeof(S) == 4 ? k.w[shell_of(q)] : 0.0);
        for (int slot = 0; slot < NSLOT; slot++)
            gh[((side * NQ + q) * NSLOT + slot) * ncol + col] = (S)val;
    }
}

// ---------------------------------------------------------------------------
// initial state, moments, totals
// ---------------------------------------------------------------------------
// Push F_i(rho, u, theta_T I) of each site to where the next pull reads it:
// population i of site x is read from position x - c_i (a ghost slot when
// that lies beyond a bounded face).
template <typename S, bool BOUNDED>
__global__ __launch_bounds__(WG) void k_init(S *__restrict__ dst, S *__restrict__ gh, double *__restrict__ thR,
                                             const double *__restrict__ rho, const double *__restrict__ u,
                                             const double *__restrict__ thT, const double *__restrict__ thRin,
                                             Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s >= k.ns) return;
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    Solve so;
    so.rho = rho[s];
    so.u[0] = u[s];
    so.u[1] = u[(size_t)k.ns + s];
    so.u[2] = u[(size_t)2 * k.ns + s];
    for (int i = 0; i < 6; i++) so.lamF[i] = i < 3 ? thT[s] : 0.0;
    Eq<double> e = make_eq<double>(so, k);
    thR[s] = thRin[s];
    for (int q = 0; q < NQ; q++) {
        int cx = c2(q, 0), cy = c2(q, 1), cz = c2(q, 2);
        double hx = 0.5 * cx, hy = 0.5 * cy, hz = 0.5 * cz;
        double cu = hx * e.u0 + hy * e.u1 + hz * e.u2;
        double cDc = hx * hx * e.D0 + hy * hy * e.D1 + hz * hz * e.D2 + 2.0 * (hx * hy * e.D3 + hx * hz * e.D4 + hy * hz * e.D5);
        double cDu = hx * e.Du0 + hy * e.Du1 + hz * e.Du2;
        double even = (cu * cu + cDc) * e.k2 - e.k0;
        double odd = cu * e.A1 + cu * cu * cu * e.k3 + cDc * cu * e.k4 - cDu * e.k5;
        double w = k.w[shell_of(q)];
        double F = w * e.rho * (1.0 + even + odd);
        S val = (S)(sizeof(S) == 4 ? w * (e.drho + e.rho * (even + odd)) : F);
        // destination: position x - c_q
        int qx = 2 * x + sub - cx, qy = 2 * y + sub - cy, qz = 2 * z + sub - cz;
        int ssub = qx & 1;
        int sy = wrapc((qy - ssub) >> 1, k.ny), sz = wrapc((qz - ssub) >> 1, k.nz);
        if (BOUNDED && qx < 0 && k.bc[0] != PGK_PERIODIC) {
            gh[((0 * NQ + q) * NSLOT + (-qx - 1)) * k.nz * k.ny + sz * k.ny + sy] = val;
        } else if (BOUNDED && qx > 2 * k.nx - 1 && k.bc[1] != PGK_PERIODIC) {
            gh[((1 * NQ + q) * NSLOT + (qx - 2 * k.nx)) * k.nz * k.ny + sz * k.ny + sy] = val;
        } else {
            int sx = wrapc((qx - ssub) >> 1, k.nx);
            dst[(size_t)q * k.ns + ((ssub * k.nz + sz) * k.ny + sy) * k.nx + sx] = val;
        }
    }
}

template <typename S, bool BOUNDED, bool REDUCE>
__global__ __launch_bounds__(WG) void k_moments(const S *__restrict__ src, const S *__restrict__ gh,
                                                const double *__restrict__ thR, double *__restrict__ orho,
                                                double *__restrict__ ou, double *__restrict__ othT,
                                                double *__restrict__ othR, double *__restrict__ oP,
                                                double *__restrict__ partial, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    double red[5] = {0, 0, 0, 0, 0};
    if (s < k.ns) {
        int x, y, z, sub;
        decode(s, k, x, y, z, sub);
        S v[NQ];
        if constexpr (BOUNDED) load_all<S, true>(src, gh, x, y, z, sub, k, v);
        else load_periodic<S>(src, pull_map(x, y, z, sub, k), k.ns, v);
        double r = thR[s];
        Mom m = moments<S>(v, k);
        if (REDUCE) {
            red[0] = m.rho;
            red[1] = m.j[0];
            red[2] = m.j[1];
            red[3] = m.j[2];
            red[4] = 0.5 * (m.P[0] + m.P[1] + m.P[2]) + 0.5 * k.delta * m.rho * r;
        } else {
            Solve so = site_solve(m, r, k);
            if (orho) orho[s] = so.rho;
            if (ou) {
                ou[s] = so.u[0];
                ou[(size_t)k.ns + s] = so.u[1];
                ou[(size_t)2 * k.ns + s] = so.u[2];
            }
            if (othT) othT[s] = so.T;
            if (othR) othR[s] = so.r;
            if (oP) {
                // P(f) = rho u u + rho T I + sigma(g)/s_sigma
                const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
                for (int c = 0; c < 6; c++)
                    oP[(size_t)c * k.ns + s] = so.rho * so.u[ia[c]] * so.u[ib[c]] + (c < 3 ? so.rho * so.T : 0.0)
                                             + so.sg[c] / k.ssig;
            }
        }
    }
    if (REDUCE) block_sum<5>(red, partial + (size_t)blockIdx.x * 5);
}

__global__ void k_sum_partials(const double *__restrict__ partial, int nblk, double *__restrict__ out)
{
    // one block of WG threads; deterministic order
    double acc[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nblk; i += WG)
        for (int c = 0; c < 5; c++) acc[c] += partial[(size_t)i * 5 + c];
    block_sum<5>(acc, out);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// F3 on the host for boundary equilibria: rho, u, isotropic temperature theta
static void f3_host(double th0, const double w6[6], double rho, const double u[3], double theta, double F[NQ])
{
    double D = theta - th0;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double trD = 3.0 * D;
    for (int q = 0; q < NQ; q++) {
        double c[3] = {0.5 * c2(q, 0), 0.5 * c2(q, 1), 0.5 * c2(q, 2)};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
        double cDc = D * cc, cDu = D * cu;
        double a2 = cu * cu + cDc - th0 * (uu + trD);
        double a3 = cu * cu * cu + 3.0 * cDc * cu - th0 * (3.0 * uu * cu + 6.0 * cDu + 3.0 * trD * cu);
        F[q] = w6[shell_of(q)] * rho * (1.0 + cu / th0 + a2 / (2 * th0 * th0) + a3 / (6 * th0 * th0 * th0));
    }
}

}  // namespace pgk

using namespace pgk;

struct pgk_ctx {
    pgk_grid g{};
    hipStream_t stream = nullptr;
    void *buf[PGK_NBUF] = {nullptr, nullptr, nullptr, nullptr};
    size_t bytes[PGK_NBUF] = {0, 0, 0, 0};
    bool bound = false, params_set = false, initialised = false;
    int cur = 0;                  // which population buffer holds the state
    int64_t steps = 0;
    Consts k{};
    pgk_resolved res{};
    double bc_u[2][3]{};
    std::string err;
    // carved from the aux buffer
    double *that_ = nullptr, *tmc = nullptr, *partial = nullptr, *totals = nullptr;
    void *aux = nullptr, *gh = nullptr;
    int nblk = 0;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> events;   // pool
    std::vector<int> marks;           // kernel id of the interval ending at event i (-1: start)
    size_t nev = 0;
    ~pgk_ctx()
    {
        for (auto e : events) (void)hipEventDestroy(e);
    }
};

// record an event on the context stream closing an interval of kernel `id`
// (id < 0 opens a new sequence)
static void mark(pgk_ctx *c, int id)
{
    if (!c->timing) return;
    if (c->nev == c->events.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) { c->timing = false; return; }
        c->events.push_back(e);
        c->marks.push_back(-1);
    }
    (void)hipEventRecord(c->events[c->nev], c->stream);
    c->marks[c->nev] = id;
    c->nev++;
}

// magic numbers for q = (umulhi(n, m) + n) >> sh = n / d, valid for n < 2^31
static void magic_div(unsigned d, unsigned &m, int &sh)
{
    int s = 0;
    while ((1ull << s) < d) s++;
    m = (unsigned)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
    sh = s;
}

static int fail(pgk_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHECK(ctx, call)                                                               \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, PGK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static bool grid_ok(const pgk_grid *g)
{
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return false;
    if ((long long)g->nx * g->ny * g->nz * 2 > (long long)INT_MAX) return false;  // site ids are int
    if (g->precision != PGK_FP64 && g->precision != PGK_FP32DEV) return false;
    if (g->variant != PGK_CN && g->variant != PGK_LIT) return false;
    if (g->equilibrium != PGK_F3) return false;
    for (int s = 0; s < 2; s++)
        if (g->bc_x[s] < PGK_PERIODIC || g->bc_x[s] > PGK_DIRICHLET) return false;
    if ((g->bc_x[0] == PGK_PERIODIC) != (g->bc_x[1] == PGK_PERIODIC)) return false;
    if (g->bc_x[0] != PGK_PERIODIC && g->nx < 2) return false;
    return true;
}

// aux layout (bytes, each part 256-aligned): that_[ns] f64, tmc[ns] f64,
// aux fields [5][ns] (f64 or f32), partial[nblk*5] f64, totals[8] f64,
// ghosts [2][41][4][nz*ny] (population type)
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void aux_layout(const pgk_grid *g, size_t off[7])
{
    size_t ns = 2ull * g->nx * g->ny * g->nz;
    size_t elt = g->precision == PGK_FP64 ? 8 : 4;
    size_t nblk = (ns + WG - 1) / WG;
    off[0] = 0;
    off[1] = off[0] + align256(ns * 8);
    off[2] = off[1] + align256(ns * 8);
    off[3] = off[2] + align256(5 * ns * elt);
    off[4] = off[3] + align256(nblk * 5 * 8);
    off[5] = off[4] + align256(8 * 8);
    off[6] = off[5] + align256(2ull * NQ * NSLOT * g->ny * g->nz * elt);
}

extern "C" int pgk_buffer_sizes(const pgk_grid *g, size_t sizes[PGK_NBUF])
{
    if (!grid_ok(g) || !sizes) return PGK_EINVAL;
    size_t ns = 2ull * g->nx * g->ny * g->nz;
    size_t elt = g->precision == PGK_FP64 ? 8 : 4;
    size_t off[7];
    aux_layout(g, off);
    sizes[PGK_BUF_POP0] = NQ * ns * elt;
    sizes[PGK_BUF_POP1] = NQ * ns * elt;
    sizes[PGK_BUF_THETAR] = ns * 8;
    sizes[PGK_BUF_AUX] = off[6];
    return PGK_OK;
}

extern "C" int pgk_resolve(const pgk_targets *t, pgk_resolved *out)
{
    if (!t || !out) return PGK_EINVAL;
    double th0 = t->theta0 > 0 ? t->theta0 : THETA0_PRINTED;
    double d = t->delta, nu = t->nu, Pr = t->Pr, lb = t->mub_over_mu;
    if (!(d >= 0) || !(nu > 0) || !(Pr > 0) || !(lb > 0)) return PGK_EINVAL;
    double cd = 2.0 * d / (3.0 * (3.0 + d));
    double b = t->b;
    if (std::isnan(b)) {
        double kr0 = std::isnan(t->kr) ? d / 5.0 : t->kr;
        double P = Pr * (1.0 + kr0) / (1.0 + d / 5.0);   // B/(B - b)
        double r = lb * P / cd - 1.0;                    // tau1/tau
        if (!(r > 0)) return PGK_EINFEASIBLE;
        double B = 1.0 + 1.0 / r;
        b = B * (1.0 - 1.0 / P);
        b = std::fmin(std::fmax(b, -0.5), 1.0);
    }
    if (!(b < 1.0) || b < -0.5) return PGK_EINFEASIBLE;
    double r = (lb / cd - 1.0) / (1.0 - b);              // eta_b/eta = cd (1 + (1-b) tau1/tau)
    if (!(r > 0)) return PGK_EINFEASIBLE;
    double B = 1.0 + 1.0 / r;
    double kr = (B / (B - b)) * (1.0 + d / 5.0) / Pr - 1.0;
    if (kr < -1e-12) return PGK_EINFEASIBLE;
    kr = std::fmax(kr, 0.0);
    double tau = nu * (B - b) / th0;
    pgk_resolved o{};
    o.tau = tau; o.tau1 = r * tau; o.b = b; o.kr = kr; o.delta = d; o.theta0 = th0;
    o.B = B;
    o.tau_star = tau * o.tau1 / (tau + o.tau1);
    o.beta = 1.0 / (2.0 * o.tau_star + 1.0);
    o.X = 3.0 / (2.0 * o.tau1 * (3.0 + d));
    o.Y = d / (2.0 * o.tau1 * (3.0 + d));
    o.s_sigma = 1.0 + 1.0 / (2.0 * o.tau_star) - b / (2.0 * tau);
    o.nu = th0 * tau / (B - b);
    o.mub_over_mu = cd * o.tau1 * (B - b) / tau;
    o.Pr = (B / (B - b)) * (1.0 + d / 5.0) / (1.0 + kr);
    o.gamma = (5.0 + d) / (3.0 + d);
    o.D_R = d > 0 ? 5.0 * kr * th0 * tau / (B * d) : 0.0;
    *out = o;
    return PGK_OK;
}

extern "C" int pgk_create(const pgk_grid *g, void *stream, pgk_ctx **out)
{
    if (!out) return PGK_EINVAL;
    *out = nullptr;
    if (!grid_ok(g)) return PGK_EINVAL;
    pgk_ctx *c = new pgk_ctx();
    c->g = *g;
    c->stream = (hipStream_t)stream;
    c->k.nx = g->nx; c->k.ny = g->ny; c->k.nz = g->nz;
    c->k.ns = 2 * g->nx * g->ny * g->nz;
    c->k.bc[0] = g->bc_x[0]; c->k.bc[1] = g->bc_x[1];
    magic_div((unsigned)g->nx, c->k.mx, c->k.shx);
    magic_div((unsigned)g->ny, c->k.my, c->k.shy);
    magic_div((unsigned)g->nz, c->k.mz, c->k.shz);
    c->nblk = (c->k.ns + WG - 1) / WG;
    *out = c;
    return PGK_OK;
}

extern "C" int pgk_bind(pgk_ctx *c, void *const bufs[PGK_NBUF], const size_t bytes[PGK_NBUF])
{
    if (!c || !bufs || !bytes) return PGK_EINVAL;
    size_t need[PGK_NBUF];
    pgk_buffer_sizes(&c->g, need);
    for (int i = 0; i < PGK_NBUF; i++) {
        if (!bufs[i]) return fail(c, PGK_EINVAL, "null buffer");
        if (bytes[i] < need[i]) return fail(c, PGK_ENOMEM, "buffer " + std::to_string(i) + " too small");
        if (((uintptr_t)bufs[i]) & 255) return fail(c, PGK_EINVAL, "buffers must be 256-byte aligned");
        c->buf[i] = bufs[i];
        c->bytes[i] = bytes[i];
    }
    size_t off[7];
    aux_layout(&c->g, off);
    char *a = (char *)bufs[PGK_BUF_AUX];
    c->that_ = (double *)(a + off[0]);
    c->tmc = (double *)(a + off[1]);
    c->aux = (void *)(a + off[2]);
    c->partial = (double *)(a + off[3]);
    c->totals = (double *)(a + off[4]);
    c->gh = (void *)(a + off[5]);
    c->bound = true;
    c->initialised = false;
    return PGK_OK;
}

static void fill_bc(pgk_ctx *c)
{
    Consts &k = c->k;
    for (int side = 0; side < 2; side++) {
        if (k.bc[side] == PGK_PERIODIC) continue;
        double rho = k.bc[side] == PGK_WALL ? 1.0 : k.rhobc[side];
        f3_host(k.th0, k.w, rho, c->bc_u[side], k.thbc[side], k.Fbc[side]);
        // mass re-emitted into one ghost column at unit density: every
        // population pulled from beyond the face, over both sublattices
        double in = 0.0;
        for (int q = 0; q < NQ; q++)
            for (int sub = 0; sub < 2; sub++)
                for (int x = 0; x < k.nx; x++) {
                    int qx = 2 * x + sub - c2(q, 0);
                    bool outside = side == 0 ? qx < 0 : qx > 2 * k.nx - 1;
                    if (outside) in += k.Fbc[side][q];
                }
        k.in_col[side] = in;
    }
}

extern "C" int pgk_set_params(pgk_ctx *c, const pgk_params *p, pgk_resolved *out)
{
    if (!c || !p) return PGK_EINVAL;
    if (!(p->tau > 0) || !(p->tau1 > 0) || !(p->delta >= 0) || p->b < -0.5 || p->b > 1.0 || !(p->kr >= 0))
        return fail(c, PGK_EINVAL, "parameters out of range");
    Consts &k = c->k;
    k.th0 = p->theta0 > 0 ? p->theta0 : THETA0_PRINTED;
    shell_weights(k.th0, k.w);
    for (int i = 0; i < 6; i++) {
        k.whi[i] = (float)k.w[i];
        k.wlo[i] = (float)(k.w[i] - (double)k.whi[i]);
    }
    k.tau = p->tau; k.tau1 = p->tau1; k.b = p->b; k.delta = p->delta;
    double taus = p->tau * p->tau1 / (p->tau + p->tau1);
    double B = 1.0 + p->tau / p->tau1;
    k.beta = 1.0 / (2.0 * taus + 1.0);
    k.X = 3.0 / (2.0 * p->tau1 * (3.0 + p->delta));
    k.Y = p->delta / (2.0 * p->tau1 * (3.0 + p->delta));
    k.ssig = 1.0 + 1.0 / (2.0 * taus) - p->b / (2.0 * p->tau);
    k.kfac = p->kr * 5.0 * p->tau / (2.0 * B);
    k.inv1X = 1.0 / (1.0 + k.X);
    k.inv1XY = 1.0 / (1.0 + k.X + k.Y);
    k.inv3d = 1.0 / (3.0 + p->delta);
    k.wt1 = p->tau1 / (p->tau + p->tau1);
    k.wt = p->tau / (p->tau + p->tau1);
    k.bs = p->b / k.ssig;
    double t = k.th0;
    k.it = 1.0 / t;
    k.i2t = 1.0 / (2.0 * t);
    k.ih2 = 1.0 / (2.0 * t * t);
    k.i6t3 = 1.0 / (6.0 * t * t * t);
    k.i2t3 = 1.0 / (2.0 * t * t * t);
    k.it2 = 1.0 / (t * t);
    pgk_resolved r{};
    r.tau = p->tau; r.tau1 = p->tau1; r.b = p->b; r.kr = p->kr; r.delta = p->delta; r.theta0 = k.th0;
    r.tau_star = taus; r.beta = k.beta; r.X = k.X; r.Y = k.Y; r.s_sigma = k.ssig; r.B = B;
    double cd = p->delta > 0 ? 2.0 * p->delta / (3.0 * (3.0 + p->delta)) : 0.0;
    r.nu = k.th0 * p->tau / (B - p->b);
    r.mub_over_mu = cd * p->tau1 * (B - p->b) / p->tau;
    r.Pr = (B / (B - p->b)) * (1.0 + p->delta / 5.0) / (1.0 + p->kr);
    r.gamma = (5.0 + p->delta) / (3.0 + p->delta);
    r.D_R = p->delta > 0 ? 5.0 * p->kr * k.th0 * p->tau / (B * p->delta) : 0.0;
    c->res = r;
    if (out) *out = r;
    c->params_set = true;
    fill_bc(c);
    return PGK_OK;
}

extern "C" int pgk_set_bc_x(pgk_ctx *c, int side, double rho, const double u[3], double theta)
{
    if (!c || side < 0 || side > 1 || !(theta > 0)) return PGK_EINVAL;
    if (c->k.bc[side] == PGK_PERIODIC) return fail(c, PGK_EINVAL, "face is periodic");
    if (c->k.bc[side] == PGK_DIRICHLET && !(rho > 0)) return fail(c, PGK_EINVAL, "Dirichlet density must be positive");
    if (u && u[0] != 0.0 && c->k.bc[side] == PGK_WALL) return fail(c, PGK_EINVAL, "a wall cannot move normal to itself");
    c->k.rhobc[side] = rho;
    c->k.thbc[side] = theta;
    for (int a = 0; a < 3; a++) c->bc_u[side][a] = u ? u[a] : 0.0;
    if (c->params_set) fill_bc(c);
    return PGK_OK;
}

static bool bounded(const pgk_ctx *c) { return c->k.bc[0] != PGK_PERIODIC; }

template <typename S>
static int init_t(pgk_ctx *c, const double *rho, const double *u, const double *thT, const double *thR)
{
    dim3 grid(c->nblk), block(WG);
    S *dst = (S *)c->buf[c->cur];
    if (bounded(c))
        hipLaunchKernelGGL((k_init<S, true>), grid, block, 0, c->stream, dst, (S *)c->gh,
                           (double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, c->k);
    else
        hipLaunchKernelGGL((k_init<S, false>), grid, block, 0, c->stream, dst, (S *)c->gh,
                           (double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, c->k);
    HIPCHECK(c, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_init_fields(pgk_ctx *c, const double *rho, const double *u, const double *thT, const double *thR)
{
    if (!c) return PGK_EINVAL;
    if (!c->bound) return fail(c, PGK_ENOTBOUND, "buffers not bound");
    if (!c->params_set) return fail(c, PGK_EINVAL, "parameters not set");
    if (!rho || !u || !thT || !thR) return fail(c, PGK_EINVAL, "null field");
    c->cur = 0;
    c->steps = 0;
    int rc = c->g.precision == PGK_FP64 ? init_t<double>(c, rho, u, thT, thR) : init_t<float>(c, rho, u, thT, thR);
    if (rc == PGK_OK) c->initialised = true;
    return rc;
}

template <typename S, typename A, int VAR, bool BND>
static int step_t(pgk_ctx *c, int64_t n)
{
    dim3 grid(c->nblk), block(WG);
    int nbc = (2 * c->k.ny * c->k.nz + 63) / 64;
    for (int64_t it = 0; it < n; it++) {
        S *src = (S *)c->buf[c->cur], *dst = (S *)c->buf[1 - c->cur];
        mark(c, -1);
        if (BND && c->steps > 0) {
            hipLaunchKernelGGL((k_bc<S>), dim3(nbc), dim3(64), 0, c->stream, src, (S *)c->gh, c->k);
            mark(c, 3);
        }
        hipLaunchKernelGGL((k_lb<S, A, VAR, BND, false>), grid, block, 0, c->stream, src, dst, (const S *)c->gh,
                           (double *)c->buf[PGK_BUF_THETAR], c->that_, (A *)c->aux, c->partial, c->k);
        mark(c, 0);
        if constexpr (BND) {
            hipLaunchKernelGGL((k_mc<A, BND>), grid, block, 0, c->stream, c->that_, (const A *)c->aux, c->tmc, c->k);
            mark(c, 1);
            hipLaunchKernelGGL((k_dif<A, VAR, BND>), grid, block, 0, c->stream, c->tmc, c->that_,
                               (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 2);
        } else {
            int ntile = ((c->k.nx + TX - 1) / TX) * ((c->k.ny + TY - 1) / TY) * ((c->k.nz + TZ - 1) / TZ) * 2;
            hipLaunchKernelGGL((k_tr<A, VAR>), dim3(ntile), block, 0, c->stream, c->that_, (const A *)c->aux,
                               (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 1);
        }
        c->cur = 1 - c->cur;
        c->steps++;
    }
    HIPCHECK(c, hipGetLastError());
    return PGK_OK;
}

template <typename S, typename A>
static int step_v(pgk_ctx *c, int64_t n)
{
    bool b = bounded(c);
    if (c->g.variant == PGK_CN)
        return b ? step_t<S, A, PGK_CN, true>(c, n) : step_t<S, A, PGK_CN, false>(c, n);
    return b ? step_t<S, A, PGK_LIT, true>(c, n) : step_t<S, A, PGK_LIT, false>(c, n);
}

extern "C" int pgk_step(pgk_ctx *c, int64_t n)
{
    if (!c || n < 0) return PGK_EINVAL;
    if (!c->initialised) return fail(c, PGK_EINVAL, "fields not initialised");
    if (n == 0) return PGK_OK;
    return c->g.precision == PGK_FP64 ? step_v<double, double>(c, n) : step_v<float, float>(c, n);
}

template <typename S, bool REDUCE>
static int moments_t(pgk_ctx *c, double *rho, double *u, double *thT, double *thR, double *P)
{
    dim3 grid(c->nblk), block(WG);
    const S *src = (const S *)c->buf[c->cur];
    // ghosts for the current pull: after a step they must be refreshed first
    if (bounded(c) && c->steps > 0) {
        int nbc = (2 * c->k.ny * c->k.nz + 63) / 64;
        hipLaunchKernelGGL((k_bc<S>), dim3(nbc), dim3(64), 0, c->stream, src, (S *)c->gh, c->k);
    }
    if (bounded(c))
        hipLaunchKernelGGL((k_moments<S, true, REDUCE>), grid, block, 0, c->stream, src, (const S *)c->gh,
                           (const double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, P, c->partial, c->k);
    else
        hipLaunchKernelGGL((k_moments<S, false, REDUCE>), grid, block, 0, c->stream, src, (const S *)c->gh,
                           (const double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, P, c->partial, c->k);
    HIPCHECK(c, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_read_moments(pgk_ctx *c, double *rho, double *u, double *thT, double *thR, double *P)
{
    if (!c) return PGK_EINVAL;
    if (!c->initialised) return fail(c, PGK_EINVAL, "fields not initialised");
    return c->g.precision == PGK_FP64 ? moments_t<double, false>(c, rho, u, thT, thR, P)
                                      : moments_t<float, false>(c, rho, u, thT, thR, P);
}

extern "C" int pgk_conserved(pgk_ctx *c, double out[5])
{
    if (!c || !out) return PGK_EINVAL;
    if (!c->initialised) return fail(c, PGK_EINVAL, "fields not initialised");
    int rc = c->g.precision == PGK_FP64 ? moments_t<double, true>(c, nullptr, nullptr, nullptr, nullptr, nullptr)
                                        : moments_t<float, true>(c, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(WG), 0, c->stream, c->partial, c->nblk, c->totals);
    HIPCHECK(c, hipGetLastError());
    HIPCHECK(c, hipMemcpyAsync(out, c->totals, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return PGK_OK;
}

extern "C" int pgk_set_timing(pgk_ctx *c, int enable)
{
    if (!c) return PGK_EINVAL;
    c->timing = enable != 0;
    c->nev = 0;
    return PGK_OK;
}

extern "C" int pgk_kernel_times(pgk_ctx *c, double ms[PGK_NKERNEL], int64_t launches[PGK_NKERNEL])
{
    if (!c || !ms || !launches) return PGK_EINVAL;
    for (int i = 0; i < PGK_NKERNEL; i++) { ms[i] = 0.0; launches[i] = 0; }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (size_t i = 1; i < c->nev; i++) {
        int id = c->marks[i];
        if (id < 0) continue;
        float t = 0.f;
        HIPCHECK(c, hipEventElapsedTime(&t, c->events[i - 1], c->events[i]));
        ms[id] += t;
        launches[id] += 1;
    }
    c->nev = 0;
    return PGK_OK;
}

extern "C" int64_t pgk_steps_done(const pgk_ctx *c) { return c ? c->steps : -1; }

extern "C" const char *pgk_last_error(const pgk_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" void pgk_destroy(pgk_ctx *c) { delete c; }
