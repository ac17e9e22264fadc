// device.hpp -- device code shared by the single-grid kernels (pgk.hip) and
// the batched kernel (batch.hip): constants, pull indexing, moments, the
// per-site solve, the F3 equilibrium and collide, theta_R transport stencils,
// boundary ghosts, initial state and moments.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

#include "pgk.h"
#include "lattice.hpp"
#include "e2.hpp"

namespace pgk {

constexpr int WG = 256;
constexpr int NSLOT = 4;  // ghost slots per x face: doubled x offsets 1..4 beyond the face
// which faces a grid has, a template level of the step kernels: none (every
// axis periodic), faces on x only, faces on x and y
constexpr int BND_NONE = 0, BND_X = 1, BND_XY = 2;

struct Consts {
    int nx, ny, nz, ns;
    int bc[4];              // kinds of the faces f = 2 axis + side: low x, high x, low y, high y
    double th0;
    double w[6];            // shell weights
    float whi[6], wlo[6];   // the same as float hi + lo parts (w = whi + wlo to ~1e-15)
    double tau, tau1, b, delta;
    double X, Y, ssig, beta, kfac;
    double thbc[4], rhobc[4];
    double Fbc[4][NQ];      // wall equilibrium at unit density / Dirichlet equilibrium
    double in_col[4];       // re-emitted mass per ghost column at unit wall density (uniform columns)
    // division by nx, ny, nz: q = (umulhi(n, m) + n) >> sh for n < 2^31
    unsigned mx, my, mz;
    int shx, shy, shz;
    // per-step constants computed once on the host
    double inv1X, inv1XY, inv3d;  // 1/(1+X), 1/(1+X+Y), 1/(3+delta)
    double wt1, wt, bs;           // tau1/(tau+tau1), tau/(tau+tau1), b/s_sigma
    double it, i2t, ih2, i6t3, i2t3, it2;  // 1/t, 1/(2t), 1/(2t^2), 1/(6t^3), 1/(2t^3), 1/t^2 with t = theta0
    int nsub;                     // FTCS sub-steps of the theta_R diffusion per step
    double isub;                  // 1/nsub
    double f4inv[36];             // F4: inverse of the lattice map K -> contracted fourth moment
};

// F4 coefficients K (xx yy zz xy xz yz) of the target (rho, u, lam): the
// contracted fourth moment of the Gaussian N(u, lam) less that of F3,
//   rho [tr E E + 2 E E - 2 u^2 u u],  E = u u + lam - theta0 I,
// mapped through the inverse lattice matrix (the correction's own moment).
__host__ __device__ __forceinline__ void f4_coeffs(const double *inv, double th0, double rho, const double *u,
                                                   const double *lam, double *K)
{
    double E[6] = {u[0] * u[0] + lam[0] - th0, u[1] * u[1] + lam[1] - th0, u[2] * u[2] + lam[2] - th0,
                   u[0] * u[1] + lam[3],       u[0] * u[2] + lam[4],       u[1] * u[2] + lam[5]};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double tr = E[0] + E[1] + E[2];
    double EE[6] = {E[0] * E[0] + E[3] * E[3] + E[4] * E[4], E[3] * E[3] + E[1] * E[1] + E[5] * E[5],
                    E[4] * E[4] + E[5] * E[5] + E[2] * E[2], E[0] * E[3] + E[3] * E[1] + E[4] * E[5],
                    E[0] * E[4] + E[3] * E[5] + E[4] * E[2], E[3] * E[4] + E[1] * E[5] + E[5] * E[2]};
    double uiuj[6] = {u[0] * u[0], u[1] * u[1], u[2] * u[2], u[0] * u[1], u[0] * u[2], u[1] * u[2]};
    double d[6];
    for (int i = 0; i < 6; i++) d[i] = rho * (tr * E[i] + 2.0 * EE[i] - 2.0 * uu * uiuj[i]);
    for (int i = 0; i < 6; i++) {
        double t = 0.0;
        for (int j = 0; j < 6; j++) t += inv[i * 6 + j] * d[j];
        K[i] = t;
    }
}

// Sub-steps that keep the explicit (FTCS) diffusion of theta_R stable: it
// needs 2 dim D_R dt <= dx^2, D_R = 2 kappa_R/(rho delta) = 5 k_r theta tau/(B delta),
// taken at 1.5 times the largest of theta0 and the face temperatures.  One
// sub-step is the printed scheme.
__host__ inline int diffusion_substeps(const Consts &k, double kr)
{
    int dim = (k.nx > 1) + (k.ny > 1) + (k.nz > 1);
    double th = k.th0;
    for (int f = 0; f < 4; f++)
        if (k.bc[f] != PGK_PERIODIC && k.thbc[f] > th) th = k.thbc[f];
    double B = 1.0 + k.tau / k.tau1;
    double DR = k.delta > 0 ? 5.0 * kr * th * k.tau / (B * k.delta) : 0.0;
    int n = (int)std::ceil(2.0 * dim * DR * 1.5);
    return n < 1 ? 1 : n;
}

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


// Ghosts: the values a pull reads from beyond a bounded face.  Face f of
// axis a = f/2 (x or y; z is periodic) keeps, for every population and each of
// NSLOT doubled distances beyond the face, one value per ghost column: the
// column is the cell coordinate along the other in-plane axis b and along z.
// Along a bounded axis b a column may lie outside the grid by up to two cells
// (the corners: a position beyond an x face and a y face at once belongs to
// the x face), so x faces have ny + 4 columns per z when y is bounded.
// Layout: x faces [2][NQ][NSLOT][nz][ghost_wy], then y faces [2][NQ][NSLOT][nz][nx].
__host__ __device__ __forceinline__ int ghost_wy(const Consts &k) { return k.bc[2] != PGK_PERIODIC ? k.ny + 4 : k.ny; }

__host__ __device__ __forceinline__ long long ghost_count(const Consts &k)
{
    long long n = 2LL * NQ * NSLOT * k.nz * ghost_wy(k);
    if (k.bc[2] != PGK_PERIODIC) n += 2LL * NQ * NSLOT * k.nz * k.nx;
    return n;
}

// index of ghost (face f, population q, slot, column col) in the ghost array
__host__ __device__ __forceinline__ int ghost_index(int f, int q, int slot, int col, const Consts &k)
{
    if (f < 2) return ((f * NQ + q) * NSLOT + slot) * k.nz * ghost_wy(k) + col;
    return 2 * NQ * NSLOT * k.nz * ghost_wy(k) + (((f - 2) * NQ + q) * NSLOT + slot) * k.nz * k.nx + col;
}

// Array index of the value of population q at doubled position (qx, qy, qz):
// a site of the population arrays (periodic axes wrap; `ghost` = 0), or on a
// bounded grid a ghost slot beyond face f (`ghost` = 1 + f).  BOUNDED is the
// grid's level: BND_NONE (every axis periodic), BND_X (faces on x only, y
// periodic) or BND_XY (faces on x and on y); the lower levels leave out the
// tests and index arithmetic of the faces they do not have.
template <int BOUNDED>
__device__ __forceinline__ int position_index(int qx, int qy, int qz, int q, const Consts &k, int &ghost)
{
    const int ssub = qx & 1;
    const int hx = (qx - ssub) >> 1, hy = (qy - ssub) >> 1, sz = wrapc((qz - ssub) >> 1, k.nz);
    ghost = 0;
    if (BOUNDED) {
        int f = -1, slot = 0;
        if (qx < 0 && k.bc[0] != PGK_PERIODIC) { f = 0; slot = -qx - 1; }
        else if (qx > 2 * k.nx - 1 && k.bc[1] != PGK_PERIODIC) { f = 1; slot = qx - 2 * k.nx; }
        else if (BOUNDED >= BND_XY && qy < 0 && k.bc[2] != PGK_PERIODIC) { f = 2; slot = -qy - 1; }
        else if (BOUNDED >= BND_XY && qy > 2 * k.ny - 1 && k.bc[3] != PGK_PERIODIC) { f = 3; slot = qy - 2 * k.ny; }
        if (f >= 0) {
            ghost = 1 + f;
            if (BOUNDED < BND_XY) {
                // x faces of a grid periodic in y: ny columns per z
                return ((f * NQ + q) * NSLOT + slot) * k.nz * k.ny + sz * k.ny + wrapc(hy, k.ny);
            }
            if (f < 2) {
                const int w = ghost_wy(k);
                const int iy = k.bc[2] != PGK_PERIODIC ? hy + 2 : wrapc(hy, k.ny);
                return ghost_index(f, q, slot, sz * w + iy, k);
            }
            return ghost_index(f, q, slot, sz * k.nx + wrapc(hx, k.nx), k);
        }
    }
    return ((ssub * k.nz + sz) * k.ny + wrapc(hy, k.ny)) * k.nx + wrapc(hx, k.nx);
}

// Ghost columns of the pull sources of one site on a grid with faces, the
// companion of PullMap: the column (coordinates along the face) of every
// source position for the x faces and (BND_XY) the y faces, for offsets -2..2
// and for the half velocities, and the doubled site coordinates that decide
// whether a source lies beyond a face.  The slot of a source beyond a face is
// linear in the doubled coordinate, so slot * (slot stride) splits into a
// per-site product (xsm, ysm) and a constant per population.
template <int BOUNDED>
struct GhostMap {
    int xs, ys;             // 2x + sub, 2y + sub
    int xsm, ysm;           // xs * nz * (x-face columns per z), ys * nz * nx
    int xcz;                // x-face columns per z: ny, or ny + 4 with y bounded
    Off5 XZ, XY;            // x-face column parts: wrapped z * xcz, y column
    int hxz[2], hxy[2];     // the same for half velocities: [0] c > 0, [1] c < 0
    Off5 YZ;                // y-face column part wrapped z * nx (the x part is PullMap.X)
    int hyz[2];
};

template <int BOUNDED>
__device__ __forceinline__ GhostMap<BOUNDED> ghost_map(int x, int y, int z, int sub, const Consts &k)
{
    GhostMap<BOUNDED> g;
    g.xs = 2 * x + sub;
    g.ys = 2 * y + sub;
    const bool yb = BOUNDED >= BND_XY && k.bc[2] != PGK_PERIODIC;
    g.xcz = yb ? k.ny + 4 : k.ny;
    g.xsm = g.xs * (k.nz * g.xcz);
    g.ysm = g.ys * (k.nz * k.nx);
    const int zz[5] = {wrap2(z - 2, k.nz), wrap2(z - 1, k.nz), z, wrap2(z + 1, k.nz), wrap2(z + 2, k.nz)};
    int yy[5];
    for (int d = 0; d < 5; d++) yy[d] = yb ? y + d : wrap2(y + d - 2, k.ny);   // iy = hy + 2 with y bounded
    g.XZ = {zz[0] * g.xcz, zz[1] * g.xcz, zz[2] * g.xcz, zz[3] * g.xcz, zz[4] * g.xcz};
    g.XY = {yy[0], yy[1], yy[2], yy[3], yy[4]};
    g.YZ = {zz[0] * k.nx, zz[1] * k.nx, zz[2] * k.nx, zz[3] * k.nx, zz[4] * k.nx};
    const bool b = sub != 0;
    g.hxz[0] = b ? g.XZ.z0 : g.XZ.m1; g.hxz[1] = b ? g.XZ.p1 : g.XZ.z0;
    g.hxy[0] = b ? g.XY.z0 : g.XY.m1; g.hxy[1] = b ? g.XY.p1 : g.XY.z0;
    g.hyz[0] = b ? g.YZ.z0 : g.YZ.m1; g.hyz[1] = b ? g.YZ.p1 : g.YZ.z0;
    return g;
}

// Index of the population Q pulled by a site inside a grid with faces: the
// index position_index gives for position x - c_Q, from the site's maps.  The
// sign of the compile-time c_Q decides which face the pull can cross (c_a > 0
// only the low face of axis a, c_a < 0 only the high one, c_a = 0 none);
// every candidate index is computed and one selected, so the kernels that pull
// on bounded grids run the same instructions on every lane, with no branch
// per population.  An x face wins a corner, as in position_index.
template <int Q, int BOUNDED>
__device__ __forceinline__ int pull_index_b(const PullMap &p, const GhostMap<BOUNDED> &g, const Consts &k,
                                            int &ghost)
{
    constexpr int cx = c2(Q, 0), cy = c2(Q, 1), cz = c2(Q, 2);
    constexpr bool half = (cx & 1) != 0;   // all three components odd
    int idx = (int)pull_off<Q>(p);
    ghost = 0;
    if constexpr (BOUNDED >= BND_XY && cy != 0) {
        constexpr int f = cy > 0 ? 2 : 3;
        // beyond the face: qy = ys - cy < 0, or qy > 2 ny - 1
        const bool gy = cy > 0 ? (g.ys < cy && k.bc[2] != PGK_PERIODIC)
                               : (g.ys - cy > 2 * k.ny - 1 && k.bc[3] != PGK_PERIODIC);
        int col;
        if constexpr (half) col = g.hyz[cz > 0 ? 0 : 1] + p.hx[cx > 0 ? 0 : 1];
        else col = g.YZ.template at<-cz / 2>() + p.X.template at<-cx / 2>();
        // slot = cy - 1 - ys (low face) or ys - cy - 2 ny (high face)
        const int base = 2 * NQ * NSLOT * k.nz * g.xcz + ((f - 2) * NQ + Q) * NSLOT * k.nz * k.nx;
        const int gi = cy > 0 ? base + (cy - 1) * k.nz * k.nx - g.ysm + col
                              : base - (cy + 2 * k.ny) * k.nz * k.nx + g.ysm + col;
        idx = gy ? gi : idx;
        ghost = gy ? 1 + f : ghost;
    }
    if constexpr (cx != 0) {
        constexpr int f = cx > 0 ? 0 : 1;
        const bool gx = cx > 0 ? (g.xs < cx && k.bc[0] != PGK_PERIODIC)
                               : (g.xs - cx > 2 * k.nx - 1 && k.bc[1] != PGK_PERIODIC);
        int col;
        if constexpr (half) col = g.hxz[cz > 0 ? 0 : 1] + g.hxy[cy > 0 ? 0 : 1];
        else col = g.XZ.template at<-cz / 2>() + g.XY.template at<-cy / 2>();
        const int base = (f * NQ + Q) * NSLOT * k.nz * g.xcz;
        const int gi = cx > 0 ? base + (cx - 1) * k.nz * g.xcz - g.xsm + col
                              : base - (cx + 2 * k.nx) * k.nz * g.xcz + g.xsm + col;
        idx = gx ? gi : idx;
        ghost = gx ? 1 + f : ghost;
    }
    return idx;
}

template <typename S, int BOUNDED, int Q = 0>
__device__ __forceinline__ void load_bounded(const S *__restrict__ src, const S *__restrict__ gh, const PullMap &p,
                                             const GhostMap<BOUNDED> &g, const Consts &k, S *v)
{
    if constexpr (Q < NQ) {
        int ghost;
        const int idx = pull_index_b<Q, BOUNDED>(p, g, k, ghost);
        const S *base = ghost ? gh : src + (size_t)Q * k.ns;
        v[Q] = base[idx];
        load_bounded<S, BOUNDED, Q + 1>(src, gh, p, g, k, v);
    }
}

// the 41 populations pulled by site (x, y, z, sub) of a grid with faces
template <typename S, int BOUNDED>
__device__ __forceinline__ void load_all(const S *__restrict__ src, const S *__restrict__ gh,
                                         int x, int y, int z, int sub, const Consts &k, S *v)
{
    static_assert(BOUNDED != BND_NONE, "periodic grids pull through load_periodic");
    load_bounded<S, BOUNDED>(src, gh, pull_map(x, y, z, sub, k), ghost_map<BOUNDED>(x, y, z, sub, k), k, v);
}

// The pull of one lane of a site pair (lane r = 0: the member +c of every
// opposite pair, r = 1: the member -c): v[0] the rest population, v[1 + P] the
// lane's member of pair P.  Both members' sources are computed and one
// selected, so the two lanes run the same instructions.
template <typename S, int BOUNDED, int P = 0>
__device__ __forceinline__ void load_lane(const S *__restrict__ src, const S *__restrict__ gh, const PullMap &p,
                                          const GhostMap<BOUNDED> &g, const Consts &k, int r, S *v)
{
    if constexpr (P == 0) v[0] = src[pull_off<0>(p)];   // c = 0 never crosses a face
    if constexpr (P < NPAIR) {
        constexpr int QP = 1 + P, QM = 1 + NPAIR + P;
        const S *base;
        size_t idx;
        if constexpr (BOUNDED) {
            int gp, gm;
            const int ip = pull_index_b<QP, BOUNDED>(p, g, k, gp), im = pull_index_b<QM, BOUNDED>(p, g, k, gm);
            const int ghost = r ? gm : gp;
            base = ghost ? gh : src + (size_t)(r ? QM : QP) * k.ns;
            idx = (size_t)(r ? im : ip);
        } else {
            base = src + (size_t)(r ? QM : QP) * k.ns;
            idx = r ? pull_off<QM>(p) : pull_off<QP>(p);
        }
        v[1 + P] = base[idx];
        load_lane<S, BOUNDED, P + 1>(src, gh, p, g, k, r, v);
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

// value held by the other lane of a site pair (lane ^ 1), by a DPP quad
// permutation [1, 0, 3, 2]; both lanes of the pair must be active
__device__ __forceinline__ double pair_swap(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0xB1, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Moments of a site pulled by a lane pair (load_lane): each lane receives the
// partner's members by DPP and sums all 41 values as moments() does, so both
// lanes hold the same bits as a lane that pulled the whole site.
template <typename S>
__device__ __forceinline__ S pair_swap_s(S v)
{
    if constexpr (sizeof(S) == 8) {
        return pair_swap(v);
    } else {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    }
}

template <typename S>
__device__ __forceinline__ Mom moments_pair(const S *v, const Consts &k, int r)
{
    S w[NQ];
    w[0] = v[0];
#pragma unroll
    for (int P = 0; P < NPAIR; P++) {
        const S o = pair_swap_s(v[1 + P]);
        w[1 + P] = r ? o : v[1 + P];
        w[1 + NPAIR + P] = r ? v[1 + P] : o;
    }
    return moments<S>(w, k);
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
    // F4 only: correction w [cKc (c^2 - 7 theta0) - q1 c^2 + q0]
    R K0, K1, K2, K3, K4, K5;
    R t7, q1, q0;       // 7 theta0, theta0 tr K, 5 theta0^2 tr K
};

template <typename R>
__device__ __forceinline__ void set_f4(Eq<R> &e, const double *K, const Consts &k)
{
    double trK = K[0] + K[1] + K[2];
    e.K0 = (R)K[0]; e.K1 = (R)K[1]; e.K2 = (R)K[2]; e.K3 = (R)K[3]; e.K4 = (R)K[4]; e.K5 = (R)K[5];
    e.t7 = (R)(7.0 * k.th0);
    e.q1 = (R)(k.th0 * trK);
    e.q0 = (R)(5.0 * k.th0 * k.th0 * trK);
}

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
// F4: the even correction of the contracted fourth-order terms is added.
template <typename S, bool F4 = false, int P = 0>
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
        S corr = (S)0;
        if constexpr (F4) {
            constexpr S cc = hx * hx + hy * hy + hz * hz;
            S cKc = hx * hx * e.K0 + hy * hy * e.K1 + hz * hz * e.K2
                  + (S)2 * (hx * hy * e.K3 + hx * hz * e.K4 + hy * hz * e.K5);
            corr = cKc * (cc - e.t7) - e.q1 * cc + e.q0;
        }
        if constexpr (sizeof(S) == 4) {
            // deviation form: F - w = w [(rho - 1) + rho (even +- odd)], with w
            // carried as hi + lo floats so the rounding of w adds no bias to the
            // moments of F; h* = h + 2 beta (F - w - h) conserves the moments of
            // the collision whatever the rounding of 2 beta
            S wh = k.whi[Lattice::SHELL[P]], wl = k.wlo[Lattice::SHELL[P]];
            S Xp = e.drho + e.rho * (even + odd), Xm = e.drho + e.rho * (even - odd);
            if constexpr (F4) {
                Xp += corr;
                Xm += corr;
            }
            S Fp = wh * Xp + wl * Xp, Fm = wh * Xm + wl * Xm;
            // the next read of these values is a step away: stream them past the caches
            __builtin_nontemporal_store(v[1 + P] + e.tb * (Fp - v[1 + P]), &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(v[1 + NPAIR + P] + e.tb * (Fm - v[1 + NPAIR + P]),
                                        &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        } else {
            S w = (S)k.w[Lattice::SHELL[P]];
            S Fp, Fm;
            if constexpr (F4) {
                Fp = w * (e.rho * ((S)1 + even + odd) + corr);
                Fm = w * (e.rho * ((S)1 + even - odd) + corr);
            } else {
                Fp = w * e.rho * ((S)1 + even + odd);
                Fm = w * e.rho * ((S)1 + even - odd);
            }
            __builtin_nontemporal_store(e.omb * v[1 + P] + e.tb * Fp, &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(e.omb * v[1 + NPAIR + P] + e.tb * Fm, &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        }
        collide_store<S, F4, P + 1>(v, e, k, dst, s);
    } else {
        if constexpr (sizeof(S) == 4) {
            S X0 = e.drho - e.rho * e.k0;
            if constexpr (F4) X0 += e.q0;
            S F0 = k.whi[0] * X0 + k.wlo[0] * X0;
            __builtin_nontemporal_store(v[0] + e.tb * (F0 - v[0]), &dst[s]);
        } else {
            S w0 = (S)k.w[0];
            S F0;
            if constexpr (F4) F0 = w0 * (e.rho * ((S)1 - e.k0) + e.q0);
            else F0 = w0 * e.rho * ((S)1 - e.k0);
            __builtin_nontemporal_store(e.omb * v[0] + e.tb * F0, &dst[s]);
        }
    }
}

// Collide toward the gain term of the E2 form and write the own site.  The
// gain term is the rate-weighted mixture of the two targets, F =
// wt1 F(lam_ES) + wt F(theta I) with wt1 = tau1/(tau+tau1), wt = tau/(tau+tau1)
// (Sec. 4): for an equilibrium that is not linear in the covariance the two
// terms do not merge into one.  p1, p2: the exponential factors (e2_pow_bases)
// of the multipliers of the two E2 targets, in double; FP32 deviation storage
// takes F - w = w (wt1 (F1/w - 1) + wt (F2/w - 1)), each F/w - 1 as one fused
// multiply-add.
template <typename S, int P = 0>
__device__ __forceinline__ void collide_e2_pairs(S *v, const E2Pow &p1, const E2Pow &p2, const Consts &k,
                                                 S *__restrict__ dst, int s)
{
    if constexpr (P < NPAIR) {
        double e1, x1p, x1m, e2, x2p, x2m;
        e2_pair_exp<P>(p1, e1, x1p, x1m);
        e2_pair_exp<P>(p2, e2, x2p, x2m);
        double w = k.w[Lattice::SHELL[P]];
        if constexpr (sizeof(S) == 4) {
            S tb = (S)(2.0 * k.beta);
            S Fp = (S)(w * (k.wt1 * fma(e1, x1p, -1.0) + k.wt * fma(e2, x2p, -1.0)));
            S Fm = (S)(w * (k.wt1 * fma(e1, x1m, -1.0) + k.wt * fma(e2, x2m, -1.0)));
            __builtin_nontemporal_store(v[1 + P] + tb * (Fp - v[1 + P]), &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(v[1 + NPAIR + P] + tb * (Fm - v[1 + NPAIR + P]),
                                        &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        } else {
            double omb = 1.0 - 2.0 * k.beta, tb = 2.0 * k.beta;
            double Fp = w * (k.wt1 * (e1 * x1p) + k.wt * (e2 * x2p));
            double Fm = w * (k.wt1 * (e1 * x1m) + k.wt * (e2 * x2m));
            __builtin_nontemporal_store(omb * v[1 + P] + tb * Fp, &dst[(size_t)(1 + P) * k.ns + s]);
            __builtin_nontemporal_store(omb * v[1 + NPAIR + P] + tb * Fm, &dst[(size_t)(1 + NPAIR + P) * k.ns + s]);
        }
        collide_e2_pairs<S, P + 1>(v, p1, p2, k, dst, s);
    } else {
        double w0 = k.w[0];
        if constexpr (sizeof(S) == 4) {
            S tb = (S)(2.0 * k.beta);
            S F0 = (S)(w0 * (k.wt1 * (p1.e0 - 1.0) + k.wt * (p2.e0 - 1.0)));
            __builtin_nontemporal_store(v[0] + tb * (F0 - v[0]), &dst[s]);
        } else {
            double F0 = w0 * (k.wt1 * p1.e0 + k.wt * p2.e0);
            __builtin_nontemporal_store((1.0 - 2.0 * k.beta) * v[0] + 2.0 * k.beta * F0, &dst[s]);
        }
    }
}

template <typename S>
__device__ __forceinline__ void collide_store_e2(S *v, const double *l1, const double *l2, const Consts &k,
                                                 S *__restrict__ dst, int s)
{
    E2Pow p1, p2;
    e2_pow_bases(l1, p1);
    e2_pow_bases(l2, p2);
    collide_e2_pairs<S>(v, p1, p2, k, dst, s);
}

// The same collide spread over the two lanes of a site pair.  Lane r holds the
// powers pw of its own final multipliers (r = 0: the lam_ES target, r = 1:
// theta I) and stores the member +c (r = 0) or -c (r = 1) of every opposite
// pair, lane 0 also the rest velocity.  Each lane forms the exponential of its
// multipliers at both members and hands the partner the one the partner stores,
// so each exponential is formed once, by the same instructions as in
// collide_store_e2, and every population is the same bits.
template <typename S, int P = 0>
__device__ __forceinline__ void collide_e2_lane_pairs(const S *v, const E2Pow &pw, const Consts &k,
                                                      S *__restrict__ dst, int s, int r)
{
    if constexpr (P < NPAIR) {
        double e, xp, xm;
        e2_pair_exp<P>(pw, e, xp, xm);
        const double xo = r ? xm : xp, xg = r ? xp : xm;   // the own member, the partner's
        double w = k.w[Lattice::SHELL[P]];
        const size_t q = r ? 1 + NPAIR + P : 1 + P;
        const S vq = v[1 + P];   // the lane's member (load_lane)
        if constexpr (sizeof(S) == 4) {
            const double own = fma(e, xo, -1.0), got = pair_swap(fma(e, xg, -1.0));
            const double t1 = r ? got : own, t2 = r ? own : got;   // ES term, theta I term
            S tb = (S)(2.0 * k.beta);
            S F = (S)(w * (k.wt1 * t1 + k.wt * t2));
            __builtin_nontemporal_store(vq + tb * (F - vq), &dst[q * k.ns + s]);
        } else {
            const double own = e * xo, got = pair_swap(e * xg);
            const double t1 = r ? got : own, t2 = r ? own : got;
            double omb = 1.0 - 2.0 * k.beta, tb = 2.0 * k.beta;
            double F = w * (k.wt1 * t1 + k.wt * t2);
            __builtin_nontemporal_store(omb * vq + tb * F, &dst[q * k.ns + s]);
        }
        collide_e2_lane_pairs<S, P + 1>(v, pw, k, dst, s, r);
    } else {
        const double e2o = pair_swap(pw.e0);   // lane 0 receives theta I's exp(l0)
        if (r == 0) {
            double w0 = k.w[0];
            if constexpr (sizeof(S) == 4) {
                S tb = (S)(2.0 * k.beta);
                S F0 = (S)(w0 * (k.wt1 * (pw.e0 - 1.0) + k.wt * (e2o - 1.0)));
                __builtin_nontemporal_store(v[0] + tb * (F0 - v[0]), &dst[s]);
            } else {
                double F0 = w0 * (k.wt1 * pw.e0 + k.wt * e2o);
                __builtin_nontemporal_store((1.0 - 2.0 * k.beta) * v[0] + 2.0 * k.beta * F0, &dst[s]);
            }
        }
    }
}

// E2 multipliers of density rho, velocity u, covariance lam; a target out of
// the lattice's reach gives NaN multipliers, so the site's populations turn
// NaN (never silently replaced by another equilibrium)
__device__ __forceinline__ void e2_site(double rho, const double *u, const double *lam, const Consts &k, double *l)
{
    if (e2_solve(k.th0, k.w, rho, u, lam, l) < 0)
        for (int i = 0; i < E2_NL; i++) l[i] = __builtin_nan("");
}

// the same, Newton started from the multipliers in l when they are finite
__device__ __forceinline__ void e2_site_from(double rho, const double *u, const double *lam, const Consts &k,
                                             double *l)
{
    if (e2_solve_from(k.th0, k.w, rho, u, lam, l) < 0)
        for (int i = 0; i < E2_NL; i++) l[i] = __builtin_nan("");
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
// per-site bodies shared by the single-grid kernels and the batched kernel
// ---------------------------------------------------------------------------
// fused pull - moments - solve - equilibrium - collide of site s; returns the
// moments of g (time level n) and the stored theta_R in r_out
// lmul (E2 only, may be null): per-site store [2 E2_NL][ns] of the two
// multiplier sets of the last step; each Newton run starts from them
template <typename S, typename A, int VAR, int BOUNDED, int EQ = PGK_F3>
__device__ __forceinline__ Mom lb_site(int s, const S *__restrict__ src, S *__restrict__ dst,
                                       const S *__restrict__ gh, double *__restrict__ thR,
                                       double *__restrict__ that_, A *__restrict__ aux, const Consts &k,
                                       double &r_out, double *__restrict__ lmul = nullptr)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    S v[NQ];
    if constexpr (BOUNDED) load_all<S, BOUNDED>(src, gh, x, y, z, sub, k, v);
    else load_periodic<S>(src, pull_map(x, y, z, sub, k), k.ns, v);
    double r = thR[s];
    Mom m = moments<S>(v, k);
    Solve so = site_solve(m, r, k);
    if constexpr (EQ == PGK_E2) {
        // the two targets: lam_ES = T I + b sigma(f)/rho and theta I
        double les[6], lmb[6], l1[E2_NL], l2[E2_NL];
        double cb = k.bs / so.rho;
        for (int i = 0; i < 6; i++) {
            les[i] = (i < 3 ? so.T : 0.0) + cb * so.sg[i];
            lmb[i] = i < 3 ? so.theta : 0.0;
        }
        if (lmul) {
            for (int i = 0; i < E2_NL; i++) {
                l1[i] = lmul[(size_t)i * k.ns + s];
                l2[i] = lmul[(size_t)(E2_NL + i) * k.ns + s];
            }
            e2_site_from(so.rho, so.u, les, k, l1);
            e2_site_from(so.rho, so.u, lmb, k, l2);
            for (int i = 0; i < E2_NL; i++) {
                lmul[(size_t)i * k.ns + s] = l1[i];
                lmul[(size_t)(E2_NL + i) * k.ns + s] = l2[i];
            }
        } else {
            e2_site(so.rho, so.u, les, k, l1);
            e2_site(so.rho, so.u, lmb, k, l2);
        }
        collide_store_e2<S>(v, l1, l2, k, dst, s);
    } else if constexpr (EQ == PGK_F4) {
        // the F3 part is linear in the covariance (lam_F); the fourth-order
        // coefficients mix those of the two targets at their rates
        double les[6], lmb[6], K1[6], K2[6], K[6];
        double cb = k.bs / so.rho;
        for (int i = 0; i < 6; i++) {
            les[i] = (i < 3 ? so.T : 0.0) + cb * so.sg[i];
            lmb[i] = i < 3 ? so.theta : 0.0;
        }
        f4_coeffs(k.f4inv, k.th0, so.rho, so.u, les, K1);
        f4_coeffs(k.f4inv, k.th0, so.rho, so.u, lmb, K2);
        for (int i = 0; i < 6; i++) K[i] = k.wt1 * K1[i] + k.wt * K2[i];
        Eq<S> e = make_eq<S>(so, k);
        set_f4(e, K, k);
        collide_store<S, true>(v, e, k, dst, s);
    } else {
        Eq<S> e = make_eq<S>(so, k);
        collide_store<S>(v, e, k, dst, s);
    }
    that_[s] = so.R;                                  // theta_R after step 1
    if (VAR == PGK_LIT) thR[s] = so.T;                // the printed second half needs theta_T
    aux[s] = (A)so.u[0];
    aux[(size_t)k.ns + s] = (A)so.u[1];
    aux[(size_t)2 * k.ns + s] = (A)so.u[2];
    aux[(size_t)3 * k.ns + s] = (A)so.rho;
    aux[(size_t)4 * k.ns + s] = (A)(so.rho * so.theta);
    r_out = r;
    return m;
}

// E2 with the two Newton solves of site s on a pair of adjacent lanes (r = 0:
// the lam_ES target, r = 1: theta I).  Each lane pulls the rest population
// and one member of every opposite pair (the one it later stores), receives
// the other members from its partner, and both lanes solve the site's
// temperatures; each runs one Newton solve from its multipliers of the last
// step (lmul, [2 E2_NL][ns], never null here); the pair collides with each
// lane storing its members (the exponentials of each solve formed by its own
// lane and passed across), and lane 0 hands the fields to the transport.
// The arithmetic per site is that of lb_site<..., PGK_E2>.
template <typename S, typename A, int VAR, int BOUNDED>
__device__ __forceinline__ void lb_site_e2pair(int s, int r, const S *__restrict__ src, S *__restrict__ dst,
                                               const S *__restrict__ gh, double *__restrict__ thR,
                                               double *__restrict__ that_, A *__restrict__ aux, const Consts &k,
                                               double *__restrict__ lmul)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    S v[1 + NPAIR];   // the rest population and the lane's member of every pair
    if constexpr (BOUNDED)
        load_lane<S, BOUNDED>(src, gh, pull_map(x, y, z, sub, k), ghost_map<BOUNDED>(x, y, z, sub, k), k, r, v);
    else
        load_lane<S, BOUNDED>(src, gh, pull_map(x, y, z, sub, k), GhostMap<BOUNDED>{}, k, r, v);
    Mom m = moments_pair<S>(v, k, r);
    Solve so = site_solve(m, thR[s], k);
    double lam[6], l[E2_NL];
    double cb = k.bs / so.rho;
    for (int i = 0; i < 6; i++)
        lam[i] = r == 0 ? (i < 3 ? so.T : 0.0) + cb * so.sg[i] : (i < 3 ? so.theta : 0.0);
    double *lm = lmul + (size_t)r * E2_NL * k.ns + s;
    for (int i = 0; i < E2_NL; i++) l[i] = lm[(size_t)i * k.ns];
    e2_site_from(so.rho, so.u, lam, k, l);
    for (int i = 0; i < E2_NL; i++) lm[(size_t)i * k.ns] = l[i];
    E2Pow pw;
    e2_pow_bases(l, pw);
    collide_e2_lane_pairs<S>(v, pw, k, dst, s, r);
    if (r != 0) return;
    that_[s] = so.R;
    if (VAR == PGK_LIT) thR[s] = so.T;
    aux[s] = (A)so.u[0];
    aux[(size_t)k.ns + s] = (A)so.u[1];
    aux[(size_t)2 * k.ns + s] = (A)so.u[2];
    aux[(size_t)3 * k.ns + s] = (A)so.rho;
    aux[(size_t)4 * k.ns + s] = (A)(so.rho * so.theta);
}

// ---------------------------------------------------------------------------
// theta_R transport
// ---------------------------------------------------------------------------
// same-sublattice neighbour along axis a (0,1,2) by dir (+-1); across a bounded
// face f it returns -1 - f (-1 / -2: low / high x, -3 / -4: low / high y)
template <int BOUNDED>
__device__ __forceinline__ int nbr(int x, int y, int z, int sub, int a, int dir, const Consts &k)
{
    if (a == 0) {
        x += dir;
        if (BOUNDED) {
            if (x < 0 && k.bc[0] != PGK_PERIODIC) return -1;
            if (x >= k.nx && k.bc[1] != PGK_PERIODIC) return -2;
        }
        x = wrapc(x, k.nx);
    } else if (a == 1) {
        y += dir;
        if (BOUNDED >= BND_XY) {
            if (y < 0 && k.bc[2] != PGK_PERIODIC) return -3;
            if (y >= k.ny && k.bc[3] != PGK_PERIODIC) return -4;
        }
        y = wrapc(y, k.ny);
    } else {
        z = wrapc(z + dir, k.nz);
    }
    return ((sub * k.nz + z) * k.ny + y) * k.nx + x;
}

template <typename A, int BOUNDED>
__device__ __forceinline__ double theta_star(const double *__restrict__ th, const A *__restrict__ aux,
                                             int idx, const Consts &k)
{
    // predictor at site idx (forward differences); ghosts keep their value
    if (BOUNDED && idx < 0) return k.thbc[-1 - idx];
    int x, y, z, sub;
    decode(idx, k, x, y, z, sub);
    double t = th[idx], adv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        int p = nbr<BOUNDED>(x, y, z, sub, a, +1, k);
        double tp = (BOUNDED && p < 0) ? k.thbc[-1 - p] : th[p];
        adv += (double)aux[(size_t)a * k.ns + idx] * (tp - t);
    }
    return t - adv;
}

template <typename A, int BOUNDED>
__device__ __forceinline__ void mc_site(int s, const double *__restrict__ that_, const A *__restrict__ aux,
                                        double *__restrict__ tmc, const Consts &k)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    double ts = theta_star<A, BOUNDED>(that_, aux, s, k);
    double adv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        int m = nbr<BOUNDED>(x, y, z, sub, a, -1, k);
        double tm = theta_star<A, BOUNDED>(that_, aux, m, k);
        adv += (double)aux[(size_t)a * k.ns + s] * (ts - tm);
    }
    tmc[s] = 0.5 * (that_[s] + ts - adv);
}

// one FTCS sub-step of the theta_R diffusion from tin; the last sub-step
// (FINAL) also applies the second half of the relaxation and writes theta_R
template <typename A, int VAR, int BOUNDED, bool FINAL>
__device__ __forceinline__ void dif_site(int s, const double *__restrict__ tin, double *__restrict__ tout,
                                         const double *__restrict__ that_, const A *__restrict__ aux,
                                         double *__restrict__ thR, const Consts &k)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    double rho = (double)aux[(size_t)3 * k.ns + s];
    double ks = k.kfac * (double)aux[(size_t)4 * k.ns + s];
    double t = tin[s];
    double flux = 0.0, lap = 0.0;
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int dir = -1; dir <= 1; dir += 2) {
            int q = nbr<BOUNDED>(x, y, z, sub, a, dir, k);
            double tq, kq;
            if (BOUNDED && q < 0) {
                const int f = -1 - q;
                tq = k.thbc[f];
                double rg = k.bc[f] == PGK_WALL ? rho : k.rhobc[f];
                kq = k.kfac * rg * tq;
            } else {
                tq = tin[q];
                kq = k.kfac * (double)aux[(size_t)4 * k.ns + q];
            }
            flux += 0.5 * (ks + kq) * (tq - t);
            lap += tq - t;
        }
    double tdif = VAR == PGK_CN ? t + k.isub * 2.0 * flux / (rho * k.delta)
                                : t + k.isub * 2.0 * ks / (rho * k.delta) * lap;
    if constexpr (!FINAL) {
        tout[s] = tdif;
    } else {
        double v = thR[s];
        if (VAR == PGK_CN) thR[s] = tdif + (that_[s] - v);   // second half: repeat R - r
        else thR[s] = (tdif + k.X * v) * k.inv1X;            // backward Euler, as printed
    }
}

__host__ __device__ __forceinline__ int floor2(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

// Number of ghost columns of face f (see ghost_wy).
__host__ __device__ __forceinline__ int face_columns(int f, const Consts &k)
{
    return f < 2 ? k.nz * ghost_wy(k) : k.nz * k.nx;
}

// Ghost populations of face f, column col, by one wavefront (lane 0..63).
// Diffuse wall: the density of the re-emitted populations comes from zero net
// mass flux through the column in the last collision: the mass sent into the
// column (the outgoing sum, spread over the lanes: lane l takes the
// candidates (q, sub, distance) numbered l, l + 64, l + 128) over the mass the
// wall re-emits into it at unit density (the same candidates pulling from it;
// uniform on a face whose other in-plane axis is periodic, k.in_col[f]),
// reduced by a butterfly.  Dirichlet: the equilibrium of the ghost state.
// Lanes 0..40 write population q = lane into every slot.
template <typename S>
__device__ __forceinline__ void bc_column(int f, int col, int lane, const S *__restrict__ src,
                                          S *__restrict__ gh, const Consts &k)
{
    if (k.bc[f] == PGK_PERIODIC) return;
    const int a = f >> 1, side = f & 1, b = 1 - a;           // face axis, the other in-plane axis
    const int na = a == 0 ? k.nx : k.ny, nb = b == 0 ? k.nx : k.ny;
    const bool bb = k.bc[2 * b] != PGK_PERIODIC;              // axis b bounded
    const bool xb = k.bc[0] != PGK_PERIODIC;
    const int width = f < 2 ? ghost_wy(k) : k.nx;
    const int gz = col / width, ib = col - gz * width;
    const int gb = (f < 2 && bb) ? ib - 2 : ib;               // cell coordinate of the column along b
    double scale = 1.0;
    if (k.bc[f] == PGK_WALL) {
        double out = 0.0, in = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            int idx = lane + 64 * j;                 // 160 candidates: q = 1..40, sub, distance di
            if (idx >= 4 * (NQ - 1)) break;
            int q = 1 + (idx >> 2), sub = (idx >> 1) & 1, di = idx & 1;
            if (di == 1 && na == 1) continue;
            const int ca = c2(q, a), cb = c2(q, b), cz = c2(q, 2);
            const int sa = side == 0 ? di : na - 1 - di;      // site coordinate along a
            // outgoing: population q of a site near the face lands beyond it, in column gb
            if ((side == 0 && ca < 0) || (side == 1 && ca > 0)) {
                int da = 2 * sa + sub + ca;
                bool crosses = side == 0 ? da < 0 : da > 2 * na - 1;
                int sb = gb - floor2(sub + cb);
                int db = 2 * sb + sub + cb;
                bool ok = crosses && (bb ? (sb >= 0 && sb < nb) : true);
                // a y face never takes what lands beyond a bounded x face
                if (ok && f >= 2 && xb && (db < 0 || db > 2 * k.nx - 1)) ok = false;
                if (ok) {
                    int z = k.nz == 1 ? 0 : wrapc(gz - floor2(sub + cz), k.nz);
                    int sbw = bb ? sb : wrapc(sb, nb);
                    int x = a == 0 ? sa : sbw, y = a == 0 ? sbw : sa;
                    int s = ((sub * k.nz + z) * k.ny + y) * k.nx + x;
                    out += (double)src[(size_t)q * k.ns + s] + (sizeof(S) == 4 ? k.w[shell_of(q)] : 0.0);
                }
            }
            // incoming: a site near the face pulls population q from column gb
            // (along a periodic b every column takes the same: k.in_col[f])
            if (bb && ((side == 0 && ca > 0) || (side == 1 && ca < 0))) {
                int pa = 2 * sa + sub - ca;
                bool crosses = side == 0 ? pa < 0 : pa > 2 * na - 1;
                int sb = gb - floor2(sub - cb);
                int pb = 2 * sb + sub - cb;
                bool ok = crosses && (bb ? (sb >= 0 && sb < nb) : true);
                if (ok && f >= 2 && xb && (pb < 0 || pb > 2 * k.nx - 1)) ok = false;
                if (ok) in += k.Fbc[f][q];
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) out += __shfl_xor(out, o, 64);
        if (bb) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) in += __shfl_xor(in, o, 64);
        }
        double inc = bb ? in : k.in_col[f];
        scale = inc > 0.0 ? out / inc : 0.0;
    }
    if (lane < NQ) {
        double val = scale * k.Fbc[f][lane] - (sizeof(S) == 4 ? k.w[shell_of(lane)] : 0.0);
#pragma unroll
        for (int slot = 0; slot < NSLOT; slot++) gh[ghost_index(f, lane, slot, col, k)] = (S)val;
    }
}

// push F_i(rho, u, theta_T I) of site s to where the next pull reads it:
// population i of site x is read from position x - c_i (a ghost slot when that
// lies beyond a bounded face)
template <typename S, int BOUNDED, int EQ = PGK_F3>
__device__ __forceinline__ void init_site(int s, S *__restrict__ dst, S *__restrict__ gh, double *__restrict__ thR,
                                          const double *__restrict__ rho, const double *__restrict__ u,
                                          const double *__restrict__ thT, const double *__restrict__ thRin,
                                          const Consts &k, size_t ustride)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    Solve so;
    so.rho = rho[s];
    so.u[0] = u[s];
    so.u[1] = u[ustride + s];
    so.u[2] = u[2 * ustride + s];
    for (int i = 0; i < 6; i++) so.lamF[i] = i < 3 ? thT[s] : 0.0;
    Eq<double> e = make_eq<double>(so, k);
    double l[E2_NL], K[6] = {0, 0, 0, 0, 0, 0};
    if constexpr (EQ == PGK_E2) e2_site(so.rho, so.u, so.lamF, k, l);
    if constexpr (EQ == PGK_F4) f4_coeffs(k.f4inv, k.th0, so.rho, so.u, so.lamF, K);
    double trK = K[0] + K[1] + K[2];
    thR[s] = thRin[s];
    for (int q = 0; q < NQ; q++) {
        int cx = c2(q, 0), cy = c2(q, 1), cz = c2(q, 2);
        double hx = 0.5 * cx, hy = 0.5 * cy, hz = 0.5 * cz;
        double w = k.w[shell_of(q)];
        S val;
        if constexpr (EQ == PGK_E2) {
            double ex = l[0] + hx * l[1] + hy * l[2] + hz * l[3] + hx * hx * l[4] + hy * hy * l[5] + hz * hz * l[6] +
                        hx * hy * l[7] + hx * hz * l[8] + hy * hz * l[9];
            val = (S)(sizeof(S) == 4 ? w * expm1(ex) : w * exp(ex));
        } else {
            double cu = hx * e.u0 + hy * e.u1 + hz * e.u2;
            double cDc = hx * hx * e.D0 + hy * hy * e.D1 + hz * hz * e.D2 + 2.0 * (hx * hy * e.D3 + hx * hz * e.D4 + hy * hz * e.D5);
            double cDu = hx * e.Du0 + hy * e.Du1 + hz * e.Du2;
            double even = (cu * cu + cDc) * e.k2 - e.k0;
            double odd = cu * e.A1 + cu * cu * cu * e.k3 + cDc * cu * e.k4 - cDu * e.k5;
            double corr = 0.0;
            if constexpr (EQ == PGK_F4) {
                double cc = hx * hx + hy * hy + hz * hz;
                double cKc = hx * hx * K[0] + hy * hy * K[1] + hz * hz * K[2] +
                             2.0 * (hx * hy * K[3] + hx * hz * K[4] + hy * hz * K[5]);
                corr = cKc * (cc - 7.0 * k.th0) - k.th0 * trK * (cc - 5.0 * k.th0);
            }
            double F, X;
            if constexpr (EQ == PGK_F4) {
                F = w * (e.rho * (1.0 + even + odd) + corr);
                X = w * (e.drho + e.rho * (even + odd) + corr);
            } else {
                F = w * e.rho * (1.0 + even + odd);
                X = w * (e.drho + e.rho * (even + odd));
            }
            val = (S)(sizeof(S) == 4 ? X : F);
        }
        // destination: position x - c_q (a ghost slot beyond a bounded face)
        int ghost;
        int idx = position_index<BOUNDED>(2 * x + sub - cx, 2 * y + sub - cy, 2 * z + sub - cz, q, k, ghost);
        if (BOUNDED && ghost) gh[idx] = val;
        else dst[(size_t)q * k.ns + idx] = val;
    }
}

// f-moments of site s at the current time level (after the g -> f map)
template <typename S, int BOUNDED>
__device__ __forceinline__ Solve moments_site(int s, const S *__restrict__ src, const S *__restrict__ gh,
                                              const double *__restrict__ thR, const Consts &k, Mom &m)
{
    int x, y, z, sub;
    decode(s, k, x, y, z, sub);
    S v[NQ];
    if constexpr (BOUNDED) load_all<S, BOUNDED>(src, gh, x, y, z, sub, k, v);
    else load_periodic<S>(src, pull_map(x, y, z, sub, k), k.ns, v);
    m = moments<S>(v, k);
    return site_solve(m, thR[s], k);
}

// F3 on the host for boundary equilibria: rho, u, isotropic temperature theta
static inline void f3_host(double th0, const double w6[6], double rho, const double u[3], double theta, double F[NQ])
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

// magic numbers for q = (umulhi(n, m) + n) >> sh = n / d, valid for n < 2^31
static inline void magic_div(unsigned d, unsigned &m, int &sh)
{
    int s = 0;
    while ((1ull << s) < d) s++;
    m = (unsigned)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
    sh = s;
}

}  // namespace pgk
