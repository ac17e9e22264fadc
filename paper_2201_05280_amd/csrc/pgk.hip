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

#include <type_traits>
#include <utility>

#include "device.hpp"

namespace pgk {

// ---------------------------------------------------------------------------
// single-grid kernels: one thread per site
// ---------------------------------------------------------------------------
// Work-group size of the fused kernel: 1024 for FP32 storage, where against
// 256 a step of the 256^3 benchmark grid takes 1.5% less (fewer, longer-lived
// groups) and the kernel fits the 128 registers this allows without spilling;
// 256 for FP64 storage and for F4 with faces, which would spill at 128.
template <typename S, int BOUNDED, int EQ>
constexpr int lb_wg() { return sizeof(S) == 4 && (EQ == PGK_F3 || !BOUNDED) ? 1024 : WG; }

template <typename S, typename A, int VAR, int BOUNDED, int EQ, int NT>
__global__ __launch_bounds__(NT) void k_lb(const S *__restrict__ src, S *__restrict__ dst, const S *__restrict__ gh,
                                           double *__restrict__ thR, double *__restrict__ that_, A *__restrict__ aux,
                                           double *__restrict__ lmul, Consts k)
{
    int s = blockIdx.x * NT + threadIdx.x;
    if (s < k.ns) {
        double r;
        lb_site<S, A, VAR, BOUNDED, EQ>(s, src, dst, gh, thR, that_, aux, k, r, lmul);
    }
}

// E2 grids: two lanes per site, one Newton solve each (lb_site_e2pair), in
// work-groups of one wavefront: the kernel holds 256 registers per lane, so a
// SIMD runs one of its wavefronts at a time whatever the group size, and
// groups of 64 spread a short line's wavefronts over four times as many
// compute units as groups of 256 (their pulls over as many L1 caches): the
// 4096-cell shock line steps 3-4% faster than with 128 and 256
constexpr int E2_WG = 64;

template <typename S, typename A, int VAR, int BOUNDED>
__global__ __launch_bounds__(E2_WG) void k_lb_e2(const S *__restrict__ src, S *__restrict__ dst,
                                              const S *__restrict__ gh, double *__restrict__ thR,
                                              double *__restrict__ that_, A *__restrict__ aux,
                                              double *__restrict__ lmul, Consts k)
{
    const int t = blockIdx.x * E2_WG + threadIdx.x;
    const int s = t >> 1;   // both lanes of a pair see the same s, so they branch alike
    if (s < k.ns) lb_site_e2pair<S, A, VAR, BOUNDED>(s, t & 1, src, dst, gh, thR, that_, aux, k, lmul);
}

template <typename A, int BOUNDED>
__global__ __launch_bounds__(WG) void k_mc(const double *__restrict__ that_, const A *__restrict__ aux,
                                           double *__restrict__ tmc, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s < k.ns) mc_site<A, BOUNDED>(s, that_, aux, tmc, k);
}

template <typename A, int VAR, int BOUNDED, bool FINAL>
__global__ __launch_bounds__(WG) void k_dif(const double *__restrict__ tin, double *__restrict__ tout,
                                            const double *__restrict__ that_, const A *__restrict__ aux,
                                            double *__restrict__ thR, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s < k.ns) dif_site<A, VAR, BOUNDED, FINAL>(s, tin, tout, that_, aux, thR, k);
}

// The theta_R transport of a small grid (at most TR_SMALL sites; lines take
// k_tr_line) in one work-group: MacCormack into LDS, then every FTCS sub-step ping-ponging in
// LDS with a work-group barrier between them, the last one with the second
// half of the relaxation.  One launch instead of 1 + n_sub; the per-site
// arithmetic is that of k_mc and k_dif, so the results are the same bits.
constexpr int TR_SMALL = 4096, TR_SMALL_WG = 1024;

template <typename A, int VAR, int BOUNDED>
__global__ __launch_bounds__(TR_SMALL_WG) void k_tr_small(const double *__restrict__ that_,
                                                          const A *__restrict__ aux, double *__restrict__ thR,
                                                          Consts k)
{
    extern __shared__ double lds[];
    double *tin = lds, *tout = lds + k.ns;
    for (int s = threadIdx.x; s < k.ns; s += TR_SMALL_WG) mc_site<A, BOUNDED>(s, that_, aux, tin, k);
    __syncthreads();
    for (int it = 0; it + 1 < k.nsub; it++) {
        for (int s = threadIdx.x; s < k.ns; s += TR_SMALL_WG)
            dif_site<A, VAR, BOUNDED, false>(s, tin, tout, that_, aux, thR, k);
        __syncthreads();
        double *t = tin;
        tin = tout;
        tout = t;
    }
    for (int s = threadIdx.x; s < k.ns; s += TR_SMALL_WG) dif_site<A, VAR, BOUNDED, true>(s, tin, tout, that_, aux, thR, k);
}

// The theta_R transport of a line (ny = nz = 1), bounded or sub-cycled, in one
// launch (any length; at most TL_HMAX - 1 sub-steps).  Unlike the one-work-group
// kernel it keeps every field of a sub-step in LDS, which also makes it the
// faster of the two on short lines.  Along a line the transport is two
// independent 1D problems, one per sublattice.  A work-group of WG threads owns
// WG - 2 H cells of one sublattice and stages them with a halo of H = nsub + 1
// cells on each side (theta_hat, u_x, rho, kfac rho theta), WG cells in all so
// that every thread holds one window cell (WG = 64, one wavefront, while the
// halos take at most half of it, else 256); MacCormack and every FTCS
// sub-step then run in LDS, the valid window shrinking by one cell per stage,
// so the halo cells are recomputed by both neighbours and no work-group waits
// for another.  The y and z terms of the stencils of mc_site / dif_site vanish
// on a line (their neighbours are the site itself and add exact zeros), and
// the x terms are evaluated in the same order; the compiler's fused
// multiply-adds may still round differently, so the results agree with
// k_mc + k_dif to round-off (a last bit here and there), not bit for bit.
constexpr int TL_HMAX = 64;

// work-group size of k_tr_line for nsub sub-steps, and the cells of a line each
// work-group produces (its window: these and a halo of nsub + 1 cells on each
// side, one per thread)
__host__ __device__ inline int tl_wg(int nsub) { return 2 * (nsub + 1) <= 32 ? 64 : 256; }
__host__ __device__ inline int tl_cells(int nsub, int wg) { return wg - 2 * (nsub + 1); }

template <typename A, int VAR, int BOUNDED, int TL_WG>
__global__ __launch_bounds__(TL_WG) void k_tr_line(const double *__restrict__ that_, const A *__restrict__ aux,
                                                   double *__restrict__ thR, Consts k)
{
    constexpr int TL_L = TL_WG;
    __shared__ double l_th[TL_L], l_u[TL_L], l_rho[TL_L], l_ks[TL_L], l_a[TL_L], l_b[TL_L];
    const int C = tl_cells(k.nsub, TL_WG), nx = k.nx, nchunk = (nx + C - 1) / C;
    const int sub = blockIdx.x / nchunk, x0 = (blockIdx.x - sub * nchunk) * C;
    const int H = k.nsub + 1, nout = min(C, nx - x0), Lw = nout + 2 * H;   // Lw <= TL_WG
    const int base = sub * nx, tid = threadIdx.x;
    // window cell i is the line's cell x0 - H + i (wrapped on a periodic line);
    // on a bounded line the cells beyond a face hold nothing and are never read
    auto cell = [&](int i, bool &in) {
        int x = x0 - H + i;
        if (BOUNDED) {
            in = x >= 0 && x < nx;
            return x;
        }
        in = true;
        x %= nx;
        return x < 0 ? x + nx : x;
    };
    // theta_R of the cell this thread updates in the last stage (cell
    // tid + 1 + nsub: the stages' cell ranges shift by one each), read now so
    // that its latency overlaps the staging and the sub-steps
    double thR_old = 0.0;
    {
        const int i = tid + 1 + k.nsub;
        bool in = false;
        const int x = i < Lw - 1 - k.nsub ? cell(i, in) : 0;
        if (in) thR_old = thR[base + x];
    }
    for (int i = tid; i < Lw; i += TL_WG) {
        bool in;
        int x = cell(i, in);
        if (in) {
            int s = base + x;
            l_th[i] = that_[s];
            l_u[i] = (double)aux[s];
            l_rho[i] = (double)aux[(size_t)3 * k.ns + s];
            l_ks[i] = k.kfac * (double)aux[(size_t)4 * k.ns + s];
        }
    }
    __syncthreads();
    // predictor theta* on [0, Lw-1)
    for (int i = tid; i < Lw - 1; i += TL_WG) {
        bool in;
        int x = cell(i, in);
        if (!in) continue;
        double t = l_th[i];
        double tp = (BOUNDED && x + 1 >= nx) ? k.thbc[1] : l_th[i + 1];
        double adv = 0.0;
        adv += l_u[i] * (tp - t);
        l_a[i] = t - adv;
    }
    __syncthreads();
    // corrector theta^mc on [1, Lw-1)
    for (int i = tid + 1; i < Lw - 1; i += TL_WG) {
        bool in;
        int x = cell(i, in);
        if (!in) continue;
        double ts = l_a[i];
        double tm = (BOUNDED && x - 1 < 0) ? k.thbc[0] : l_a[i - 1];
        double adv = 0.0;
        adv += l_u[i] * (ts - tm);
        l_b[i] = 0.5 * (l_th[i] + ts - adv);
    }
    __syncthreads();
    double *tin = l_b, *tout = l_a;
    for (int j = 1; j <= k.nsub; j++) {
        const bool last = j == k.nsub;
        for (int i = tid + 1 + j; i < Lw - 1 - j; i += TL_WG) {   // the last stage covers exactly the outputs
            bool in;
            int x = cell(i, in);
            if (!in) continue;
            double rho = l_rho[i], ks = l_ks[i], t = tin[i];
            double flux = 0.0, lap = 0.0;
#pragma unroll
            for (int dir = -1; dir <= 1; dir += 2) {
                double tq, kq;
                bool face = BOUNDED && (dir < 0 ? x - 1 < 0 : x + 1 >= nx);
                if (face) {
                    bool hi = dir > 0;
                    tq = hi ? k.thbc[1] : k.thbc[0];
                    bool wall = (hi ? k.bc[1] : k.bc[0]) == PGK_WALL;
                    double rg = wall ? rho : (hi ? k.rhobc[1] : k.rhobc[0]);
                    kq = k.kfac * rg * tq;
                } else {
                    tq = tin[i + dir];
                    kq = l_ks[i + dir];
                }
                flux += 0.5 * (ks + kq) * (tq - t);
                lap += tq - t;
            }
            double tdif = VAR == PGK_CN ? t + k.isub * 2.0 * flux / (rho * k.delta)
                                        : t + k.isub * 2.0 * ks / (rho * k.delta) * lap;
            if (!last) {
                tout[i] = tdif;
            } else {
                int s = base + x;
                const double v = thR_old;   // this is the thread's cell tid + 1 + nsub
                if (VAR == PGK_CN) thR[s] = tdif + (l_th[i] - v);
                else thR[s] = (tdif + k.X * v) * k.inv1X;
            }
        }
        __syncthreads();
        double *t = tin;
        tin = tout;
        tout = t;
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
#ifndef PGK_TR_TY
#define PGK_TR_TY 8
#endif
#ifndef PGK_TR_TZ
#define PGK_TR_TZ 128
#endif
constexpr int TX = 64, TY = PGK_TR_TY, TZ = PGK_TR_TZ;
constexpr int TWG = TX * TY;                 // one output column per thread
constexpr int HX = TX + 4, HY = TY + 4;      // theta_hat plane (origin -2)
constexpr int SX = TX + 3, SY = TY + 3;      // theta* and u plane (origin -2)
constexpr int MX = TX + 2, MY = TY + 2;      // theta^mc and rho*theta plane (origin -1)
constexpr int NH = (HX * HY + TWG - 1) / TWG; // staged points per thread
constexpr int NS = (SX * SY + TWG - 1) / TWG;
constexpr int NM = (MX * MY + TWG - 1) / TWG;

__device__ __forceinline__ int wrapn(int v, int n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

template <typename A, int VAR>
__global__ __launch_bounds__(TWG) void k_tr(const double *__restrict__ that_, const A *__restrict__ aux,
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
        int i = min(tid + j * TWG, HX * HY - 1);
        int ly = i / HX, lx = i - ly * HX;
        oh[j] = wrapn(y0 + ly - 2, k.ny) * k.nx + wrapn(x0 + lx - 2, k.nx);
    }
#pragma unroll
    for (int j = 0; j < NS; j++) {
        int i = min(tid + j * TWG, SX * SY - 1);
        int ly = i / SX, lx = i - ly * SX;
        os[j] = wrapn(y0 + ly - 2, k.ny) * k.nx + wrapn(x0 + lx - 2, k.nx);
    }
#pragma unroll
    for (int j = 0; j < NM; j++) {
        int i = min(tid + j * TWG, MX * MY - 1);
        int ly = i / MX, lx = i - ly * MX;
        om[j] = wrapn(y0 + ly - 1, k.ny) * k.nx + wrapn(x0 + lx - 1, k.nx);
    }
    const int lxo = tid % TX, lyo = tid / TX;
    const bool outv = (x0 + lxo < k.nx) && (y0 + lyo < k.ny);
    const int oo = outv ? (y0 + lyo) * k.nx + (x0 + lxo) : 0;
    auto zoff = [&](int z) { return subo + wrapn(z, k.nz) * plane; };

    // registers carrying the data of the next two iterations (slot = iteration
    // parity, a compile-time index): each plane's loads have two planes of
    // work to arrive in
    double r_th[2][NH];
    A r_u[2][3][NS], r_pt[2][NM];
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    // data of iteration j: theta_hat(j + 1), u(j), rho theta(j)
    auto fetch = [&](auto slot, int zth, int zu) {
        constexpr int S = decltype(slot)::value;
        int zt = zoff(zth), zuo = zoff(zu);
#pragma unroll
        for (int j = 0; j < NH; j++) r_th[S][j] = that_[zt + oh[j]];
#pragma unroll
        for (int j = 0; j < NS; j++) {
            r_u[S][0][j] = aux[zuo + os[j]];
            r_u[S][1][j] = aux[(size_t)k.ns + zuo + os[j]];
            r_u[S][2][j] = aux[(size_t)2 * k.ns + zuo + os[j]];
        }
#pragma unroll
        for (int j = 0; j < NM; j++) r_pt[S][j] = aux[(size_t)4 * k.ns + zuo + om[j]];
    };
    auto stash = [&](auto slot, int slot_th, int slot3) {
        constexpr int S = decltype(slot)::value;
#pragma unroll
        for (int j = 0; j < NH; j++)
            if (tid + j * TWG < HX * HY) l_th[slot_th][tid + j * TWG] = r_th[S][j];
#pragma unroll
        for (int j = 0; j < NS; j++)
            if (tid + j * TWG < SX * SY) {
                l_u[0][tid + j * TWG] = r_u[S][0][j];
                l_u[1][tid + j * TWG] = r_u[S][1][j];
                l_u[2][tid + j * TWG] = r_u[S][2][j];
            }
#pragma unroll
        for (int j = 0; j < NM; j++)
            if (tid + j * TWG < MX * MY) l_pt[slot3][tid + j * TWG] = r_pt[S][j];
    };

    // prologue: theta_hat(z0-2) straight into its slot, then the data of
    // iterations z0-2 and z0-1
    {
        int zt = zoff(z0 - 2);
#pragma unroll
        for (int j = 0; j < NH; j++)
            if (tid + j * TWG < HX * HY) l_th[(z0 + 2) & 1][tid + j * TWG] = that_[zt + oh[j]];
    }
    fetch(I0{}, z0 - 1, z0 - 2);
    fetch(I1{}, z0, z0 - 1);

    // theta_hat of this thread's column at the previous plane, taken from the
    // LDS ring while it still holds that plane (the output plane lags by one)
    double th_prev = 0.0;
    const int hc = (lyo + 2) * HX + lxo + 2;

    auto iteration = [&](auto slot, int zz) {
        const int rz = zz + 4;                          // non-negative ring index
        stash(slot, (rz + 1) & 1, rz % 3);             // theta_hat(zz+1), u(zz), rho theta(zz)
        if (zz + 2 <= zend) fetch(slot, zz + 3, zz + 2);   // iteration zz+2, in flight for two planes
        const int zo = zz - 1;                          // output plane of this iteration
        double o_rho = 0.0, o_v = 0.0;
        const double o_th = th_prev;                    // theta_hat(zo)
        if (zz >= z0 + 1 && outv) {
            int g = zoff(zo) + oo;
            o_rho = (double)aux[(size_t)3 * k.ns + g];
            o_v = thR[g];
        }
        __syncthreads();
        // predictor theta*(zz) = th - sum_a u_a (th(+e_a) - th), region origin -2
        for (int i = tid; i < SY * SX; i += TWG) {
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
            for (int i = tid; i < MY * MX; i += TWG) {
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
        th_prev = l_th[rz & 1][hc];                     // theta_hat(zz), the next output plane
        __syncthreads();
    };

    for (int zz = z0 - 2; zz <= zend; zz += 2) {
        iteration(I0{}, zz);
        if (zz + 1 <= zend) iteration(I1{}, zz + 1);
    }
}

// ---------------------------------------------------------------------------
// boundaries: x ghost populations
// ---------------------------------------------------------------------------
// One thread per (side, ghost column gz*ny+gy).  Diffuse wall: the density of
// the re-emitted populations balances the mass that left through the face in
// the last collision (zero net mass flux per column); Dirichlet: equilibrium.
// One thread per (side, ghost column).
template <typename S>
__global__ __launch_bounds__(64) void k_bc(const S *__restrict__ src, S *__restrict__ gh, Consts k)
{
    // one wavefront per (face, ghost column): the columns of the two x faces,
    // then (y bounded) those of the two y faces
    int col = blockIdx.x, f = 0;
    while (f < 3 && col >= face_columns(f, k)) col -= face_columns(f++, k);
    bc_column<S>(f, col, threadIdx.x, src, gh, k);
}

// work-groups of k_bc: one per ghost column of every face the grid bounds
// (an x face is listed even when periodic; its work-groups return at once)
static int bc_launches(const Consts &k)
{
    int n = 2 * face_columns(0, k);
    if (k.bc[2] != PGK_PERIODIC) n += 2 * face_columns(2, k);
    return n;
}

template <typename S, int BOUNDED, int EQ>
__global__ __launch_bounds__(WG) void k_init(S *__restrict__ dst, S *__restrict__ gh, double *__restrict__ thR,
                                             const double *__restrict__ rho, const double *__restrict__ u,
                                             const double *__restrict__ thT, const double *__restrict__ thRin,
                                             double *__restrict__ lmul, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    if (s < k.ns) {
        init_site<S, BOUNDED, EQ>(s, dst, gh, thR, rho, u, thT, thRin, k, (size_t)k.ns);
        // no warm start yet: the first step's Newton runs start from the Gaussian
        if (EQ == PGK_E2 && lmul)
            for (int i = 0; i < 2 * E2_NL; i++) lmul[(size_t)i * k.ns + s] = __builtin_nan("");
    }
}

template <typename S, int BOUNDED, bool REDUCE>
__global__ __launch_bounds__(WG) void k_moments(const S *__restrict__ src, const S *__restrict__ gh,
                                                const double *__restrict__ thR, double *__restrict__ orho,
                                                double *__restrict__ ou, double *__restrict__ othT,
                                                double *__restrict__ othR, double *__restrict__ oP,
                                                double *__restrict__ partial, Consts k)
{
    int s = blockIdx.x * WG + threadIdx.x;
    double red[5] = {0, 0, 0, 0, 0};
    if (s < k.ns) {
        Mom m;
        Solve so = moments_site<S, BOUNDED>(s, src, gh, thR, k, m);
        if (REDUCE) {
            red[0] = m.rho;
            red[1] = m.j[0];
            red[2] = m.j[1];
            red[3] = m.j[2];
            red[4] = 0.5 * (m.P[0] + m.P[1] + m.P[2]) + 0.5 * k.delta * m.rho * so.r;
        } else {
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
    double bc_u[4][3]{};
    bool bc_set[4] = {false, false, false, false};   // face state given by pgk_set_bc
    // x ghosts: ghosts_ok = they hold what the next pull needs (filled from the
    // face states in force when the stored populations were collided, as the
    // streaming of that step would); face_changed = a face state changed since
    bool ghosts_ok = false, face_changed = false;
    std::string err;
    // carved from the aux buffer
    double *that_ = nullptr, *tmc = nullptr, *tmc2 = nullptr, *partial = nullptr, *totals = nullptr;
    void *aux = nullptr, *gh = nullptr;
    double *lmul = nullptr;       // E2 only: Newton warm starts
    int nblk = 0;
    // kernel timing
    bool timing = false;
    std::vector<hipEvent_t> events;   // pool
    std::vector<int> marks;           // kernel id of the interval ending at event i (-1: start)
    size_t nev = 0;
    // replayed chunks of graph_steps steps (an even count), one per starting
    // buffer (invalid after a change of parameters, faces or buffers); 0: launch
    // every kernel directly.  32 steps per graph take 4-6% off a step of a
    // grid of a few thousand sites and are neutral on large grids; 2 steps
    // per graph are slower than direct launches.
    int graph_steps = 32;
    bool transport_ref = false;   // theta_R transport by k_mc + k_dif on every grid
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    hipStream_t capture = nullptr;   // private stream the pair is recorded on (the null stream cannot be)
    void drop_graphs()
    {
        for (auto &g : graph)
            if (g) {
                (void)hipGraphExecDestroy(g);
                g = nullptr;
            }
    }
    ~pgk_ctx()
    {
        drop_graphs();
        if (capture) (void)hipStreamDestroy(capture);
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
    if (g->equilibrium != PGK_F3 && g->equilibrium != PGK_E2 && g->equilibrium != PGK_F4) return false;
    for (int s = 0; s < 2; s++)
        if (g->bc_x[s] < PGK_PERIODIC || g->bc_x[s] > PGK_DIRICHLET || g->bc_y[s] < PGK_PERIODIC ||
            g->bc_y[s] > PGK_DIRICHLET)
            return false;
    if ((g->bc_x[0] == PGK_PERIODIC) != (g->bc_x[1] == PGK_PERIODIC)) return false;
    if ((g->bc_y[0] == PGK_PERIODIC) != (g->bc_y[1] == PGK_PERIODIC)) return false;
    if (g->bc_x[0] != PGK_PERIODIC && g->nx < 2) return false;
    if (g->bc_y[0] != PGK_PERIODIC && g->ny < 2) return false;
    return true;
}

// aux layout (bytes, each part 256-aligned): that_[ns] f64, tmc[ns] f64,
// aux fields [5][ns] (f64 or f32), partial[nblk*5] f64, totals[8] f64,
// ghosts [2][41][4][nz*ny] (population type), tmc2[ns] f64
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static void aux_layout(const pgk_grid *g, size_t off[9])
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
    Consts k{};
    k.nx = g->nx; k.ny = g->ny; k.nz = g->nz;
    k.bc[0] = g->bc_x[0]; k.bc[1] = g->bc_x[1]; k.bc[2] = g->bc_y[0]; k.bc[3] = g->bc_y[1];
    off[6] = off[5] + align256((size_t)ghost_count(k) * elt);
    off[7] = off[6] + align256(ns * 8);
    // E2: the two multiplier sets of each site's last equilibria, [2 * E2_NL][ns]
    off[8] = off[7] + (g->equilibrium == PGK_E2 ? align256(2ull * E2_NL * ns * 8) : 0);
}

extern "C" int pgk_buffer_sizes(const pgk_grid *g, size_t sizes[PGK_NBUF])
{
    if (!grid_ok(g) || !sizes) return PGK_EINVAL;
    size_t ns = 2ull * g->nx * g->ny * g->nz;
    size_t elt = g->precision == PGK_FP64 ? 8 : 4;
    size_t off[9];
    aux_layout(g, off);
    sizes[PGK_BUF_POP0] = NQ * ns * elt;
    sizes[PGK_BUF_POP1] = NQ * ns * elt;
    sizes[PGK_BUF_THETAR] = ns * 8;
    sizes[PGK_BUF_AUX] = off[8];
    return PGK_OK;
}

// F3 with a general covariance: the third-order Hermite projection about
// (0, theta0) of N(u, lam), D = lam - theta0 I (the device collide evaluates
// the same polynomial in even/odd pairs)
static void f3_host_lam(double th0, const double w6[6], double rho, const double u[3], const double lam[6],
                        double F[NQ])
{
    double D[3][3] = {{lam[0] - th0, lam[3], lam[4]}, {lam[3], lam[1] - th0, lam[5]}, {lam[4], lam[5], lam[2] - th0}};
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double trD = D[0][0] + D[1][1] + D[2][2];
    for (int q = 0; q < NQ; q++) {
        double c[3] = {0.5 * c2(q, 0), 0.5 * c2(q, 1), 0.5 * c2(q, 2)};
        double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2], cDc = 0.0, cDu = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                cDc += c[a] * D[a][b] * c[b];
                cDu += c[a] * D[a][b] * u[b];
            }
        double a2 = cu * cu + cDc - th0 * (uu + trD);
        double a3 = cu * cu * cu + 3.0 * cDc * cu - th0 * (3.0 * uu * cu + 6.0 * cDu + 3.0 * trD * cu);
        F[q] = w6[shell_of(q)] * rho * (1.0 + cu / th0 + a2 / (2 * th0 * th0) + a3 / (6 * th0 * th0 * th0));
    }
}

// F4 correction basis at velocity c: h_xx, h_yy, h_zz, then h_ab + h_ba for
// xy, xz, yz, with h_ab(c) = c_a c_b (c^2 - 7 theta0) - delta_ab theta0 (c^2 - 5 theta0)
static double f4_basis(int j, const double c[3], double th0)
{
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    double h = c[ia[j]] * c[ib[j]] * (cc - 7.0 * th0) - (ia[j] == ib[j] ? th0 * (cc - 5.0 * th0) : 0.0);
    return j < 3 ? h : 2.0 * h;
}

// Inverse of the 6 x 6 lattice matrix M[e][j] = sum_q w_q basis_j(c_q) c_q^2 c_qa c_qb
// (e = ab in xx yy zz xy xz yz order): maps the wanted change of the
// contracted fourth moment to the correction coefficients K.  False if singular.
static bool f4_matrix(double th0, const double w6[6], double inv[36])
{
    static const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    double M[6][12];
    for (int e = 0; e < 6; e++) {
        for (int j = 0; j < 6; j++) {
            double m = 0.0;
            for (int q = 0; q < NQ; q++) {
                double c[3] = {0.5 * c2(q, 0), 0.5 * c2(q, 1), 0.5 * c2(q, 2)};
                double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                m += w6[shell_of(q)] * f4_basis(j, c, th0) * cc * c[ia[e]] * c[ib[e]];
            }
            M[e][j] = m;
            M[e][6 + j] = e == j ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < 6; col++) {   // Gauss-Jordan with partial pivoting
        int piv = col;
        for (int r = col + 1; r < 6; r++)
            if (std::fabs(M[r][col]) > std::fabs(M[piv][col])) piv = r;
        if (!(std::fabs(M[piv][col]) > 1e-300)) return false;
        if (piv != col)
            for (int t = 0; t < 12; t++) std::swap(M[col][t], M[piv][t]);
        double d = 1.0 / M[col][col];
        for (int t = 0; t < 12; t++) M[col][t] *= d;
        for (int r = 0; r < 6; r++) {
            if (r == col) continue;
            double f = M[r][col];
            for (int t = 0; t < 12; t++) M[r][t] -= f * M[col][t];
        }
    }
    for (int e = 0; e < 6; e++)
        for (int j = 0; j < 6; j++) inv[e * 6 + j] = M[e][6 + j];
    return true;
}

// F4 on the host: F3 plus the correction of the target (rho, u, lam)
static void f4_host_lam(double th0, const double w6[6], const double inv[36], double rho, const double u[3],
                        const double lam[6], double F[NQ])
{
    f3_host_lam(th0, w6, rho, u, lam, F);
    double K[6];
    f4_coeffs(inv, th0, rho, u, lam, K);
    for (int q = 0; q < NQ; q++) {
        double c[3] = {0.5 * c2(q, 0), 0.5 * c2(q, 1), 0.5 * c2(q, 2)}, corr = 0.0;
        for (int j = 0; j < 6; j++) corr += K[j] * f4_basis(j, c, th0);
        F[q] += w6[shell_of(q)] * corr;
    }
}

extern "C" int pgk_lattice(double theta0, double *c, double *w)
{
    if (!c || !w) return PGK_EINVAL;
    double w6[6];
    shell_weights(theta0 > 0 ? theta0 : THETA0_PRINTED, w6);
    for (int q = 0; q < NQ; q++) {
        for (int a = 0; a < 3; a++) c[3 * q + a] = 0.5 * c2(q, a);
        w[q] = w6[shell_of(q)];
    }
    return PGK_OK;
}

extern "C" int pgk_equilibrium(int equilibrium, double theta0, double rho, const double *u, const double *lam,
                               double *F)
{
    if (!u || !lam || !F || !(rho > 0)) return PGK_EINVAL;
    double th0 = theta0 > 0 ? theta0 : THETA0_PRINTED, w6[6];
    shell_weights(th0, w6);
    if (equilibrium == PGK_F3) {
        f3_host_lam(th0, w6, rho, u, lam, F);
        return PGK_OK;
    }
    if (equilibrium == PGK_F4) {
        double inv[36];
        if (!f4_matrix(th0, w6, inv)) return PGK_EINVAL;
        f4_host_lam(th0, w6, inv, rho, u, lam, F);
        return PGK_OK;
    }
    if (equilibrium != PGK_E2) return PGK_EINVAL;
    double l[E2_NL];
    if (e2_solve(th0, w6, rho, u, lam, l) < 0) return PGK_EINFEASIBLE;
    for (int q = 0; q < NQ; q++) F[q] = e2_population(l, w6, q);
    return PGK_OK;
}

extern "C" int pgk_resolve(const pgk_targets *t, pgk_resolved *out)
{
    if (!t || !out) return PGK_EINVAL;
    double th0 = t->theta0 > 0 ? t->theta0 : THETA0_PRINTED;
    double d = t->delta, nu = t->nu, Pr = t->Pr, lb = t->mub_over_mu;
    if (!(d > 0) || !(nu > 0) || !(Pr > 0) || !(lb > 0)) return PGK_EINVAL;
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
    // b = 1 leaves tau1/tau free; an explicit b > 1 (the Landau-number runs of
    // Sec. 6 at Pr 5 and 10) pairs with a viscosity ratio below the floor
    if (!(b != 1.0) || b < -0.5) return PGK_EINFEASIBLE;
    double r = (lb / cd - 1.0) / (1.0 - b);              // eta_b/eta = cd (1 + (1-b) tau1/tau)
    if (!(r > 0)) return PGK_EINFEASIBLE;
    double B = 1.0 + 1.0 / r;
    if (!(b < B)) return PGK_EINFEASIBLE;                // shear viscosity p tau/(B - b) > 0
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
    c->k.bc[2] = g->bc_y[0]; c->k.bc[3] = g->bc_y[1];
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
    size_t off[9];
    aux_layout(&c->g, off);
    char *a = (char *)bufs[PGK_BUF_AUX];
    c->lmul = c->g.equilibrium == PGK_E2 ? (double *)(a + off[7]) : nullptr;
    c->tmc2 = (double *)(a + off[6]);
    c->that_ = (double *)(a + off[0]);
    c->tmc = (double *)(a + off[1]);
    c->aux = (void *)(a + off[2]);
    c->partial = (double *)(a + off[3]);
    c->totals = (double *)(a + off[4]);
    c->gh = (void *)(a + off[5]);
    c->bound = true;
    c->initialised = false;
    c->ghosts_ok = c->face_changed = false;
    c->drop_graphs();
    return PGK_OK;
}

static int settle_ghosts(pgk_ctx *c);

// face equilibria (wall: F3 at unit density; Dirichlet: the grid's
// equilibrium of the face state) and diffusion sub-steps; PGK_EINFEASIBLE if
// a Dirichlet state has no E2 equilibrium
static int fill_bc(pgk_ctx *c)
{
    Consts &k = c->k;
    k.nsub = diffusion_substeps(k, c->res.kr);
    k.isub = 1.0 / k.nsub;
    for (int f = 0; f < 4; f++) {
        if (k.bc[f] == PGK_PERIODIC || !c->bc_set[f]) continue;
        double rho = k.bc[f] == PGK_WALL ? 1.0 : k.rhobc[f];
        if (k.bc[f] == PGK_DIRICHLET && c->g.equilibrium == PGK_E2) {
            double th = k.thbc[f], lam[6] = {th, th, th, 0.0, 0.0, 0.0}, l[E2_NL];
            if (e2_solve(k.th0, k.w, rho, c->bc_u[f], lam, l) < 0)
                return fail(c, PGK_EINFEASIBLE, "the Dirichlet face state has no E2 equilibrium on the lattice");
            for (int q = 0; q < NQ; q++) k.Fbc[f][q] = e2_population(l, k.w, q);
        } else if (k.bc[f] == PGK_DIRICHLET && c->g.equilibrium == PGK_F4) {
            double th = k.thbc[f], lam[6] = {th, th, th, 0.0, 0.0, 0.0};
            f4_host_lam(k.th0, k.w, k.f4inv, rho, c->bc_u[f], lam, k.Fbc[f]);
        } else {
            f3_host(k.th0, k.w, rho, c->bc_u[f], k.thbc[f], k.Fbc[f]);
        }
        // mass re-emitted into one ghost column at unit density when the
        // face's other in-plane axis is periodic (every column alike): every
        // population pulled from beyond the face, over both sublattices
        const int a = f / 2, side = f % 2, na = a == 0 ? k.nx : k.ny;
        double in = 0.0;
        for (int q = 0; q < NQ; q++)
            for (int sub = 0; sub < 2; sub++)
                for (int i = 0; i < na; i++) {
                    int qa = 2 * i + sub - c2(q, a);
                    bool outside = side == 0 ? qa < 0 : qa > 2 * na - 1;
                    if (outside) in += k.Fbc[f][q];
                }
        k.in_col[f] = in;
    }
    return PGK_OK;
}

extern "C" int pgk_set_params(pgk_ctx *c, const pgk_params *p, pgk_resolved *out)
{
    if (!c || !p) return PGK_EINVAL;
    if (!(p->tau > 0) || !(p->tau1 > 0) || !(p->delta > 0) || !(p->b >= -0.5) || !(p->kr >= 0) ||
        !(p->b < 1.0 + p->tau / p->tau1))
        return fail(c, PGK_EINVAL, "parameters out of range");
    // beyond b = 1 the ES covariance can lose positive definiteness (Sec. 2); the
    // polynomial targets stay defined, the exponential E2 target does not
    if (p->b > 1.0 && c->g.equilibrium == PGK_E2)
        return fail(c, PGK_EINVAL, "b > 1 needs a polynomial equilibrium (F3 or F4)");
    int rc0 = settle_ghosts(c);   // the pending pull keeps the old face equilibria
    if (rc0) return rc0;
    c->face_changed = true;
    Consts &k = c->k;
    k.th0 = p->theta0 > 0 ? p->theta0 : THETA0_PRINTED;
    shell_weights(k.th0, k.w);
    for (int i = 0; i < 6; i++) {
        k.whi[i] = (float)k.w[i];
        k.wlo[i] = (float)(k.w[i] - (double)k.whi[i]);
    }
    if (c->g.equilibrium == PGK_F4 && !f4_matrix(k.th0, k.w, k.f4inv))
        return fail(c, PGK_EINVAL, "the F4 lattice matrix is singular at this theta0");
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
    c->drop_graphs();
    return fill_bc(c);
}

extern "C" int pgk_set_bc(pgk_ctx *c, int axis, int side, double rho, const double u[3], double theta)
{
    if (!c || axis < 0 || axis > 1 || side < 0 || side > 1 || !(theta > 0)) return PGK_EINVAL;
    const int f = 2 * axis + side;
    if (c->k.bc[f] == PGK_PERIODIC) return fail(c, PGK_EINVAL, "face is periodic");
    if (c->k.bc[f] == PGK_DIRICHLET && !(rho > 0)) return fail(c, PGK_EINVAL, "Dirichlet density must be positive");
    if (u && u[axis] != 0.0 && c->k.bc[f] == PGK_WALL) return fail(c, PGK_EINVAL, "a wall cannot move normal to itself");
    int rc0 = settle_ghosts(c);   // the pending pull keeps the old face state
    if (rc0) return rc0;
    c->face_changed = true;
    c->k.rhobc[f] = rho;
    c->k.thbc[f] = theta;
    c->bc_set[f] = true;
    c->drop_graphs();
    for (int a = 0; a < 3; a++) c->bc_u[f][a] = u ? u[a] : 0.0;
    return c->params_set ? fill_bc(c) : PGK_OK;
}

extern "C" int pgk_set_bc_x(pgk_ctx *c, int side, double rho, const double u[3], double theta)
{
    return pgk_set_bc(c, 0, side, rho, u, theta);
}

static bool any_wall(const pgk_ctx *c)
{
    for (int f = 0; f < 4; f++)
        if (c->k.bc[f] == PGK_WALL) return true;
    return false;
}

// every bounded face has its state
static int faces_set(pgk_ctx *c)
{
    for (int f = 0; f < 4; f++)
        if (c->k.bc[f] != PGK_PERIODIC && !c->bc_set[f])
            return fail(c, PGK_EINVAL, "a bounded face has no state (pgk_set_bc)");
    return PGK_OK;
}

static bool bounded(const pgk_ctx *c) { return c->k.bc[0] != PGK_PERIODIC || c->k.bc[2] != PGK_PERIODIC; }

// the kernels' face level: BND_NONE, BND_X (faces on x only) or BND_XY
static int face_level(const pgk_ctx *c)
{
    return c->k.bc[2] != PGK_PERIODIC ? BND_XY : c->k.bc[0] != PGK_PERIODIC ? BND_X : BND_NONE;
}

// Fill the x ghosts the next pull reads, if they are not filled yet, from the
// face states in force now (before a change of those states takes effect).
static int settle_ghosts(pgk_ctx *c)
{
    if (!c->initialised || c->steps == 0 || !bounded(c) || c->ghosts_ok) return PGK_OK;
    int nbc = bc_launches(c->k);   // one wavefront per face column
    if (c->g.precision == PGK_FP64)
        hipLaunchKernelGGL((k_bc<double>), dim3(nbc), dim3(64), 0, c->stream, (const double *)c->buf[c->cur],
                           (double *)c->gh, c->k);
    else
        hipLaunchKernelGGL((k_bc<float>), dim3(nbc), dim3(64), 0, c->stream, (const float *)c->buf[c->cur],
                           (float *)c->gh, c->k);
    HIPCHECK(c, hipGetLastError());
    c->ghosts_ok = true;
    return PGK_OK;
}

template <typename S, int EQ>
static int init_t(pgk_ctx *c, const double *rho, const double *u, const double *thT, const double *thR)
{
    dim3 grid(c->nblk), block(WG);
    S *dst = (S *)c->buf[c->cur];
    if (bounded(c))
        hipLaunchKernelGGL((k_init<S, BND_XY, EQ>), grid, block, 0, c->stream, dst, (S *)c->gh,
                           (double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, c->lmul, c->k);
    else
        hipLaunchKernelGGL((k_init<S, BND_NONE, EQ>), grid, block, 0, c->stream, dst, (S *)c->gh,
                           (double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, c->lmul, c->k);
    HIPCHECK(c, hipGetLastError());
    return PGK_OK;
}

extern "C" int pgk_init_fields(pgk_ctx *c, const double *rho, const double *u, const double *thT, const double *thR)
{
    if (!c) return PGK_EINVAL;
    if (!c->bound) return fail(c, PGK_ENOTBOUND, "buffers not bound");
    if (!c->params_set) return fail(c, PGK_EINVAL, "parameters not set");
    if (!rho || !u || !thT || !thR) return fail(c, PGK_EINVAL, "null field");
    if (int rcf = faces_set(c)) return rcf;
    c->cur = 0;
    c->steps = 0;
    // the initialisation pushes what the first pull reads; from the second
    // step on the ghosts come from the face states
    c->ghosts_ok = true;
    c->face_changed = true;
    int eq = c->g.equilibrium, rc;
    if (c->g.precision == PGK_FP64)
        rc = eq == PGK_E2 ? init_t<double, PGK_E2>(c, rho, u, thT, thR)
           : eq == PGK_F4 ? init_t<double, PGK_F4>(c, rho, u, thT, thR)
                          : init_t<double, PGK_F3>(c, rho, u, thT, thR);
    else
        rc = eq == PGK_E2 ? init_t<float, PGK_E2>(c, rho, u, thT, thR)
           : eq == PGK_F4 ? init_t<float, PGK_F4>(c, rho, u, thT, thR)
                          : init_t<float, PGK_F3>(c, rho, u, thT, thR);
    if (rc == PGK_OK) c->initialised = true;
    return rc;
}

template <typename S, typename A, int VAR, int BND, int EQ>
static int step_t(pgk_ctx *c, int64_t n)
{
    dim3 grid(c->nblk), block(WG);
    int nbc = bc_launches(c->k);   // one wavefront per face column
    for (int64_t it = 0; it < n; it++) {
        S *src = (S *)c->buf[c->cur], *dst = (S *)c->buf[1 - c->cur];
        mark(c, -1);
        if (BND && !c->ghosts_ok) {
            hipLaunchKernelGGL((k_bc<S>), dim3(nbc), dim3(64), 0, c->stream, src, (S *)c->gh, c->k);
            mark(c, 3);
            c->ghosts_ok = true;
        }
        if constexpr (EQ == PGK_E2) {
            hipLaunchKernelGGL((k_lb_e2<S, A, VAR, BND>), dim3((2 * c->k.ns + E2_WG - 1) / E2_WG), dim3(E2_WG), 0,
                               c->stream, src, dst,
                               (const S *)c->gh, (double *)c->buf[PGK_BUF_THETAR], c->that_, (A *)c->aux, c->lmul,
                               c->k);
        } else {
            constexpr int nt = lb_wg<S, BND, EQ>();
            hipLaunchKernelGGL((k_lb<S, A, VAR, BND, EQ, nt>), dim3((c->k.ns + nt - 1) / nt), dim3(nt), 0, c->stream,
                               src, dst, (const S *)c->gh, (double *)c->buf[PGK_BUF_THETAR], c->that_, (A *)c->aux,
                               c->lmul, c->k);
        }
        mark(c, 0);
        if (!c->transport_ref && (BND || c->k.nsub > 1) && c->k.ny == 1 && c->k.nz == 1 &&
            c->k.nsub + 1 <= TL_HMAX) {
            const int wg = tl_wg(c->k.nsub), C = tl_cells(c->k.nsub, wg), nchunk = (c->k.nx + C - 1) / C;
            if (wg == 64)
                hipLaunchKernelGGL((k_tr_line<A, VAR, BND, 64>), dim3(2 * nchunk), dim3(64), 0, c->stream,
                                   c->that_, (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
            else
                hipLaunchKernelGGL((k_tr_line<A, VAR, BND, 256>), dim3(2 * nchunk), dim3(256), 0, c->stream,
                                   c->that_, (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 2);
        } else if (!c->transport_ref && (BND || c->k.nsub > 1) && c->k.ns <= TR_SMALL) {
            hipLaunchKernelGGL((k_tr_small<A, VAR, BND>), dim3(1), dim3(TR_SMALL_WG), sizeof(double) * 2 * c->k.ns,
                               c->stream, c->that_, (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 2);
        } else if (c->transport_ref || BND || c->k.nsub > 1) {
            // MacCormack, then the diffusion in nsub FTCS sub-steps (ping-pong
            // between two scratch fields), the last one with the second half
            hipLaunchKernelGGL((k_mc<A, BND>), grid, block, 0, c->stream, c->that_, (const A *)c->aux, c->tmc, c->k);
            mark(c, 1);
            double *tin = c->tmc, *tout = c->tmc2;
            for (int it = 0; it + 1 < c->k.nsub; it++) {
                hipLaunchKernelGGL((k_dif<A, VAR, BND, false>), grid, block, 0, c->stream, tin, tout, c->that_,
                                   (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
                double *t = tin;
                tin = tout;
                tout = t;
            }
            hipLaunchKernelGGL((k_dif<A, VAR, BND, true>), grid, block, 0, c->stream, tin, tout, c->that_,
                               (const A *)c->aux, (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 2);
        } else {
            int ntile = ((c->k.nx + TX - 1) / TX) * ((c->k.ny + TY - 1) / TY) * ((c->k.nz + TZ - 1) / TZ) * 2;
            hipLaunchKernelGGL((k_tr<A, VAR>), dim3(ntile), dim3(TWG), 0, c->stream, c->that_, (const A *)c->aux,
                               (double *)c->buf[PGK_BUF_THETAR], c->k);
            mark(c, 1);
        }
        c->cur = 1 - c->cur;
        c->steps++;
        // a wall re-emits what the last collision sent into it: new ghosts
        // every step; Dirichlet ghosts stay until a face state changes
        if (BND && (any_wall(c) || c->face_changed)) c->ghosts_ok = false;
        c->face_changed = false;
    }
    HIPCHECK(c, hipGetLastError());
    return PGK_OK;
}

using StepFn = int (*)(pgk_ctx *, int64_t);

template <typename S, typename A, int EQ>
static StepFn step_fn_v(const pgk_ctx *c)
{
    const int b = face_level(c);
    if (c->g.variant == PGK_CN)
        return b == BND_XY ? &step_t<S, A, PGK_CN, BND_XY, EQ>
             : b == BND_X  ? &step_t<S, A, PGK_CN, BND_X, EQ>
                           : &step_t<S, A, PGK_CN, BND_NONE, EQ>;
    return b == BND_XY ? &step_t<S, A, PGK_LIT, BND_XY, EQ>
         : b == BND_X  ? &step_t<S, A, PGK_LIT, BND_X, EQ>
                       : &step_t<S, A, PGK_LIT, BND_NONE, EQ>;
}

static StepFn step_fn(const pgk_ctx *c)
{
    if (c->g.equilibrium == PGK_E2)
        return c->g.precision == PGK_FP64 ? step_fn_v<double, double, PGK_E2>(c) : step_fn_v<float, float, PGK_E2>(c);
    if (c->g.equilibrium == PGK_F4)
        return c->g.precision == PGK_FP64 ? step_fn_v<double, double, PGK_F4>(c) : step_fn_v<float, float, PGK_F4>(c);
    return c->g.precision == PGK_FP64 ? step_fn_v<double, double, PGK_F3>(c) : step_fn_v<float, float, PGK_F3>(c);
}

extern "C" int pgk_step(pgk_ctx *c, int64_t n)
{
    if (!c || n < 0) return PGK_EINVAL;
    if (!c->initialised) return fail(c, PGK_EINVAL, "fields not initialised");
    if (n == 0) return PGK_OK;
    StepFn f = step_fn(c);
    const int64_t K = c->graph_steps;
    // replay off, fewer steps than a chunk, or per-kernel timing (events
    // between the launches): launch directly
    if (K == 0 || c->timing || n - (c->steps == 0) < K) return f(c, n);
    int rc;
    if (c->steps == 0) {   // the first step has no ghost refresh: not part of a chunk
        rc = f(c, 1);
        if (rc) return rc;
        n--;
    }
    // a replay starts from filled ghosts; the chunk keeps them filled (with
    // walls it refreshes them before every step, its first included)
    rc = settle_ghosts(c);
    if (rc) return rc;
    const bool walls = any_wall(c);
    // a chunk of an even number of steps returns the state to the buffer it started from
    const int p = c->cur;
    if (!c->graph[p]) {
        if (!c->capture) HIPCHECK(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
        const int cur0 = c->cur;
        const int64_t steps0 = c->steps;
        const bool ok0 = c->ghosts_ok, changed0 = c->face_changed;
        // every replay must begin like the recorded one: with walls each step
        // refreshes the ghosts, so the chunk records that refresh from its
        // first step on (a repeat of a settled fill writes the same values)
        if (walls) c->ghosts_ok = false;
        hipStream_t own = c->stream;
        HIPCHECK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
        c->stream = c->capture;
        rc = f(c, K);
        c->stream = own;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->capture, &g);
        c->cur = cur0;   // capturing launched nothing
        c->steps = steps0;
        if (rc || e != hipSuccess) {
            c->ghosts_ok = ok0;
            c->face_changed = changed0;
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : fail(c, PGK_EDEVICE, std::string("step capture: ") + hipGetErrorString(e));
        }
        hipError_t ei = hipGraphInstantiate(&c->graph[p], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            c->ghosts_ok = ok0;
            c->face_changed = changed0;
            c->graph[p] = nullptr;
            return fail(c, PGK_EDEVICE, std::string("step graph: ") + hipGetErrorString(ei));
        }
    }
    for (int64_t i = 0; i + K <= n; i += K) HIPCHECK(c, hipGraphLaunch(c->graph[p], c->stream));
    c->steps += n / K * K;
    // after a chunk: a wall's ghosts wait for the last collision, Dirichlet
    // ghosts hold the face states
    if (bounded(c)) c->ghosts_ok = !walls;
    c->face_changed = false;
    return (n % K) ? f(c, n % K) : PGK_OK;
}

template <typename S, bool REDUCE>
static int moments_t(pgk_ctx *c, double *rho, double *u, double *thT, double *thR, double *P)
{
    dim3 grid(c->nblk), block(WG);
    const S *src = (const S *)c->buf[c->cur];
    // ghosts for the current pull
    int rc0 = settle_ghosts(c);
    if (rc0) return rc0;
    if (bounded(c))
        hipLaunchKernelGGL((k_moments<S, BND_XY, REDUCE>), grid, block, 0, c->stream, src, (const S *)c->gh,
                           (const double *)c->buf[PGK_BUF_THETAR], rho, u, thT, thR, P, c->partial, c->k);
    else
        hipLaunchKernelGGL((k_moments<S, BND_NONE, REDUCE>), grid, block, 0, c->stream, src, (const S *)c->gh,
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

extern "C" int pgk_set_graph_steps(pgk_ctx *c, int k)
{
    if (!c) return PGK_EINVAL;
    if (k < 0 || (k & 1) || k > 4096) return fail(c, PGK_EINVAL, "graph steps must be 0 or even and at most 4096");
    if (k != c->graph_steps) c->drop_graphs();
    c->graph_steps = k;
    return PGK_OK;
}

extern "C" int pgk_set_transport_reference(pgk_ctx *c, int on)
{
    if (!c) return PGK_EINVAL;
    if ((on != 0) != c->transport_ref) c->drop_graphs();
    c->transport_ref = on != 0;
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

extern "C" int pgk_get_clock(const pgk_ctx *c, pgk_clock *out)
{
    if (!c || !out) return PGK_EINVAL;
    if (!c->initialised) return PGK_EINVAL;
    out->steps = c->steps;
    out->cur = c->cur;
    out->ghosts_ok = c->ghosts_ok ? 1 : 0;
    out->face_changed = c->face_changed ? 1 : 0;
    return PGK_OK;
}

extern "C" int pgk_set_clock(pgk_ctx *c, const pgk_clock *in)
{
    if (!c || !in) return PGK_EINVAL;
    if (!c->bound) return fail(c, PGK_ENOTBOUND, "buffers not bound");
    if (!c->params_set) return fail(c, PGK_EINVAL, "parameters not set");
    if (int rcf = faces_set(c)) return rcf;
    if (in->steps < 0 || (in->cur != 0 && in->cur != 1)) return fail(c, PGK_EINVAL, "bad clock");
    c->steps = in->steps;
    c->cur = in->cur;
    c->ghosts_ok = in->ghosts_ok != 0;
    c->face_changed = in->face_changed != 0;
    c->initialised = true;
    return PGK_OK;
}

extern "C" const char *pgk_last_error(const pgk_ctx *c) { return c ? c->err.c_str() : "null context"; }

extern "C" void pgk_destroy(pgk_ctx *c) { delete c; }
