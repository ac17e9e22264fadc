// batch.hip -- batched sweep of independent 1D cases in one persistent launch.
//
// Each work-group owns one case (a line of L cells, 2L sites, x faces bounded)
// and advances it K steps: ghost fill, fused pull-collide, MacCormack and
// diffusion of theta_R, separated by work-group barriers.  At the last two
// steps of a chunk it takes the f-moments, so the one-step change of rho,
// u_axis, theta_T and theta_R gives the residual; a case whose residual falls
// to the tolerance, or whose density or temperature turns non-positive or
// non-finite, freezes itself.  The host replays one HIP graph per chunk and
// reads back only the small per-case status arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <sys/stat.h>
#include <unistd.h>
#include <vector>

#include "device.hpp"

namespace pgk {

struct BatchCase {
    Consts k;
    long long off;      // first site of the case
    int vel_axis, variant, eq;
};

struct BatchArgs {
    const BatchCase *cases;
    const int *order;   // slot -> case, longest first
    int *status;
    long long *steps;
    int *cur;
    double *resid;
    double *popA, *popB, *thR, *that_, *tmc, *tmc2, *aux, *snap, *gh;
    double *lmul;       // [2 E2_NL][2L] per case: E2 multipliers of the last step (E2 batches only)
    long long max_steps;
    double tol;
    int lds_sites;      // cases with ns <= lds_sites diffuse theta_R in LDS
    int chain_sites;    // cases with ns <= chain_sites may keep their conductances in the dynamic LDS
};

// dynamic LDS of k_batch: theta ping-pong and the two face coefficients
constexpr int LDS_ARRAYS = 4;
constexpr int LDS_SITES_MAX = 2048;   // 64 KiB
constexpr int CHAIN_SITES_MAX = 8192; // 128 KiB of conductances (two per site)

constexpr int GHOSTS_PER_CASE = 2 * NQ * NSLOT;   // ny = nz = 1

template <int NV, int NTH>
__device__ __forceinline__ void block_sum_n(double *val)
{
    // sum over the work-group; every thread gets the result
    __shared__ double red[NTH / 64][NV];
    for (int off = 32; off > 0; off >>= 1)
        for (int c = 0; c < NV; c++) val[c] += __shfl_xor(val[c], off, 64);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int c = 0; c < NV; c++) red[wv][c] = val[c];
    __syncthreads();
    for (int c = 0; c < NV; c++) {
        double t = 0.0;
        for (int i = 0; i < NTH / 64; i++) t += red[i][c];
        val[c] = t;
    }
    __syncthreads();
}

// FTCS diffusion of a line (ny = nz = 1) in LDS.  The y and z neighbours of
// a line are the site itself and contribute nothing, so the stencil is the
// x pair: with the face conductances fixed within a step, one sub-step is
//   CN:  t + c- (t[x-1] - t) + c+ (t[x+1] - t),  c+- = 2 (k_s + k_x+-1) / (2 rho delta nsub)
//   LIT: the same with c+- = 2 k_s / (rho delta nsub)
// (k = kfac rho theta_hat; a bounded face contributes its ghost value theta_w
// with the ghost conductance of dif_site).  Site s = sub * nx + x.
template <int VAR>
__device__ __forceinline__ void dif_line_coef(int s, const double *__restrict__ aux, const Consts &k, double &cm,
                                              double &cp)
{
    const int ns = k.ns, sub = s >= k.nx, x = s - sub * k.nx;
    const double rho = aux[(size_t)3 * ns + s], ks = k.kfac * aux[(size_t)4 * ns + s];
    const double fac = k.isub * 2.0 / (rho * k.delta);
    double c[2];
#pragma unroll
    for (int d = 0; d < 2; d++) {
        int xq = x + (d ? 1 : -1);
        int side = xq < 0 ? 0 : (xq >= k.nx ? 1 : -1);
        double kq;
        if (side >= 0 && k.bc[side] != PGK_PERIODIC) {
            double rg = k.bc[side] == PGK_WALL ? rho : k.rhobc[side];
            kq = k.kfac * rg * k.thbc[side];
        } else {
            kq = k.kfac * aux[(size_t)4 * ns + sub * k.nx + wrapc(xq, k.nx)];
        }
        c[d] = VAR == PGK_CN ? fac * 0.5 * (ks + kq) : fac * ks;
    }
    cm = c[0];
    cp = c[1];
}

// one FTCS sub-step of a cell, with its fused multiply-adds written out so
// that every diffusion path of the batched kernel (registers, LDS, global
// memory) gives the same bits whatever the launch shape picks
__device__ __forceinline__ double ftcs(double t, double tm, double tp, double cm, double cp)
{
    return fma(cp, tp - t, fma(cm, tm - t, t));
}

__device__ __forceinline__ double dif_line(int s, const double *tin, const double *cm, const double *cp,
                                           const Consts &k)
{
    const int sub = s >= k.nx, x = s - sub * k.nx;
    const double t = tin[s];
    double tm, tp;
    if (x > 0) tm = tin[s - 1];
    else tm = k.bc[0] != PGK_PERIODIC ? k.thbc[0] : tin[s + k.nx - 1];
    if (x + 1 < k.nx) tp = tin[s + 1];
    else tp = k.bc[1] != PGK_PERIODIC ? k.thbc[1] : tin[s + 1 - k.nx];
    return ftcs(t, tm, tp, cm[s], cp[s]);
}

// The same sub-step with the line in global memory (lines too long for LDS):
// the conductances of dif_line_coef recomputed from aux at every sub-step
template <int VAR>
__device__ __forceinline__ double dif_line_global(int s, const double *__restrict__ tin,
                                                  const double *__restrict__ aux, const Consts &k)
{
    double cm, cp;
    dif_line_coef<VAR>(s, aux, k, cm, cp);
    const int sub = s >= k.nx, x = s - sub * k.nx;
    const double t = tin[s];
    const double tm = x > 0 ? tin[s - 1] : k.thbc[0];   // bounded faces (every batched case)
    const double tp = x + 1 < k.nx ? tin[s + 1] : k.thbc[1];
    return ftcs(t, tm, tp, cm, cp);
}

// The same sub-steps with the line in registers: wavefront `sub` holds the
// sites of one sublattice chain, lane l the sites x = l + 64 j (j < DW_P), so
// that the neighbours x -+ 1 come from lanes l -+ 1 (lane 63 / 0 of the next
// j across the seam) by cross-lane moves, with no barrier between sub-steps.
// Bounded faces only (both faces bounded, as every batched case is); the
// arithmetic is that of dif_line.
constexpr int DW_P = 8;   // lines of up to 512 cells

// whole-wavefront rotations by one lane (DPP wave_ror:1 / wave_rol:1): lane i
// receives the value of lane i - 1 / i + 1, modulo 64
__device__ __forceinline__ double lane_prev(double v)
{
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x13C, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x13C, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double lane_next(double v)
{
    int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x134, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x134, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// value of lane `l` of v in every lane
__device__ __forceinline__ double lane_bcast(double v, int l)
{
    int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

template <int VAR>
__device__ __forceinline__ void dif_chain(int sub, const double *__restrict__ tmc, const double *__restrict__ aux,
                                          const double *__restrict__ that_, double *__restrict__ thR, const Consts &k)
{
    const int lane = threadIdx.x & 63, L = k.nx;
    double t[DW_P], cm[DW_P], cp[DW_P];
#pragma unroll
    for (int j = 0; j < DW_P; j++) {
        int x = lane + 64 * j;
        t[j] = cm[j] = cp[j] = 0.0;
        if (x < L) {
            int s = sub * L + x;
            t[j] = tmc[s];
            dif_line_coef<VAR>(s, aux, k, cm[j], cp[j]);
        }
    }
    for (int it = 0; it < k.nsub; it++) {
        double tn[DW_P];
#pragma unroll
        for (int j = 0; j < DW_P; j++) {
            double a = lane_prev(t[j]);                                          // x - 1, lanes 1..63
            double b = j > 0 ? lane_bcast(t[j - 1], 63) : k.thbc[0];             // x - 1, lane 0
            double c = lane_next(t[j]);                                          // x + 1, lanes 0..62
            double d = j + 1 < DW_P ? lane_bcast(t[j + 1], 0) : 0.0;             // x + 1, lane 63
            double tm = lane == 0 ? b : a, tp = lane == 63 ? d : c;
            if (lane + 64 * j == L - 1) tp = k.thbc[1];
            tn[j] = ftcs(t[j], tm, tp, cm[j], cp[j]);
        }
#pragma unroll
        for (int j = 0; j < DW_P; j++) t[j] = tn[j];
    }
#pragma unroll
    for (int j = 0; j < DW_P; j++) {
        int x = lane + 64 * j;
        if (x < L) {
            int s = sub * L + x;
            double v = thR[s];
            if (VAR == PGK_CN) thR[s] = t[j] + (that_[s] - v);
            else thR[s] = (t[j] + k.X * v) * k.inv1X;
        }
    }
}

// The same sub-steps for longer lines on every wavefront of the work-group:
// W = NTH / 128 wavefronts per sublattice, wavefront w of a sublattice holding
// the segment x in [w S, (w + 1) S), S = 64 P, lane l the cells
// x = w S + l + 64 j (j < P).  Inside a segment the neighbours come by
// cross-lane moves as in dif_chain; the cells on either side of a segment come
// from the neighbouring wavefronts through LDS (each publishes its first and
// last cell), with one barrier per sub-step (double-buffered slots: a
// wavefront writes the other slot next sub-step, and cannot write this one
// again before every wavefront has passed the next barrier).  LDSC: the two
// conductances of each cell live in cl ([2][ns], each read only by the thread
// that wrote it) instead of registers, which leaves room for P = 16.  Every
// thread of the work-group must call it.  Bounded faces only; the arithmetic
// is that of dif_line.
constexpr int DQ_P = 8;    // cells per lane with the conductances in registers: lines of up to 512 W cells
// with the conductances in LDS, only with 256 threads (the 512-thread kernel
// has no registers to spare): 32 cells per lane, lines of up to 4096 cells
constexpr int DQL_P = 32;

template <int VAR, int NTH, int P, bool LDSC>
__device__ __forceinline__ void dif_wchain(const double *__restrict__ tmc, const double *__restrict__ aux,
                                           const double *__restrict__ that_, double *__restrict__ thR,
                                           const Consts &k, double *xch, double *cl)
{
    constexpr int W = NTH / 128;
    constexpr int S = 64 * P;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = wave / W, w = wave - sub * W, x0 = w * S, L = k.nx;
    double t[P], cmr[LDSC ? 1 : P], cpr[LDSC ? 1 : P];
#pragma unroll
    for (int j = 0; j < P; j++) {
        const int x = x0 + lane + 64 * j;
        t[j] = 0.0;
        if constexpr (!LDSC) cmr[j] = cpr[j] = 0.0;
        if (x < L) {
            const int s = sub * L + x;
            double cm, cp;
            t[j] = tmc[s];
            dif_line_coef<VAR>(s, aux, k, cm, cp);
            if constexpr (LDSC) {
                cl[s] = cm;
                cl[k.ns + s] = cp;
            } else {
                cmr[j] = cm;
                cpr[j] = cp;
            }
        }
    }
    // xch: [parity][sublattice][wavefront][first, last]
    auto slot = [&](int par, int ww, int end) { return ((par * 2 + sub) * W + ww) * 2 + end; };
    for (int it = 0; it < k.nsub; it++) {
        const int par = it & 1;
        if (lane == 0) xch[slot(par, w, 0)] = t[0];
        if (lane == 63) xch[slot(par, w, 1)] = t[P - 1];
        __syncthreads();
        const double right = w + 1 < W ? xch[slot(par, w + 1, 0)] : 0.0;     // cell x0 + S
        // in place, j ascending: slot j + 1 still holds the old values, and the
        // old lane-63 value of slot j - 1 is carried (cell x0 - 1 for j = 0)
        double carry = w > 0 ? xch[slot(par, w - 1, 1)] : k.thbc[0];
#pragma unroll
        for (int j = 0; j < P; j++) {
            const double old = t[j];
            double a = lane_prev(old);                                        // x - 1, lanes 1..63
            double c = lane_next(old);                                        // x + 1, lanes 0..62
            double d = j + 1 < P ? lane_bcast(t[j + 1], 0) : right;           // x + 1, lane 63
            double tm = lane == 0 ? carry : a, tp = lane == 63 ? d : c;
            carry = lane_bcast(old, 63);
            const int x = x0 + lane + 64 * j;
            if (x == L - 1) tp = k.thbc[1];
            double cm, cp;
            if constexpr (LDSC) {
                const bool in = x < L;
                const int s = sub * L + (in ? x : 0);
                cm = in ? cl[s] : 0.0;
                cp = in ? cl[k.ns + s] : 0.0;
            } else {
                cm = cmr[j];
                cp = cpr[j];
            }
            t[j] = ftcs(old, tm, tp, cm, cp);
        }
    }
#pragma unroll
    for (int j = 0; j < P; j++) {
        const int x = x0 + lane + 64 * j;
        if (x < L) {
            const int s = sub * L + x;
            const double v = thR[s];
            if (VAR == PGK_CN) thR[s] = t[j] + (that_[s] - v);
            else thR[s] = (t[j] + k.X * v) * k.inv1X;
        }
    }
}

// Ghost populations of both x faces of a line (ny = nz = 1), wavefront w
// taking face w: the same quantities as bc_column, with the outgoing-mass sum
// of a diffuse wall spread over the 64 lanes (lane l takes the candidates
// (q, sub, xi) numbered l, l + 64, l + 128) and a butterfly reduction.  The
// caller synchronises the work-group before the ghosts are read.
__device__ __forceinline__ void bc_line(const double *__restrict__ src, double *__restrict__ gh, const Consts &k)
{
    const int side = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (side > 1 || k.bc[side] == PGK_PERIODIC) return;
    double scale = 1.0;
    if (k.bc[side] == PGK_WALL) {
        double out = 0.0;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            int idx = lane + 64 * j;                 // 160 candidates: q = 1..40, sub, xi
            if (idx >= 4 * (NQ - 1)) break;
            int q = 1 + (idx >> 2), sub = (idx >> 1) & 1, xi = idx & 1;
            int cx = c2(q, 0);
            if ((side == 0 && cx >= 0) || (side == 1 && cx <= 0)) continue;
            if (xi == 1 && k.nx == 1) continue;
            int x = side == 0 ? xi : k.nx - 1 - xi;
            int dx = 2 * x + sub + cx;
            bool crosses = side == 0 ? dx < 0 : dx > 2 * k.nx - 1;
            if (crosses) out += src[(size_t)q * k.ns + sub * k.nx + x];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) out += __shfl_xor(out, o, 64);
        scale = out / k.in_col[side];
    }
    if (lane < NQ) {
        double val = scale * k.Fbc[side][lane];
#pragma unroll
        for (int slot = 0; slot < NSLOT; slot++) gh[(side * NQ + lane) * NSLOT + slot] = val;
    }
}

template <int VAR, int NTH, bool E2CAP>
__global__ __launch_bounds__(NTH) void k_batch(BatchArgs a, int K)
{
    __shared__ double xch[2 * 2 * (NTH / 128) * 2];   // segment ends of the diffusion chains
    const int c = a.order[blockIdx.x];
    if (a.status[c] != PGK_CASE_RUNNING) return;
    const BatchCase &bc = a.cases[c];
    const Consts &k = bc.k;
    const long long off = bc.off;
    double *pA = a.popA + (size_t)NQ * off, *pB = a.popB + (size_t)NQ * off;
    double *thR = a.thR + off, *that_ = a.that_ + off, *tmc = a.tmc + off, *tmc2 = a.tmc2 + off;
    double *aux = a.aux + (size_t)5 * off, *snap = a.snap + (size_t)4 * off;
    double *gh = a.gh + (size_t)c * GHOSTS_PER_CASE;
    const int ns = k.ns, tid = threadIdx.x;
    int cur = a.cur[c];
    long long steps = a.steps[c];
    double resid = a.resid[c];
    bool bad = false;

    for (int j = 0; j < K; j++) {
        const double *src = cur ? pB : pA;
        double *dst = cur ? pA : pB;
        if (steps > 0) bc_line(src, gh, k);
        __syncthreads();
        if (E2CAP && bc.eq == PGK_E2) {
            double *lm = a.lmul + (size_t)2 * E2_NL * off;
            for (int s = tid; s < ns; s += NTH) {
                double r;
                lb_site<double, double, VAR, BND_X, PGK_E2>(s, src, dst, gh, thR, that_, aux, k, r, lm);
            }
        } else {
            for (int s = tid; s < ns; s += NTH) {
                double r;
                lb_site<double, double, VAR, BND_X, PGK_F3>(s, src, dst, gh, thR, that_, aux, k, r);
            }
        }
        __syncthreads();
        for (int s = tid; s < ns; s += NTH) mc_site<double, BND_X>(s, that_, aux, tmc, k);
        __syncthreads();
        if (NTH == 512 && k.nx <= (NTH / 128) * 64 * 2) {
            // short lines on every wavefront (two cells per lane): faster than two
            // wavefronts alone with 512 threads, slower with 256
            if constexpr (NTH == 512) dif_wchain<VAR, NTH, 2, false>(tmc, aux, that_, thR, k, xch, nullptr);
        } else if (k.nx <= 64 * DW_P) {
            if (tid < 128) dif_chain<VAR>(tid >> 6, tmc, aux, that_, thR, k);
        } else if (k.nx <= (NTH / 128) * 64 * DQ_P && (NTH == 256 || ns > a.lds_sites)) {
            // (with 512 threads the LDS path below is the faster one where it fits)
            dif_wchain<VAR, NTH, DQ_P, false>(tmc, aux, that_, thR, k, xch, nullptr);
        } else if (NTH == 256 && ns > a.lds_sites && k.nx <= (NTH / 128) * 64 * DQL_P && ns <= a.chain_sites) {
            if constexpr (NTH == 256) {
                extern __shared__ double lds[];
                dif_wchain<VAR, NTH, DQL_P, true>(tmc, aux, that_, thR, k, xch, lds);
            }
        } else if (ns <= a.lds_sites) {
            extern __shared__ double lds[];
            double *tin = lds, *tout = lds + a.lds_sites, *cm = lds + 2 * a.lds_sites, *cp = lds + 3 * a.lds_sites;
            for (int s = tid; s < ns; s += NTH) {
                tin[s] = tmc[s];
                dif_line_coef<VAR>(s, aux, k, cm[s], cp[s]);
            }
            __syncthreads();
            for (int it = 0; it + 1 < k.nsub; it++) {
                for (int s = tid; s < ns; s += NTH) tout[s] = dif_line(s, tin, cm, cp, k);
                __syncthreads();
                double *t = tin;
                tin = tout;
                tout = t;
            }
            for (int s = tid; s < ns; s += NTH) {
                double tdif = dif_line(s, tin, cm, cp, k), v = thR[s];
                if (VAR == PGK_CN) thR[s] = tdif + (that_[s] - v);
                else thR[s] = (tdif + k.X * v) * k.inv1X;
            }
        } else {
            double *tin = tmc, *tout = tmc2;
            for (int it = 0; it + 1 < k.nsub; it++) {
                for (int s = tid; s < ns; s += NTH) tout[s] = dif_line_global<VAR>(s, tin, aux, k);
                __syncthreads();
                double *t = tin;
                tin = tout;
                tout = t;
            }
            for (int s = tid; s < ns; s += NTH) {
                double tdif = dif_line_global<VAR>(s, tin, aux, k), v = thR[s];
                if (VAR == PGK_CN) thR[s] = tdif + (that_[s] - v);
                else thR[s] = (tdif + k.X * v) * k.inv1X;
            }
        }
        __syncthreads();
        cur ^= 1;
        steps++;
        if (j >= K - 2) {
            // moments of the new state: refresh the ghosts it pulls from
            const double *nsrc = cur ? pB : pA;
            bc_line(nsrc, gh, k);
            __syncthreads();
            double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int s = tid; s < ns; s += NTH) {
                Mom m;
                Solve so = moments_site<double, BND_X>(s, nsrc, gh, thR, k, m);
                double ua = bc.vel_axis == 0 ? so.u[0] : (bc.vel_axis == 1 ? so.u[1] : so.u[2]);
                double phi[4] = {so.rho, ua, so.T, so.r};
                if (!(so.rho > 0.0) || !(so.T > 0.0) || !(so.r > 0.0) || !isfinite(so.u[0]) ||
                    !isfinite(so.u[1]) || !isfinite(so.u[2]))
                    acc[8] = 1.0;
                if (j == K - 2) {
                    for (int i = 0; i < 4; i++) snap[(size_t)i * ns + s] = phi[i];
                } else {
                    for (int i = 0; i < 4; i++) {
                        double d = phi[i] - snap[(size_t)i * ns + s];
                        acc[i] += d * d;
                        acc[4 + i] += phi[i] * phi[i];
                    }
                }
            }
            block_sum_n<9, NTH>(acc);
            if (acc[8] > 0.0) bad = true;
            if (j == K - 1) {
                resid = 0.0;
                for (int i = 0; i < 4; i++) resid = fmax(resid, sqrt(acc[i] / fmax(acc[4 + i], 1e-300)));
            }
        }
    }
    if (tid == 0) {
        a.cur[c] = cur;
        a.steps[c] = steps;
        a.resid[c] = resid;
        int st = PGK_CASE_RUNNING;
        if (bad || !isfinite(resid)) st = PGK_CASE_DIVERGED;
        else if (resid <= a.tol) st = PGK_CASE_CONVERGED;
        else if (steps >= a.max_steps) st = PGK_CASE_MAXSTEPS;
        a.status[c] = st;
    }
}

template <int NTH>
__global__ __launch_bounds__(NTH) void k_batch_init(BatchArgs a, const double *__restrict__ rho,
                                                    const double *__restrict__ u, const double *__restrict__ thT,
                                                    const double *__restrict__ thRin, long long ns_total)
{
    const int c = blockIdx.x;
    const BatchCase &bc = a.cases[c];
    const Consts &k = bc.k;
    const long long off = bc.off;
    double *dst = a.popA + (size_t)NQ * off;
    double *gh = a.gh + (size_t)c * GHOSTS_PER_CASE;
    // the case's slices of the input fields; u is [3][ns_total]
    if (bc.eq == PGK_E2) {
        // no previous multipliers: the first step starts Newton from the Gaussian
        double *lm = a.lmul + (size_t)2 * E2_NL * off;
        for (long long i = threadIdx.x; i < (long long)2 * E2_NL * k.ns; i += NTH) lm[i] = __builtin_nan("");
    }
    for (int s = threadIdx.x; s < k.ns; s += NTH) {
        if (bc.eq == PGK_E2)
            init_site<double, BND_X, PGK_E2>(s, dst, gh, a.thR + off, rho + off, u + off, thT + off, thRin + off, k,
                                            (size_t)ns_total);
        else
            init_site<double, BND_X, PGK_F3>(s, dst, gh, a.thR + off, rho + off, u + off, thT + off, thRin + off, k,
                                            (size_t)ns_total);
    }
    if (threadIdx.x == 0) {
        a.status[c] = PGK_CASE_RUNNING;
        a.steps[c] = 0;
        a.cur[c] = 0;
        a.resid[c] = 1.0;
    }
}

template <int NTH>
__global__ __launch_bounds__(NTH) void k_batch_moments(BatchArgs a, double *__restrict__ orho,
                                                       double *__restrict__ ou, double *__restrict__ othT,
                                                       double *__restrict__ othR, long long ns_total)
{
    const int c = blockIdx.x;
    const BatchCase &bc = a.cases[c];
    const Consts &k = bc.k;
    const long long off = bc.off;
    const double *src = (a.cur[c] ? a.popB : a.popA) + (size_t)NQ * off;
    double *gh = a.gh + (size_t)c * GHOSTS_PER_CASE;
    if (a.steps[c] > 0) bc_line(src, gh, k);
    __syncthreads();
    for (int s = threadIdx.x; s < k.ns; s += NTH) {
        Mom m;
        Solve so = moments_site<double, BND_X>(s, src, gh, a.thR + off, k, m);
        if (orho) orho[off + s] = so.rho;
        if (ou)
            for (int i = 0; i < 3; i++) ou[i * ns_total + off + s] = so.u[i];
        if (othT) othT[off + s] = so.T;
        if (othR) othR[off + s] = so.r;
    }
}

}  // namespace pgk

using namespace pgk;

struct pgk_batch {
    int n = 0;
    long long ns_total = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<BatchCase> host_cases;
    std::vector<long long> off;
    BatchArgs args{};
    bool has_e2 = false;          // some case uses E2: the E2-capable kernel, work-groups of 256
    long long stall_window = 0;   // steps without halving the best residual before STALLED (0: off)
    // stall bookkeeping per case, kept across pgk_batch_run calls (reset by pgk_batch_init):
    // the best residual so far and the steps since it last halved
    std::vector<double> best;
    std::vector<long long> since;
    int wg = 0, K = 0;            // fixed config (0 = tune)
    int tuned_wg = 0, tuned_K = 0;
    double tuned_ns = 0.0;
    std::map<long long, hipGraphExec_t> graphs;   // key wg*100000 + K
    int *h_status = nullptr;
    long long *h_steps = nullptr;
    double *h_resid = nullptr;
    std::string err;
    ~pgk_batch()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.second);
        if (h_status) (void)hipHostFree(h_status);
        if (h_steps) (void)hipHostFree(h_steps);
        if (h_resid) (void)hipHostFree(h_resid);
        if (own_stream) (void)hipStreamDestroy(stream);
    }
};

static int bfail(pgk_batch *b, int code, const std::string &m)
{
    if (b) b->err = m;
    return code;
}

#define BHIP(b, call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) return bfail(b, PGK_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    size_t cases, order, status, steps, cur, resid, popA, popB, thR, that_, tmc, tmc2, aux, snap, gh, lmul, total;
};

static BatchLayout layout(int n, long long ns, bool e2)
{
    BatchLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += al256(bytes); return at; };
    L.cases = take(sizeof(BatchCase) * n);
    L.order = take(sizeof(int) * n);
    L.status = take(sizeof(int) * n);
    L.steps = take(sizeof(long long) * n);
    L.cur = take(sizeof(int) * n);
    L.resid = take(sizeof(double) * n);
    L.popA = take(8ull * NQ * ns);
    L.popB = take(8ull * NQ * ns);
    L.thR = take(8ull * ns);
    L.that_ = take(8ull * ns);
    L.tmc = take(8ull * ns);
    L.tmc2 = take(8ull * ns);
    L.aux = take(8ull * 5 * ns);
    L.snap = take(8ull * 4 * ns);
    L.gh = take(8ull * GHOSTS_PER_CASE * n);
    L.lmul = e2 ? take(8ull * 2 * E2_NL * ns) : 0;
    L.total = o;
    return L;
}

static bool case_ok(const pgk_case &c)
{
    if (c.L < 4 || c.L > 8192) return false;
    if (c.bc != PGK_WALL && c.bc != PGK_DIRICHLET) return false;
    if (c.vel_axis < 0 || c.vel_axis > 2) return false;
    if (c.variant != PGK_CN && c.variant != PGK_LIT) return false;
    if (c.equilibrium != PGK_F3 && c.equilibrium != PGK_E2) return false;
    const pgk_params &p = c.p;
    if (!(p.tau > 0) || !(p.tau1 > 0) || !(p.delta > 0) || p.b < -0.5 || p.b > 1.0 || !(p.kr >= 0)) return false;
    for (int s = 0; s < 2; s++) {
        if (!(c.theta[s] > 0)) return false;
        if (c.bc == PGK_DIRICHLET && !(c.rho[s] > 0)) return false;
        if (c.bc == PGK_WALL && c.u[s][0] != 0.0) return false;
    }
    return true;
}

extern "C" int pgk_batch_bytes(const pgk_case *cases, int n, size_t *bytes)
{
    if (!cases || n <= 0 || !bytes) return PGK_EINVAL;
    long long ns = 0;
    bool e2 = false;
    for (int i = 0; i < n; i++) {
        if (!case_ok(cases[i])) return PGK_EINVAL;
        ns += 2LL * cases[i].L;
        e2 = e2 || cases[i].equilibrium == PGK_E2;
    }
    *bytes = layout(n, ns, e2).total;
    return PGK_OK;
}

// model constants of one case, as pgk_set_params derives them for a grid;
// false when a Dirichlet face state has no E2 equilibrium
static bool case_consts(const pgk_case &cs, Consts &k)
{
    k = Consts{};
    k.nx = cs.L; k.ny = 1; k.nz = 1; k.ns = 2 * cs.L;
    k.bc[0] = k.bc[1] = cs.bc;
    magic_div((unsigned)k.nx, k.mx, k.shx);
    magic_div(1u, k.my, k.shy);
    magic_div(1u, k.mz, k.shz);
    const pgk_params &p = cs.p;
    k.th0 = p.theta0 > 0 ? p.theta0 : THETA0_PRINTED;
    shell_weights(k.th0, k.w);
    for (int i = 0; i < 6; i++) {
        k.whi[i] = (float)k.w[i];
        k.wlo[i] = (float)(k.w[i] - (double)k.whi[i]);
    }
    k.tau = p.tau; k.tau1 = p.tau1; k.b = p.b; k.delta = p.delta;
    double taus = p.tau * p.tau1 / (p.tau + p.tau1), B = 1.0 + p.tau / p.tau1;
    k.beta = 1.0 / (2.0 * taus + 1.0);
    k.X = 3.0 / (2.0 * p.tau1 * (3.0 + p.delta));
    k.Y = p.delta / (2.0 * p.tau1 * (3.0 + p.delta));
    k.ssig = 1.0 + 1.0 / (2.0 * taus) - p.b / (2.0 * p.tau);
    k.kfac = p.kr * 5.0 * p.tau / (2.0 * B);
    k.inv1X = 1.0 / (1.0 + k.X);
    k.inv1XY = 1.0 / (1.0 + k.X + k.Y);
    k.inv3d = 1.0 / (3.0 + p.delta);
    k.wt1 = p.tau1 / (p.tau + p.tau1);
    k.wt = p.tau / (p.tau + p.tau1);
    k.bs = p.b / k.ssig;
    double t = k.th0;
    k.it = 1.0 / t; k.i2t = 1.0 / (2.0 * t); k.ih2 = 1.0 / (2.0 * t * t);
    k.i6t3 = 1.0 / (6.0 * t * t * t); k.i2t3 = 1.0 / (2.0 * t * t * t); k.it2 = 1.0 / (t * t);
    for (int side = 0; side < 2; side++) {
        k.thbc[side] = cs.theta[side];
        k.rhobc[side] = cs.bc == PGK_WALL ? 1.0 : cs.rho[side];
        if (cs.bc == PGK_DIRICHLET && cs.equilibrium == PGK_E2) {
            double th = k.thbc[side], lam[6] = {th, th, th, 0.0, 0.0, 0.0}, l[E2_NL];
            if (e2_solve(k.th0, k.w, k.rhobc[side], cs.u[side], lam, l) < 0) return false;
            for (int q = 0; q < NQ; q++) k.Fbc[side][q] = e2_population(l, k.w, q);
        } else {
            f3_host(k.th0, k.w, k.rhobc[side], cs.u[side], k.thbc[side], k.Fbc[side]);
        }
        double in = 0.0;
        for (int q = 0; q < NQ; q++)
            for (int sub = 0; sub < 2; sub++)
                for (int x = 0; x < k.nx; x++) {
                    int qx = 2 * x + sub - c2(q, 0);
                    if (side == 0 ? qx < 0 : qx > 2 * k.nx - 1) in += k.Fbc[side][q];
                }
        k.in_col[side] = in;
    }
    k.nsub = diffusion_substeps(k, p.kr);
    k.isub = 1.0 / k.nsub;
    return true;
}

extern "C" int pgk_batch_create(const pgk_case *cases, int n, void *stream, void *buf, size_t bytes, pgk_batch **out)
{
    if (!out) return PGK_EINVAL;
    *out = nullptr;
    size_t need;
    int rc = pgk_batch_bytes(cases, n, &need);
    if (rc) return rc;
    if (!buf || bytes < need || ((uintptr_t)buf & 255)) return PGK_EINVAL;
    pgk_batch *b = new pgk_batch();
    b->n = n;
    b->stream = (hipStream_t)stream;
    if (!b->stream) {
        // graph capture needs a stream other than the null stream
        if (hipStreamCreate(&b->stream) != hipSuccess) { delete b; return PGK_EDEVICE; }
        b->own_stream = true;
    }
    long long o = 0;
    b->off.resize(n + 1);
    for (int i = 0; i < n; i++) {
        BatchCase bc{};
        if (!case_consts(cases[i], bc.k)) {
            delete b;
            return PGK_EINFEASIBLE;
        }
        bc.off = o;
        bc.vel_axis = cases[i].vel_axis;
        bc.variant = cases[i].variant;
        bc.eq = cases[i].equilibrium;
        if (bc.eq == PGK_E2) b->has_e2 = true;
        b->host_cases.push_back(bc);
        b->off[i] = o;
        o += 2LL * cases[i].L;
    }
    b->off[n] = o;
    b->ns_total = o;
    BatchLayout L = layout(n, o, b->has_e2);
    char *base = (char *)buf;
    BatchArgs &a = b->args;
    a.cases = (const BatchCase *)(base + L.cases);
    a.order = (const int *)(base + L.order);
    a.status = (int *)(base + L.status);
    a.steps = (long long *)(base + L.steps);
    a.cur = (int *)(base + L.cur);
    a.resid = (double *)(base + L.resid);
    a.popA = (double *)(base + L.popA);
    a.popB = (double *)(base + L.popB);
    a.thR = (double *)(base + L.thR);
    a.that_ = (double *)(base + L.that_);
    a.tmc = (double *)(base + L.tmc);
    a.tmc2 = (double *)(base + L.tmc2);
    a.aux = (double *)(base + L.aux);
    a.snap = (double *)(base + L.snap);
    a.gh = (double *)(base + L.gh);
    a.lmul = b->has_e2 ? (double *)(base + L.lmul) : nullptr;
    long long maxns = 0;
    for (auto &c : b->host_cases) maxns = std::max<long long>(maxns, c.k.ns);
    a.lds_sites = (int)std::min<long long>(maxns, LDS_SITES_MAX);
    a.chain_sites = (int)std::min<long long>(maxns, CHAIN_SITES_MAX);
    // slots ordered by size, longest first (the cost model: work per step)
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cases[x].L > cases[y].L; });
    hipError_t e1 = hipMemcpyAsync((void *)a.cases, b->host_cases.data(), sizeof(BatchCase) * n,
                                   hipMemcpyHostToDevice, b->stream);
    hipError_t e2 = hipMemcpyAsync((void *)a.order, order.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream);
    hipError_t e3 = hipStreamSynchronize(b->stream);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) { delete b; return PGK_EDEVICE; }
    if (hipHostMalloc((void **)&b->h_status, sizeof(int) * n) != hipSuccess ||
        hipHostMalloc((void **)&b->h_steps, sizeof(long long) * n) != hipSuccess ||
        hipHostMalloc((void **)&b->h_resid, sizeof(double) * n) != hipSuccess) {
        delete b;
        return PGK_EDEVICE;
    }
    *out = b;
    return PGK_OK;
}

extern "C" int pgk_batch_offsets(const pgk_batch *b, int64_t *off)
{
    if (!b || !off) return PGK_EINVAL;
    for (int i = 0; i <= b->n; i++) off[i] = b->off[i];
    return PGK_OK;
}

extern "C" int pgk_batch_init(pgk_batch *b, const double *rho, const double *u, const double *thT, const double *thR)
{
    if (!b || !rho || !u || !thT || !thR) return PGK_EINVAL;
    hipLaunchKernelGGL(k_batch_init<256>, dim3(b->n), dim3(256), 0, b->stream, b->args, rho, u, thT, thR,
                       b->ns_total);
    BHIP(b, hipGetLastError());
    BHIP(b, hipStreamSynchronize(b->stream));
    b->best.assign(b->n, 1e300);
    b->since.assign(b->n, 0);
    return PGK_OK;
}

extern "C" int pgk_batch_config(pgk_batch *b, int wg, int K)
{
    if (!b) return PGK_EINVAL;
    if (!(wg == 0 && K == 0) && !((wg == 256 || wg == 512) && K >= 2)) return bfail(b, PGK_EINVAL, "bad config");
    if (b->has_e2 && wg == 512) return bfail(b, PGK_EINVAL, "a batch with E2 cases runs with work-groups of 256");
    b->wg = wg;
    b->K = K;
    return PGK_OK;
}

// dynamic LDS of a launch: the arrays of the LDS diffusion path, or the
// conductances of the longest chain, whichever is larger
static size_t batch_lds_bytes(const BatchArgs &a)
{
    return std::max(sizeof(double) * LDS_ARRAYS * a.lds_sites, sizeof(double) * 2 * a.chain_sites);
}

// let every batched kernel take `bytes` of dynamic LDS (above the default 64 KiB)
static hipError_t allow_batch_lds(size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    const void *fns[] = {(const void *)&k_batch<PGK_CN, 256, true>, (const void *)&k_batch<PGK_LIT, 256, true>,
                         (const void *)&k_batch<PGK_CN, 256, false>, (const void *)&k_batch<PGK_CN, 512, false>,
                         (const void *)&k_batch<PGK_LIT, 256, false>, (const void *)&k_batch<PGK_LIT, 512, false>};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// the instantiated graph of one chunk (wg, K, variant), captured on first use
static int chunk_graph(pgk_batch *b, int wg, int K, int variant, hipGraphExec_t *out)
{
    long long key = (long long)wg * 100000 + K * 10 + variant;
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        hipGraph_t g;
        BHIP(b, allow_batch_lds(batch_lds_bytes(b->args)));
        BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        const size_t lds = batch_lds_bytes(b->args);
        dim3 grid(b->n);
        if (b->has_e2) {
            // the E2 Newton needs more registers than two wavefronts per SIMD leave
            if (variant == PGK_CN) hipLaunchKernelGGL((k_batch<PGK_CN, 256, true>), grid, dim3(256), lds, b->stream, b->args, K);
            else hipLaunchKernelGGL((k_batch<PGK_LIT, 256, true>), grid, dim3(256), lds, b->stream, b->args, K);
        } else if (variant == PGK_CN) {
            if (wg == 256) hipLaunchKernelGGL((k_batch<PGK_CN, 256, false>), grid, dim3(256), lds, b->stream, b->args, K);
            else hipLaunchKernelGGL((k_batch<PGK_CN, 512, false>), grid, dim3(512), lds, b->stream, b->args, K);
        } else {
            if (wg == 256) hipLaunchKernelGGL((k_batch<PGK_LIT, 256, false>), grid, dim3(256), lds, b->stream, b->args, K);
            else hipLaunchKernelGGL((k_batch<PGK_LIT, 512, false>), grid, dim3(512), lds, b->stream, b->args, K);
        }
        BHIP(b, hipStreamEndCapture(b->stream, &g));
        hipGraphExec_t ge;
        BHIP(b, hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        (void)hipGraphDestroy(g);
        it = b->graphs.emplace(key, ge).first;
    }
    *out = it->second;
    return PGK_OK;
}

static int chunk(pgk_batch *b, int wg, int K, int variant)
{
    hipGraphExec_t ge;
    int rc = chunk_graph(b, wg, K, variant, &ge);
    if (rc) return rc;
    BHIP(b, hipGraphLaunch(ge, b->stream));
    return PGK_OK;
}

static int readback(pgk_batch *b)
{
    BHIP(b, hipMemcpyAsync(b->h_status, b->args.status, sizeof(int) * b->n, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_steps, b->args.steps, sizeof(long long) * b->n, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipMemcpyAsync(b->h_resid, b->args.resid, sizeof(double) * b->n, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return PGK_OK;
}

// ---- autotuner cache: a flat JSON object {"key": [wg, K], ...} ----------------
static std::string cache_path()
{
    const char *p = getenv("PGK_TUNE_CACHE");
    if (p && *p) return p;
    const char *h = getenv("HOME");
    return std::string(h ? h : "/tmp") + "/.cache/pgk_tune.json";
}

static std::map<std::string, std::pair<int, int>> cache_load()
{
    std::map<std::string, std::pair<int, int>> m;
    FILE *f = fopen(cache_path().c_str(), "r");
    if (!f) return m;
    std::string s;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
    fclose(f);
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        std::string key = s.substr(i + 1, j - i - 1);
        int wg = 0, K = 0;
        if (sscanf(s.c_str() + j + 1, " : [ %d , %d ]", &wg, &K) == 2) m[key] = {wg, K};
        i = j + 1;
    }
    return m;
}

// batches tuned from several host threads share the file: one lock per
// process around load-modify-store, and a rename so that a reader never sees
// a half-written file
static std::mutex cache_mutex;

static void cache_store(const std::map<std::string, std::pair<int, int>> &m)
{
    std::string path = cache_path();
    size_t slash = path.rfind('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (auto &e : m) fprintf(f, "  \"%s\": [%d, %d]%s\n", e.first.c_str(), e.second.first, e.second.second,
                              ++i < m.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    if (rename(tmp.c_str(), path.c_str()) != 0) (void)remove(tmp.c_str());
}

static std::string tune_key(const pgk_batch *b)
{
    hipDeviceProp_t prop;
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipGetDeviceProperties(&prop, dev);
    long long maxL = 0;
    int nrun = 0;
    for (int i = 0; i < b->n; i++)
        if (b->h_status[i] == PGK_CASE_RUNNING) {
            maxL = std::max<long long>(maxL, b->host_cases[i].k.nx);
            nrun++;
        }
    char key[256];
    // arch, number of running cases (log2 bucket), longest running case (log2
    // bucket), variant
    int nb = 0, lb = 0;
    while ((1 << nb) < nrun) nb++;
    while ((1LL << lb) < maxL) lb++;
    snprintf(key, sizeof key, "%s/batch/n%d/L%d/v%d/e%d", prop.gcnArchName, nb, lb, b->host_cases[0].variant,
             b->has_e2 ? 1 : 0);
    for (char *p = key; *p; p++)
        if (*p == '"' || *p == ':') *p = '_';
    return key;
}

static long long running_sites(const pgk_batch *b)
{
    long long act = 0;
    for (int i = 0; i < b->n; i++)
        if (b->h_status[i] == PGK_CASE_RUNNING) act += b->host_cases[i].k.ns;
    return act;
}

static int running_cases(const pgk_batch *b)
{
    int n = 0;
    for (int i = 0; i < b->n; i++) n += b->h_status[i] == PGK_CASE_RUNNING;
    return n;
}

// Work-group size and chunk length for the cases still running: the cached
// choice for this mix, else one chunk of every candidate timed on the live
// state (the chunks advance the cases like any other) and the fastest per
// site update cached.
static int tune(pgk_batch *b, int variant, int &wg, int &K)
{
    std::string key = tune_key(b);
    std::map<std::string, std::pair<int, int>> cache;
    {
        std::lock_guard<std::mutex> lock(cache_mutex);
        cache = cache_load();
    }
    auto hit = cache.find(key);
    bool usable = hit != cache.end() && (hit->second.first == 256 || (hit->second.first == 512 && !b->has_e2)) &&
                  hit->second.second >= 2;
    if (usable) {
        wg = hit->second.first;
        K = hit->second.second;
        return PGK_OK;
    }
    const int cand[][2] = {{256, 32}, {512, 32}, {256, 64}, {512, 64}, {256, 128}, {512, 128}, {256, 256}, {512, 256}};
    double best = 1e300;
    int bw = 0, bk = 0, rc;
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    for (auto &cd : cand) {
        // (a batch holding E2 cases has one work-group size: only K is tuned)
        if (b->has_e2 && cd[0] != 256) continue;
        if (running_sites(b) == 0) break;
        // capture and instantiate outside the timed interval, and time the
        // second of two chunks
        hipGraphExec_t ge;
        rc = chunk_graph(b, cd[0], cd[1], variant, &ge);
        if (rc) return rc;
        BHIP(b, hipGraphLaunch(ge, b->stream));
        rc = readback(b);
        if (rc) return rc;
        long long act = running_sites(b);
        if (act == 0) break;
        BHIP(b, hipEventRecord(e0, b->stream));
        BHIP(b, hipGraphLaunch(ge, b->stream));
        BHIP(b, hipEventRecord(e1, b->stream));
        BHIP(b, hipEventSynchronize(e1));
        float ms = 0.f;
        BHIP(b, hipEventElapsedTime(&ms, e0, e1));
        double nsps = ms * 1e6 / ((double)act * cd[1]);
        if (nsps < best) { best = nsps; bw = cd[0]; bk = cd[1]; }
        rc = readback(b);
        if (rc) return rc;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (bw == 0) return PGK_OK;   // every case stopped while timing: keep the last choice
    wg = bw;
    K = bk;
    b->tuned_ns = best;
    std::lock_guard<std::mutex> lock(cache_mutex);
    cache = cache_load();
    cache[key] = {wg, K};
    cache_store(cache);
    return PGK_OK;
}

extern "C" int pgk_batch_run(pgk_batch *b, int64_t max_steps, double tol, int64_t *steps, double *resid, int *status)
{
    if (!b || max_steps < 1 || !(tol >= 0)) return PGK_EINVAL;
    int variant = b->host_cases[0].variant;
    for (auto &c : b->host_cases)
        if (c.variant != variant) return bfail(b, PGK_EINVAL, "one variant per batch");
    b->args.max_steps = max_steps;
    b->args.tol = tol;
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);   // args changed
    b->graphs.clear();
    int rc = readback(b);
    if (rc) return rc;
    // a case stopped by an earlier, lower step cap runs on to this one
    bool resumed = false;
    for (int i = 0; i < b->n; i++)
        if (b->h_status[i] == PGK_CASE_MAXSTEPS && b->h_steps[i] < max_steps) {
            b->h_status[i] = PGK_CASE_RUNNING;
            resumed = true;
        }
    if (resumed)
        BHIP(b, hipMemcpyAsync(b->args.status, b->h_status, sizeof(int) * b->n, hipMemcpyHostToDevice, b->stream));
    if ((int)b->best.size() != b->n) {
        b->best.assign(b->n, 1e300);
        b->since.assign(b->n, 0);
    }
    auto running = [&]() { return running_sites(b); };
    // automatic choice: tuned at the start and again whenever the number of
    // running cases has halved (the last, longest cases decide the wall time,
    // and few work-groups favour other shapes than a full batch)
    const bool autotune = b->wg == 0;
    int wg = autotune ? 256 : b->wg, K = autotune ? 128 : b->K;
    int tuned_at = 0;
    if (autotune) {
        tuned_at = running_cases(b);
        rc = tune(b, variant, wg, K);
        if (rc) return rc;
    }
    b->tuned_wg = wg;
    b->tuned_K = K;
    // replay chunks until every case has stopped
    hipEvent_t t0, t1;
    BHIP(b, hipEventCreate(&t0));
    BHIP(b, hipEventCreate(&t1));
    double site_updates = 0.0, ms_total = 0.0;
    std::vector<double> &best = b->best;
    std::vector<long long> &since = b->since;
    while (true) {
        long long act = running();
        if (act == 0) break;
        if (autotune && running_cases(b) * 2 <= tuned_at) {
            tuned_at = running_cases(b);
            rc = tune(b, variant, wg, K);
            if (rc) return rc;
            b->tuned_wg = wg;
            b->tuned_K = K;
            act = running();
            if (act == 0) break;
        }
        BHIP(b, hipEventRecord(t0, b->stream));
        rc = chunk(b, wg, K, variant);
        if (rc) return rc;
        BHIP(b, hipEventRecord(t1, b->stream));
        rc = readback(b);
        if (rc) return rc;
        float ms = 0.f;
        BHIP(b, hipEventElapsedTime(&ms, t0, t1));
        ms_total += ms;
        site_updates += (double)act * K;
        if (b->stall_window > 0) {
            bool changed = false;
            for (int i = 0; i < b->n; i++) {
                if (b->h_status[i] != PGK_CASE_RUNNING) continue;
                if (b->h_resid[i] < 0.5 * best[i]) {
                    best[i] = b->h_resid[i];
                    since[i] = 0;
                } else if ((since[i] += K) >= b->stall_window) {
                    b->h_status[i] = PGK_CASE_STALLED;
                    changed = true;
                }
            }
            // the kernel skips every case whose status is not RUNNING
            if (changed)
                BHIP(b, hipMemcpyAsync(b->args.status, b->h_status, sizeof(int) * b->n, hipMemcpyHostToDevice,
                                       b->stream));
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (site_updates > 0) b->tuned_ns = ms_total * 1e6 / site_updates;
    for (int i = 0; i < b->n; i++) {
        if (steps) steps[i] = b->h_steps[i];
        if (resid) resid[i] = b->h_resid[i];
        if (status) status[i] = b->h_status[i];
    }
    return PGK_OK;
}

extern "C" int pgk_batch_stall(pgk_batch *b, int64_t window)
{
    if (!b || window < 0) return PGK_EINVAL;
    b->stall_window = window;
    return PGK_OK;
}

extern "C" int pgk_batch_tuned(const pgk_batch *b, int *wg, int *K, double *ns)
{
    if (!b) return PGK_EINVAL;
    if (wg) *wg = b->tuned_wg;
    if (K) *K = b->tuned_K;
    if (ns) *ns = b->tuned_ns;
    return PGK_OK;
}

extern "C" int pgk_batch_read_moments(pgk_batch *b, double *rho, double *u, double *thT, double *thR)
{
    if (!b) return PGK_EINVAL;
    hipLaunchKernelGGL(k_batch_moments<256>, dim3(b->n), dim3(256), 0, b->stream, b->args, rho, u, thT, thR,
                       b->ns_total);
    BHIP(b, hipGetLastError());
    return PGK_OK;
}

extern "C" const char *pgk_batch_last_error(const pgk_batch *b) { return b ? b->err.c_str() : "null batch"; }

extern "C" void pgk_batch_destroy(pgk_batch *b) { delete b; }
