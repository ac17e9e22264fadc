// Host check of the bounded pull: the index each population of a site pulls,
// computed from the per-site maps (pull_index_b), equals the direct formula
// (position_index of the position x - c) for every site, population and face
// configuration of many small grids.  The device helpers are compiled as
// host-and-device functions for this check only.
#include <hip/hip_runtime.h>
#undef __device__
#define __device__ __attribute__((host)) __attribute__((device))
#include "device.hpp"
#include <cstdio>
#include <cstdlib>
using namespace pgk;

static long long nchk = 0, nghost = 0, nbad = 0;

template <int BOUNDED, int Q = 0>
void check_site(int x, int y, int z, int sub, const Consts &k, const PullMap &p, const GhostMap<BOUNDED> &g)
{
    if constexpr (Q < NQ) {
        constexpr int cx = c2(Q, 0), cy = c2(Q, 1), cz = c2(Q, 2);
        int g0, g1;
        int i0 = position_index<BOUNDED>(2 * x + sub - cx, 2 * y + sub - cy, 2 * z + sub - cz, Q, k, g0);
        int i1 = pull_index_b<Q, BOUNDED>(p, g, k, g1);
        nchk++;
        if (g0) nghost++;
        if (i0 != i1 || g0 != g1) {
            if (nbad < 10)
                printf("MISMATCH B%d n=(%d,%d,%d) bc=(%d,%d,%d,%d) site (%d,%d,%d,%d) Q %d: %d/%d vs %d/%d\n", BOUNDED,
                       k.nx, k.ny, k.nz, k.bc[0], k.bc[1], k.bc[2], k.bc[3], x, y, z, sub, Q, i0, g0, i1, g1);
            nbad++;
        }
        check_site<BOUNDED, Q + 1>(x, y, z, sub, k, p, g);
    }
}

template <int BOUNDED>
void run(int nx, int ny, int nz, int b0, int b1, int b2, int b3)
{
    Consts k{};
    k.nx = nx; k.ny = ny; k.nz = nz; k.ns = 2 * nx * ny * nz;
    k.bc[0] = b0; k.bc[1] = b1; k.bc[2] = b2; k.bc[3] = b3;
    for (int sub = 0; sub < 2; sub++)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    PullMap p = pull_map(x, y, z, sub, k);
                    GhostMap<BOUNDED> g = ghost_map<BOUNDED>(x, y, z, sub, k);
                    check_site<BOUNDED>(x, y, z, sub, k, p, g);
                }
}

int main()
{
    const int P = PGK_PERIODIC, W = PGK_WALL, D = PGK_DIRICHLET;
    const int dims[] = {1, 2, 3, 4, 5, 7, 9};
    for (int nx : dims)
        for (int ny : dims)
            for (int nz : {1, 2, 3, 5}) {
                // x faces only (y periodic): BND_X and BND_XY kernels
                for (int bx : {W, D}) {
                    run<BND_X>(nx, ny, nz, bx, bx, P, P);
                    run<BND_X>(nx, ny, nz, W, D, P, P);
                    run<BND_XY>(nx, ny, nz, bx, bx, P, P);
                }
                // faces on y (x periodic or bounded)
                for (int by : {W, D}) {
                    run<BND_XY>(nx, ny, nz, P, P, by, by);
                    run<BND_XY>(nx, ny, nz, W, W, by, by);
                    run<BND_XY>(nx, ny, nz, D, W, W, D);
                }
                // all periodic through a bounded kernel
                run<BND_X>(nx, ny, nz, P, P, P, P);
                run<BND_XY>(nx, ny, nz, P, P, P, P);
            }
    run<BND_X>(4096, 1, 1, D, D, P, P);
    run<BND_XY>(64, 48, 2, W, W, W, W);
    printf("checked %lld pulls (%lld through ghosts), %lld mismatches\n", nchk, nghost, nbad);
    return nbad != 0;
}
