// RD3Q41 velocity set on the bcc grid (Sec. 5, Table of velocities and weights).
//
// Velocities are kept in doubled integer coordinates so that the eight
// half-velocities (+-1/2, +-1/2, +-1/2) stay integral.  The 40 moving
// velocities come in opposite pairs; pair p (0..19) is the representative
// REP2[p] and its negative.  Population index: 0 = rest, 1 + p = +c_p,
// 21 + p = -c_p.  Shells: 0 rest, 1 (1,0,0), 2 (2,0,0), 3 (1,1,0),
// 4 (1,1,1), 5 (1/2,1/2,1/2).
#pragma once

namespace pgk {

constexpr int NQ = 41;
constexpr int NPAIR = 20;

struct Lattice {
    static constexpr int REP2[NPAIR][3] = {
        {2, 0, 0}, {0, 2, 0}, {0, 0, 2},                              // shell 1
        {4, 0, 0}, {0, 4, 0}, {0, 0, 4},                              // shell 2
        {2, 2, 0}, {2, -2, 0}, {2, 0, 2}, {2, 0, -2}, {0, 2, 2}, {0, 2, -2},  // shell 3
        {2, 2, 2}, {2, 2, -2}, {2, -2, 2}, {2, -2, -2},               // shell 4
        {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};              // shell 5
    static constexpr int SHELL[NPAIR] = {1, 1, 1, 2, 2, 2, 3, 3, 3, 3, 3, 3,
                                         4, 4, 4, 4, 5, 5, 5, 5};
};

// doubled coordinate of population q along axis a
__host__ __device__ constexpr int c2(int q, int a)
{
    return q == 0 ? 0 : (q <= NPAIR ? Lattice::REP2[q - 1][a] : -Lattice::REP2[q - 1 - NPAIR][a]);
}

__host__ __device__ constexpr int shell_of(int q)
{
    return q == 0 ? 0 : Lattice::SHELL[(q - 1) % NPAIR];
}

// Shell weights as polynomials in the reference temperature t (Table of weights).
inline void shell_weights(double t, double w[6])
{
    w[0] = (52.0 - 323.0 * t + 921.0 * t * t - 1036.0 * t * t * t) / 52.0;
    w[1] = t * (12.0 - 38.0 * t + 63.0 * t * t) / 39.0;
    w[2] = t * (3.0 - 29.0 * t + 84.0 * t * t) / 312.0;
    w[3] = t * (45.0 * t - 6.0 - 77.0 * t * t) / 26.0;
    w[4] = t * (20.0 - 163.0 * t + 378.0 * t * t) / 312.0;
    w[5] = 8.0 * t * (4.0 - 17.0 * t + 21.0 * t * t) / 39.0;
}

constexpr double THETA0_PRINTED = 0.2948964908710633;

}  // namespace pgk
