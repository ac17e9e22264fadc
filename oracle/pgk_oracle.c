/*
 * pgk_oracle.c -- plain FP64 CPU oracle for the reduced polyatomic ES-BGK
 * lattice-Boltzmann step (Kolluru, Atif & Ansumali, "Reduced kinetic model of
 * polyatomic gases", arXiv:2201.05280).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path (the
 * HIP library) never calls it, and the two share no code, headers or tables.
 *
 * Everything here is written for a reader holding the paper: slow, per-site,
 * per-velocity loops in double precision, following the paper's order:
 *   1. moments of the auxiliary populations g          (Sec. 5, discrete moments)
 *   2. g -> f moment map with the first half of the
 *      rotational relaxation (backward Euler)           (Sec. 5, g-f relations and step 1)
 *   3. ES target lambda = theta_T I + b sigma/rho and the
 *      BGK target at theta, combined at rate 1/tau*      (Sec. 4 kinetic equation; Sec. 2 ES-BGK)
 *   4. discrete equilibrium on RD3Q41                    (Sec. 5, Table of weights)
 *   5. trapezoid collide  g* = (1-2b*) g + 2b* F          (Sec. 5, g evolution)
 *   6. pull streaming on the bcc grid                   (Sec. 5, bcc arrangement)
 *   7. rotational energy: MacCormack advection, FTCS
 *      diffusion, second relaxation half                 (Sec. 5, steps 2-4)
 *
 * Where the paper is silent the readings are:
 *   - the gain term of the g update is F = tau*(f^ES/tau + f^MB/tau1);
 *   - lambda uses sigma/rho (sigma carries a factor rho);
 *   - the theta_R entering the g->f temperature map is the half-relaxed one,
 *     solved jointly with theta_T in closed form;
 *   - the rotational state is theta_R, transported in the printed advective
 *     form with u^n;
 *   - variant CN (default): the second relaxation half is the explicit
 *     complement of the first (Crank-Nicolson overall), which makes the
 *     translational-rotational exchange of each collision exactly energy
 *     conserving, and the diffusion uses the conservative face-flux form of
 *     div(kappa_R grad theta_R); variant LIT: backward-Euler second half and
 *     D_R lap(theta_R), as printed;
 *   - equilibrium F3: third-order Hermite projection about (0, theta0) of the
 *     anisotropic Gaussian; E2: discrete exponential quasi-equilibrium
 *     w_i exp(alpha + beta.c_i + c_i.G.c_i) matching rho, rho u and the
 *     pressure tensor (E2 is not linear in the covariance, so its gain term
 *     mixes the ES and the Maxwellian E2 populations at their rates); F4:
 *     F3 plus contracted fourth-order Hermite terms that make the contracted
 *     fourth moment sum F c^2 c_a c_b Gaussian for every state (also
 *     nonlinear in the covariance, mixed like E2);
 *   - finite differences for E_R use the simple-cubic neighbours of the same
 *     sublattice (spacing 1);
 *   - kappa_R = k_r * 5 p tau / (2B) with the local p = rho theta; face values
 *     are arithmetic means.
 * Pins: see the oracle tests (lattice isotropy, Gaussian moments of F3 and
 * E2, exact conservation, CE decay rates, sound speed, Landau table, the
 * Couette start-up series and the thermal Couette profile of Sec. 6, the
 * effective-delta sound speeds, the acoustic pulse against the Bessel
 * integral, weak shocks against the Navier-Stokes weak-shock thickness).
 * Parity unpinned: the interior profile of a strong normal shock (its end
 * states, through the jump conditions, and its conservation are pinned, and
 * so is the thickness in the weak-shock limit; the shape of a strong shock
 * has no reference outside this code).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 41

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_DIRICHLET = 2 };
enum { VAR_CN = 0, VAR_LIT = 1 };
enum { EQ_F3 = 0, EQ_E2 = 1, EQ_F4 = 2 };

/* ------------------------------------------------------------------------ */
/* RD3Q41 velocity set (Table "weights"): doubled integer coordinates so the  */
/* half-velocities (+-1/2,+-1/2,+-1/2) stay integral.                         */
/* ------------------------------------------------------------------------ */
static void build_velocities(int c2[NQ][3], int shell[NQ])
{
    int n = 0;
    c2[n][0] = 0; c2[n][1] = 0; c2[n][2] = 0; shell[n] = 0; n++;
    for (int a = 0; a < 3; a++)               /* (+-1,0,0) and permutations */
        for (int s = -1; s <= 1; s += 2) {
            c2[n][0] = c2[n][1] = c2[n][2] = 0; c2[n][a] = 2 * s; shell[n] = 1; n++;
        }
    for (int a = 0; a < 3; a++)               /* (+-2,0,0) and permutations */
        for (int s = -1; s <= 1; s += 2) {
            c2[n][0] = c2[n][1] = c2[n][2] = 0; c2[n][a] = 4 * s; shell[n] = 2; n++;
        }
    for (int a = 0; a < 3; a++)               /* (+-1,+-1,0) and permutations */
        for (int b = a + 1; b < 3; b++)
            for (int s = -1; s <= 1; s += 2)
                for (int t = -1; t <= 1; t += 2) {
                    c2[n][0] = c2[n][1] = c2[n][2] = 0;
                    c2[n][a] = 2 * s; c2[n][b] = 2 * t; shell[n] = 3; n++;
                }
    for (int s = -1; s <= 1; s += 2)          /* (+-1,+-1,+-1) */
        for (int t = -1; t <= 1; t += 2)
            for (int r = -1; r <= 1; r += 2) {
                c2[n][0] = 2 * s; c2[n][1] = 2 * t; c2[n][2] = 2 * r; shell[n] = 4; n++;
            }
    for (int s = -1; s <= 1; s += 2)          /* (+-1/2,+-1/2,+-1/2) */
        for (int t = -1; t <= 1; t += 2)
            for (int r = -1; r <= 1; r += 2) {
                c2[n][0] = s; c2[n][1] = t; c2[n][2] = r; shell[n] = 5; n++;
            }
}

/* weight polynomials of the Table of weights, evaluated at theta0 */
static double shell_weight(int shell, double t)
{
    switch (shell) {
    case 0: return (52.0 - 323.0 * t + 921.0 * t * t - 1036.0 * t * t * t) / 52.0;
    case 1: return t * (12.0 - 38.0 * t + 63.0 * t * t) / 39.0;
    case 2: return t * (3.0 - 29.0 * t + 84.0 * t * t) / 312.0;
    case 3: return t * (45.0 * t - 6.0 - 77.0 * t * t) / 26.0;
    case 4: return t * (20.0 - 163.0 * t + 378.0 * t * t) / 312.0;
    default: return 8.0 * t * (4.0 - 17.0 * t + 21.0 * t * t) / 39.0;
    }
}

void pgko_lattice(double theta0, double *c /* [41][3] */, double *w /* [41] */)
{
    int c2[NQ][3], shell[NQ];
    build_velocities(c2, shell);
    for (int i = 0; i < NQ; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = 0.5 * c2[i][a];
        w[i] = shell_weight(shell[i], theta0);
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibria                                                               */
/* ------------------------------------------------------------------------ */
/* symmetric 3x3 from 6 comps xx,yy,zz,xy,xz,yz */
static void sym_from6(const double *s6, double m[3][3])
{
    m[0][0] = s6[0]; m[1][1] = s6[1]; m[2][2] = s6[2];
    m[0][1] = m[1][0] = s6[3];
    m[0][2] = m[2][0] = s6[4];
    m[1][2] = m[2][1] = s6[5];
}

/* F3: third-order Hermite expansion, about the lattice reference state
 * (u = 0, theta0 I), of the Gaussian with mean u and covariance lam:
 *   F_i = w_i rho [1 + a1.H1/theta0 + a2:H2/(2 theta0^2) + a3:H3/(6 theta0^3)]
 * with a1 = u, a2 = uu + D, a3 = uuu + (D u + perms), D = lam - theta0 I, and
 * the Hermite tensors H1 = c, H2 = cc - theta0 I, H3 = ccc - theta0 (c I)_sym. */
void pgko_feq_f3(double theta0, const double *w, const double *c, double rho,
                 const double *u, const double *lam6, double *F)
{
    double D[3][3];
    sym_from6(lam6, D);
    for (int a = 0; a < 3; a++) D[a][a] -= theta0;
    double trD = D[0][0] + D[1][1] + D[2][2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double t = theta0, t2 = t * t, t3 = t2 * t;
    for (int i = 0; i < NQ; i++) {
        const double *ci = c + 3 * i;
        double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
        double cDc = 0.0, cDu = 0.0;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                cDc += ci[a] * D[a][b] * ci[b];
                cDu += ci[a] * D[a][b] * u[b];
            }
        double a1H1 = cu;
        double a2H2 = cu * cu + cDc - t * (uu + trD);
        double a3H3 = cu * cu * cu + 3.0 * cDc * cu - t * (3.0 * uu * cu + 6.0 * cDu + 3.0 * trD * cu);
        F[i] = w[i] * rho * (1.0 + a1H1 / t + a2H2 / (2.0 * t2) + a3H3 / (6.0 * t3));
    }
}

/* Solve the symmetric positive definite n x n system A x = b (Cholesky);
 * returns 0 on success, -1 if A is not positive definite. */
static int spd_solve(int n, double *A, double *b)
{
    for (int j = 0; j < n; j++) {
        double s = A[j * n + j];
        for (int k = 0; k < j; k++) s -= A[j * n + k] * A[j * n + k];
        if (!(s > 0.0)) return -1;
        double d = sqrt(s);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; i++) {
            double v = A[i * n + j];
            for (int k = 0; k < j; k++) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    for (int i = 0; i < n; i++) {
        double v = b[i];
        for (int k = 0; k < i; k++) v -= A[i * n + k] * b[k];
        b[i] = v / A[i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double v = b[i];
        for (int k = i + 1; k < n; k++) v -= A[k * n + i] * b[k];
        b[i] = v / A[i * n + i];
    }
    return 0;
}

/* invert a symmetric 3x3, returns determinant */
static double inv3(double m[3][3], double r[3][3])
{
    double det = m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
               - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
               + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
    r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / det;
    r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / det;
    r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / det;
    r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / det;
    r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / det;
    r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / det;
    r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / det;
    r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / det;
    r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / det;
    return det;
}

/* F4: F3 plus contracted fourth-order Hermite terms, so that besides the
 * moments F3 carries (orders 0 to 3) the contracted fourth moment
 *   R_ab = sum_i F_i c_i^2 c_ia c_ib
 * equals that of the Gaussian N(u, lam) for every state.  The lattice's
 * weights are built so that the contracted moments of the Gaussian hold up
 * to the eighth order (Sec. 5, the weight and theta0 conditions), which is
 * what such a term needs.  The correction is w_i sum_ab K_ab h_ab(c_i) with
 *   h_ab(c) = c_a c_b (c^2 - 7 theta0) - delta_ab theta0 (c^2 - 5 theta0),
 * the contracted fourth-order Hermite polynomial of the weight w: it is
 * orthogonal to 1 and to c_e c_f under w (and even in c), so it leaves the
 * moments of orders 0 to 3 unchanged.  K follows from the 6 x 6 linear system
 *   sum_i w_i (sum_ab K_ab h_ab(c_i)) c_i^2 c_ie c_if = R^G_ef - R^F3_ef,
 * with R^G from Isserlis' theorem and R^F3 summed over the 41 velocities. */
static double f4_h(const double *ci, int a, int b, double t)
{
    double c2 = ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2];
    return ci[a] * ci[b] * (c2 - 7.0 * t) - (a == b ? t * (c2 - 5.0 * t) : 0.0);
}

/* Gauss-Jordan elimination with partial pivoting on an n x n system (n <= 6) */
static int solve_general(int n, double *A, double *x)
{
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(A[r * n + col]) > fabs(A[piv * n + col])) piv = r;
        if (!(fabs(A[piv * n + col]) > 0.0)) return -1;
        if (piv != col) {
            for (int k = 0; k < n; k++) {
                double t = A[col * n + k]; A[col * n + k] = A[piv * n + k]; A[piv * n + k] = t;
            }
            double t = x[col]; x[col] = x[piv]; x[piv] = t;
        }
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            double f = A[r * n + col] / A[col * n + col];
            for (int k = col; k < n; k++) A[r * n + k] -= f * A[col * n + k];
            x[r] -= f * x[col];
        }
    }
    for (int r = 0; r < n; r++) x[r] /= A[r * n + r];
    return 0;
}

void pgko_feq_f4(double theta0, const double *w, const double *c, double rho,
                 const double *u, const double *lam6, double *F)
{
    static const int IA[6] = {0, 1, 2, 0, 0, 1}, IB[6] = {0, 1, 2, 1, 2, 2};
    pgko_feq_f3(theta0, w, c, rho, u, lam6, F);
    double L[3][3];
    sym_from6(lam6, L);
    /* Gaussian: E[c^2 c_a c_b] for c ~ N(u, L) (Isserlis) */
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double trL = L[0][0] + L[1][1] + L[2][2];
    double Lu[3], LL[3][3];
    for (int a = 0; a < 3; a++) {
        Lu[a] = L[a][0] * u[0] + L[a][1] * u[1] + L[a][2] * u[2];
        for (int b = 0; b < 3; b++) LL[a][b] = L[a][0] * L[0][b] + L[a][1] * L[1][b] + L[a][2] * L[2][b];
    }
    double rhs[6], A[36];
    for (int e = 0; e < 6; e++) {
        int a = IA[e], b = IB[e];
        double RG = uu * u[a] * u[b] + uu * L[a][b] + 2.0 * (u[a] * Lu[b] + Lu[a] * u[b]) + trL * u[a] * u[b]
                  + trL * L[a][b] + 2.0 * LL[a][b];
        double RF = 0.0;
        for (int i = 0; i < NQ; i++) {
            const double *ci = c + 3 * i;
            RF += F[i] * (ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2]) * ci[a] * ci[b];
        }
        rhs[e] = rho * RG - RF;
        /* column j: basis h_xx, h_yy, h_zz, h_xy + h_yx, h_xz + h_zx, h_yz + h_zy */
        for (int j = 0; j < 6; j++) {
            double m = 0.0;
            for (int i = 0; i < NQ; i++) {
                const double *ci = c + 3 * i;
                double g = (j < 3 ? 1.0 : 2.0) * f4_h(ci, IA[j], IB[j], theta0);
                m += w[i] * g * (ci[0] * ci[0] + ci[1] * ci[1] + ci[2] * ci[2]) * ci[a] * ci[b];
            }
            A[e * 6 + j] = m;
        }
    }
    solve_general(6, A, rhs);   /* rhs -> K (xx yy zz xy xz yz) */
    for (int i = 0; i < NQ; i++) {
        const double *ci = c + 3 * i;
        double corr = 0.0;
        for (int j = 0; j < 6; j++) corr += (j < 3 ? 1.0 : 2.0) * rhs[j] * f4_h(ci, IA[j], IB[j], theta0);
        F[i] += w[i] * corr;
    }
}

/* E2: discrete quasi-equilibrium, the lattice analogue of the minimiser of
 * H under fixed rho, rho u and pressure tensor (Sec. 2, quasi-equilibrium):
 *   F_i = w_i exp(alpha + beta.c_i + c_i.G.c_i)
 * Newton on the 10 Lagrange multipliers so that sum_i F_i {1, c, cc} equals
 * {rho, rho u, rho (uu + lam)}.  Returns the iteration count (> 0) on
 * success, -1 if the moments are not reached (target not realisable on the
 * 41 velocities or lost positive definiteness). */
int pgko_feq_e2(double theta0, const double *w, const double *c, double rho,
                const double *u, const double *lam6, double *F)
{
    /* basis functions phi_k(c): 1, cx, cy, cz, cxcx, cycy, czcz, cxcy, cxcz, cycz */
    double phi[NQ][10];
    for (int i = 0; i < NQ; i++) {
        const double *ci = c + 3 * i;
        phi[i][0] = 1.0; phi[i][1] = ci[0]; phi[i][2] = ci[1]; phi[i][3] = ci[2];
        phi[i][4] = ci[0] * ci[0]; phi[i][5] = ci[1] * ci[1]; phi[i][6] = ci[2] * ci[2];
        phi[i][7] = ci[0] * ci[1]; phi[i][8] = ci[0] * ci[2]; phi[i][9] = ci[1] * ci[2];
    }
    double L[3][3], Li[3][3];
    sym_from6(lam6, L);
    double target[10];
    target[0] = rho;
    for (int a = 0; a < 3; a++) target[1 + a] = rho * u[a];
    target[4] = rho * (u[0] * u[0] + L[0][0]);
    target[5] = rho * (u[1] * u[1] + L[1][1]);
    target[6] = rho * (u[2] * u[2] + L[2][2]);
    target[7] = rho * (u[0] * u[1] + L[0][1]);
    target[8] = rho * (u[0] * u[2] + L[0][2]);
    target[9] = rho * (u[1] * u[2] + L[1][2]);
    /* start: ratio of the continuous Gaussian N(u, lam) to N(0, theta0 I) */
    double det = inv3(L, Li);
    if (!(det > 0.0)) return -1;
    double lm[10];
    double Liu[3];
    for (int a = 0; a < 3; a++) Liu[a] = Li[a][0] * u[0] + Li[a][1] * u[1] + Li[a][2] * u[2];
    double uLiu = u[0] * Liu[0] + u[1] * Liu[1] + u[2] * Liu[2];
    lm[0] = log(rho) - 0.5 * log(det / (theta0 * theta0 * theta0)) - 0.5 * uLiu;
    for (int a = 0; a < 3; a++) lm[1 + a] = Liu[a];
    /* c.G.c with G = -1/2 (Li - I/theta0): diagonal coefficient G_aa,
       off-diagonal coefficient 2 G_ab (since cxcy appears twice) */
    lm[4] = -0.5 * (Li[0][0] - 1.0 / theta0);
    lm[5] = -0.5 * (Li[1][1] - 1.0 / theta0);
    lm[6] = -0.5 * (Li[2][2] - 1.0 / theta0);
    lm[7] = -Li[0][1];
    lm[8] = -Li[0][2];
    lm[9] = -Li[1][2];
    double scale = 0.0;
    for (int k = 0; k < 10; k++) scale += fabs(target[k]);
    double last = 1e300;   /* largest exponent change of the last Newton step */
    for (int it = 1; it <= 100; it++) {
        double mom[10] = {0}, J[100] = {0};
        for (int i = 0; i < NQ; i++) {
            double ex = 0.0;
            for (int k = 0; k < 10; k++) ex += lm[k] * phi[i][k];
            F[i] = w[i] * exp(ex);
            for (int k = 0; k < 10; k++) {
                mom[k] += F[i] * phi[i][k];
                for (int l = 0; l < 10; l++) J[k * 10 + l] += F[i] * phi[i][k] * phi[i][l];
            }
        }
        double res = 0.0, rhs[10];
        for (int k = 0; k < 10; k++) {
            rhs[k] = target[k] - mom[k];
            res += fabs(rhs[k]);
        }
        /* the equilibrium is fixed by its moments alone: stop at the round-off
           floor (moments met and a last step too small to matter), so the
           result does not depend on where the iteration started */
        if (res <= 1e-14 * scale && last <= 1e-8) return it;
        if (spd_solve(10, J, rhs) != 0) return -1;
        /* damped step: limit the change of the exponent at any velocity */
        double maxd = 0.0;
        for (int i = 0; i < NQ; i++) {
            double d = 0.0;
            for (int k = 0; k < 10; k++) d += rhs[k] * phi[i][k];
            if (fabs(d) > maxd) maxd = fabs(d);
        }
        last = maxd;
        double damp = maxd > 2.0 ? 2.0 / maxd : 1.0;
        for (int k = 0; k < 10; k++) lm[k] += damp * rhs[k];
        if (!isfinite(lm[0])) return -1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* State                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct pgko {
    int nx, ny, nz, ns;
    int variant, eq;
    double tau, tau1, b, kr, delta, th0;
    double taus, beta, X, Y, ssig, B;
    double c[NQ][3], w[NQ];
    int c2[NQ][3];
    double *g, *gp, *er;
    /* per-site results of the collision, used by the rotational transport */
    double *rho, *u, *T, *theta, *ehat, *d;
    double *e1, *e2, *phi;
    int bc[2][2];                       /* [axis x, y][side low, high] */
    double bc_rho[2][2], bc_u[2][2][3], bc_th[2][2];
    int e2_fail;
    int nsub;          /* FTCS sub-steps of the theta_R diffusion */
} pgko;

static int site_index(const pgko *o, int sub, int z, int y, int x)
{
    return ((sub * o->nz + z) * o->ny + y) * o->nx + x;
}

static void site_coords(const pgko *o, int s, int *sub, int *z, int *y, int *x)
{
    *x = s % o->nx; s /= o->nx;
    *y = s % o->ny; s /= o->ny;
    *z = s % o->nz; *sub = s / o->nz;
}

static int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

pgko *pgko_create(int nx, int ny, int nz, int variant, int equilibrium)
{
    if (nx < 1 || ny < 1 || nz < 1) return NULL;
    pgko *o = (pgko *)calloc(1, sizeof(pgko));
    o->nx = nx; o->ny = ny; o->nz = nz;
    o->ns = 2 * nx * ny * nz;
    if (equilibrium < EQ_F3 || equilibrium > EQ_F4) { free(o); return NULL; }
    o->variant = variant; o->eq = equilibrium;
    int shell[NQ];
    build_velocities(o->c2, shell);
    size_t n = (size_t)o->ns;
    o->g = (double *)calloc(NQ * n, sizeof(double));
    o->gp = (double *)calloc(NQ * n, sizeof(double));
    o->er = (double *)calloc(n, sizeof(double));
    o->rho = (double *)calloc(n, sizeof(double));
    o->u = (double *)calloc(3 * n, sizeof(double));
    o->T = (double *)calloc(n, sizeof(double));
    o->theta = (double *)calloc(n, sizeof(double));
    o->ehat = (double *)calloc(n, sizeof(double));
    o->d = (double *)calloc(n, sizeof(double));
    o->e1 = (double *)calloc(n, sizeof(double));
    o->e2 = (double *)calloc(n, sizeof(double));
    o->phi = (double *)calloc(n, sizeof(double));
    o->bc[0][0] = o->bc[0][1] = o->bc[1][0] = o->bc[1][1] = BC_PERIODIC;
    return o;
}

void pgko_destroy(pgko *o)
{
    if (!o) return;
    free(o->g); free(o->gp); free(o->er); free(o->rho); free(o->u); free(o->T);
    free(o->theta); free(o->ehat); free(o->d); free(o->e1); free(o->e2); free(o->phi);
    free(o);
}

int pgko_sites(const pgko *o) { return o->ns; }

int pgko_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* tau, tau1: the two relaxation times; b: ES parameter; kr = kappa_R/kappa_T;
 * delta: rotational degrees of freedom; theta0: lattice reference temperature. */
int pgko_set_params(pgko *o, double tau, double tau1, double b, double kr,
                    double delta, double theta0)
{
    if (!(tau > 0) || !(tau1 > 0) || !(delta > 0) || !(theta0 > 0)) return -1;
    o->tau = tau; o->tau1 = tau1; o->b = b; o->kr = kr; o->delta = delta; o->th0 = theta0;
    o->taus = tau * tau1 / (tau + tau1);                   /* 1/tau* = 1/tau + 1/tau1 */
    o->beta = 1.0 / (2.0 * o->taus + 1.0);                 /* beta* = dt/(2 tau* + dt) */
    o->X = 3.0 / (2.0 * tau1 * (3.0 + delta));             /* step 1 of the theta_R split */
    o->Y = delta / (2.0 * tau1 * (3.0 + delta));           /* theta_T(g) - theta_T(f) map */
    o->ssig = 1.0 + 1.0 / (2.0 * o->taus) - b / (2.0 * tau); /* sigma(g) = sigma(f) ssig */
    o->B = 1.0 + tau / tau1;
    for (int i = 0; i < NQ; i++)
        for (int a = 0; a < 3; a++) o->c[i][a] = 0.5 * o->c2[i][a];
    int shell[NQ], c2[NQ][3];
    build_velocities(c2, shell);
    for (int i = 0; i < NQ; i++) o->w[i] = shell_weight(shell[i], theta0);
    return 0;
}

/* axis 0 = x, 1 = y (z is periodic); side 0 = low, 1 = high.  kind:
 * periodic, wall (diffuse, at rest or moving tangentially with velocity u
 * and temperature theta), Dirichlet (equilibrium ghost state rho, u, theta).
 * Periodic must be set on both sides of an axis. */
int pgko_set_bc(pgko *o, int axis, int side, int kind, double rho, const double *u, double theta)
{
    if (axis < 0 || axis > 1 || side < 0 || side > 1) return -1;
    if (axis == 1 && kind != BC_PERIODIC && o->ny < 2) return -1;
    o->bc[axis][side] = kind;
    o->bc_rho[axis][side] = rho;
    for (int a = 0; a < 3; a++) o->bc_u[axis][side][a] = u ? u[a] : 0.0;
    o->bc_th[axis][side] = theta;
    return 0;
}

int pgko_set_bc_x(pgko *o, int side, int kind, double rho, const double *u, double theta)
{
    return pgko_set_bc(o, 0, side, kind, rho, u, theta);
}

static int equilibrium(const pgko *o, double rho, const double *u, const double *lam6, double *F)
{
    if (o->eq == EQ_E2) {
        int it = pgko_feq_e2(o->th0, o->w, &o->c[0][0], rho, u, lam6, F);
        return it > 0 ? 0 : -1;
    }
    if (o->eq == EQ_F4) pgko_feq_f4(o->th0, o->w, &o->c[0][0], rho, u, lam6, F);
    else pgko_feq_f3(o->th0, o->w, &o->c[0][0], rho, u, lam6, F);
    return 0;
}

/* Initial state: g_i = F_i(rho, u, theta_T I), rotational state from theta_R. */
int pgko_init(pgko *o, const double *rho, const double *u, const double *thT, const double *thR)
{
    int ns = o->ns, fail = 0;
#pragma omp parallel for reduction(+ : fail)
    for (int s = 0; s < ns; s++) {
        double F[NQ], uu[3] = {u[s], u[ns + s], u[2 * ns + s]};
        double lam[6] = {thT[s], thT[s], thT[s], 0, 0, 0};
        if (equilibrium(o, rho[s], uu, lam, F)) fail++;
        for (int i = 0; i < NQ; i++) o->g[(size_t)i * ns + s] = F[i];
        o->er[s] = thR[s];
    }
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* One site: moments, coupled temperature solve, target, equilibrium, collide */
/* ------------------------------------------------------------------------ */
typedef struct {
    double rho, u[3], a, sig_g[3][3], r, T, R, theta, P_f[3][3];
} site_state;

static void site_moments(const pgko *o, const double *gi, double er, site_state *st)
{
    double rho = 0.0, j[3] = {0, 0, 0}, P[3][3] = {{0}};
    for (int i = 0; i < NQ; i++) {
        rho += gi[i];
        for (int a = 0; a < 3; a++) {
            j[a] += gi[i] * o->c[i][a];
            for (int b = 0; b < 3; b++) P[a][b] += gi[i] * o->c[i][a] * o->c[i][b];
        }
    }
    st->rho = rho;
    double uu = 0.0;
    for (int a = 0; a < 3; a++) { st->u[a] = j[a] / rho; uu += st->u[a] * st->u[a]; }
    /* theta_T(g) = (sum g c^2 - rho u^2) / (3 rho) */
    st->a = (P[0][0] + P[1][1] + P[2][2] - rho * uu) / (3.0 * rho);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            st->sig_g[a][b] = P[a][b] - rho * st->u[a] * st->u[b] - (a == b ? rho * st->a : 0.0);
    /* rotational temperature at t */
    st->r = er;
    /* joint solve of  a = T + Y (T - R)   (g -> f temperature map) and
     *                 R = (r + X T)/(1+X)  (backward-Euler half relaxation) */
    double X = o->X, Y = o->Y;
    st->T = (st->a * (1.0 + X) + Y * st->r) / (1.0 + X + Y);
    st->R = (st->r + X * st->T) / (1.0 + X);
    /* total temperature, theta = 3/(3+d) theta_T + d/(3+d) theta_R */
    st->theta = (3.0 * st->T + o->delta * st->R) / (3.0 + o->delta);
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++)
            st->P_f[a][b] = rho * st->u[a] * st->u[b] + (a == b ? rho * st->T : 0.0)
                          + st->sig_g[a][b] / o->ssig;
}

static int site_collide(const pgko *o, const double *gi, double er, double *go, site_state *st)
{
    site_moments(o, gi, er, st);
    double rho = st->rho;
    double lamES[3][3], lamF[3][3];
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
            double sig_f = st->sig_g[a][b] / o->ssig;                 /* sigma(f) */
            lamES[a][b] = (a == b ? st->T : 0.0) + o->b * sig_f / rho; /* theta_T I + b sigma/rho */
            /* gain term F = tau*(f^ES/tau + f^MB/tau1): a Gaussian mixture whose
               covariance (for a linear equilibrium) is the rate-weighted mean */
            lamF[a][b] = (o->tau1 * lamES[a][b] + (a == b ? o->tau * st->theta : 0.0))
                       / (o->tau + o->tau1);
        }
    double F[NQ];
    int rc;
    if (o->eq == EQ_F3) {
        double lam6[6] = {lamF[0][0], lamF[1][1], lamF[2][2], lamF[0][1], lamF[0][2], lamF[1][2]};
        rc = equilibrium(o, rho, st->u, lam6, F);
    } else {
        /* nonlinear equilibrium: combine the two targets at their rates */
        double l1[6] = {lamES[0][0], lamES[1][1], lamES[2][2], lamES[0][1], lamES[0][2], lamES[1][2]};
        double l2[6] = {st->theta, st->theta, st->theta, 0, 0, 0};
        double F1[NQ], F2[NQ];
        rc = equilibrium(o, rho, st->u, l1, F1);
        rc |= equilibrium(o, rho, st->u, l2, F2);
        for (int i = 0; i < NQ; i++) F[i] = (o->tau1 * F1[i] + o->tau * F2[i]) / (o->tau + o->tau1);
    }
    for (int i = 0; i < NQ; i++) go[i] = (1.0 - 2.0 * o->beta) * gi[i] + 2.0 * o->beta * F[i];
    return rc;
}

/* exported single-site collision for the algebraic pins:
 * in: g[41], rotational state er; out: g*[41], and
 * info[0..4] = rho, T, R, theta, a */
int pgko_collide_site(pgko *o, const double *g, double er, double *gout, double *info)
{
    site_state st;
    int rc = site_collide(o, g, er, gout, &st);
    info[0] = st.rho; info[1] = st.T; info[2] = st.R; info[3] = st.theta; info[4] = st.a;
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Streaming (pull) on the bcc grid with bounded x and y faces               */
/* ------------------------------------------------------------------------ */
/* Doubled coordinates: along each axis the corner sites (sublattice A) sit at
 * 2i and the body-centre sites (B) at 2i+1.  A bounded low face sits at
 * doubled coordinate -1/2, a high face at 2n - 1/2.  Faces are numbered
 * f = 2 axis + side (axis 0 = x, 1 = y; z is periodic). */
static void face_equilibrium(const pgko *o, int f, double *F)
{
    int a = f / 2, side = f % 2;
    double th = o->bc_th[a][side];
    double lam[6] = {th, th, th, 0, 0, 0};
    if (o->bc[a][side] == BC_WALL) {
        /* diffuse wall: F3 at unit density, scaled per column by the wall density */
        pgko_feq_f3(o->th0, o->w, &o->c[0][0], 1.0, o->bc_u[a][side], lam, F);
        return;
    }
    double tmp[NQ];
    if (o->eq == EQ_E2 && pgko_feq_e2(o->th0, o->w, &o->c[0][0], o->bc_rho[a][side], o->bc_u[a][side], lam, tmp) > 0) {
        memcpy(F, tmp, sizeof(tmp));
        return;
    }
    if (o->eq == EQ_F4) {
        pgko_feq_f4(o->th0, o->w, &o->c[0][0], o->bc_rho[a][side], o->bc_u[a][side], lam, F);
        return;
    }
    pgko_feq_f3(o->th0, o->w, &o->c[0][0], o->bc_rho[a][side], o->bc_u[a][side], lam, F);
}

/* floor(q/2) for a doubled coordinate */
static int half_floor(int q) { return q >= 0 ? q / 2 : -((-q + 1) / 2); }

/* The bounded face a doubled position q lies beyond, or -1 (a periodic axis
 * wraps instead).  A position beyond a bounded x face and a bounded y face at
 * once (a corner) belongs to the x face. */
static int beyond(const pgko *o, const int *q)
{
    for (int a = 0; a < 2; a++) {
        int n = a == 0 ? o->nx : o->ny;
        if (q[a] < 0 && o->bc[a][0] != BC_PERIODIC) return 2 * a;
        if (q[a] > 2 * n - 1 && o->bc[a][1] != BC_PERIODIC) return 2 * a + 1;
    }
    return -1;
}

/* Ghost column of a position q beyond face f: its cell coordinates along the
 * other in-plane axis b (y for x faces, x for y faces) and along z.  Along a
 * bounded axis b the coordinate is kept as it is, from -2 to n_b + 1 (a
 * corner column lies outside the grid), along a periodic one it wraps.
 * *ncol receives the number of columns of face f. */
static int column_of(const pgko *o, int f, const int *q, int *ncol)
{
    int b = 1 - f / 2;
    int nb = b == 0 ? o->nx : o->ny;
    int bounded = o->bc[b][0] != BC_PERIODIC;
    int width = bounded ? nb + 4 : nb;
    int hb = half_floor(q[b]);
    int ib = bounded ? hb + 2 : wrap(hb, nb);
    if (ncol) *ncol = width * o->nz;
    return wrap(half_floor(q[2]), o->nz) * width + ib;
}

/* Pull streaming.  A population that would be pulled from beyond a bounded
 * face comes from the boundary: for a diffuse wall it is rho_w F_i(1, u_w,
 * theta_w I) with rho_w fixed by zero net mass flux; for a Dirichlet face it
 * is F_i(rho_D, u_D, theta_D I).  The mass balance of a diffuse wall is kept
 * per ghost column of the position a population leaves to or arrives from
 * (both sublattices pooled). */
static void stream(pgko *o)
{
    int ns = o->ns;
    double Fb[4][NQ];
    double *rw[4] = {NULL, NULL, NULL, NULL};
    for (int f = 0; f < 4; f++) {
        int a = f / 2, side = f % 2;
        if (o->bc[a][side] == BC_PERIODIC) continue;
        face_equilibrium(o, f, Fb[f]);
        if (o->bc[a][side] != BC_WALL) continue;
        int ncol, q0[3] = {0, 0, 0};
        column_of(o, f, q0, &ncol);
        double *out = (double *)calloc(ncol, sizeof(double));
        double *in = (double *)calloc(ncol, sizeof(double));
        rw[f] = (double *)calloc(ncol, sizeof(double));
        for (int s = 0; s < ns; s++) {
            int sub, z, y, x;
            site_coords(o, s, &sub, &z, &y, &x);
            int p[3] = {2 * x + sub, 2 * y + sub, 2 * z + sub};
            for (int i = 0; i < NQ; i++) {
                /* outgoing: arrives beyond the wall */
                int d[3] = {p[0] + o->c2[i][0], p[1] + o->c2[i][1], p[2] + o->c2[i][2]};
                if (beyond(o, d) == f) out[column_of(o, f, d, NULL)] += o->gp[(size_t)i * ns + s];
                /* incoming: pulled from beyond the wall */
                int q[3] = {p[0] - o->c2[i][0], p[1] - o->c2[i][1], p[2] - o->c2[i][2]};
                if (beyond(o, q) == f) in[column_of(o, f, q, NULL)] += Fb[f][i];
            }
        }
        for (int k = 0; k < ncol; k++) rw[f][k] = in[k] > 0 ? out[k] / in[k] : 0.0;
        free(out); free(in);
    }
#pragma omp parallel for
    for (int s = 0; s < ns; s++) {
        int sub, z, y, x;
        site_coords(o, s, &sub, &z, &y, &x);
        int p[3] = {2 * x + sub, 2 * y + sub, 2 * z + sub};
        for (int i = 0; i < NQ; i++) {
            int q[3] = {p[0] - o->c2[i][0], p[1] - o->c2[i][1], p[2] - o->c2[i][2]};
            int f = beyond(o, q);
            double val;
            if (f >= 0) {
                if (o->bc[f / 2][f % 2] == BC_WALL) val = rw[f][column_of(o, f, q, NULL)] * Fb[f][i];
                else val = Fb[f][i];
            } else {
                int ssub = q[0] & 1;              /* all three share the parity */
                int sx = (q[0] - ssub) / 2, sy = (q[1] - ssub) / 2, sz = (q[2] - ssub) / 2;
                int src = site_index(o, ssub, wrap(sz, o->nz), wrap(sy, o->ny), wrap(sx, o->nx));
                val = o->gp[(size_t)i * ns + src];
            }
            o->g[(size_t)i * ns + s] = val;
        }
    }
    for (int f = 0; f < 4; f++) free(rw[f]);
}

/* ------------------------------------------------------------------------ */
/* Rotational energy transport (steps 2-4 of the theta_R split)              */
/* ------------------------------------------------------------------------ */
/* Neighbour of site s along axis a by +-1 on its own sublattice; across a
 * bounded face f it returns -1 - f (-1, -2: low, high x; -3, -4: low, high y). */
static int nb(const pgko *o, int s, int a, int dir)
{
    int sub, z, y, x;
    site_coords(o, s, &sub, &z, &y, &x);
    int co[3] = {x, y, z}, n[3] = {o->nx, o->ny, o->nz};
    co[a] += dir;
    if (a < 2 && co[a] < 0 && o->bc[a][0] != BC_PERIODIC) return -1 - 2 * a;
    if (a < 2 && co[a] >= n[a] && o->bc[a][1] != BC_PERIODIC) return -2 - 2 * a;
    co[a] = wrap(co[a], n[a]);
    return site_index(o, sub, co[2], co[1], co[0]);
}

/* theta_R held beyond the face that nb() returned as g < 0 */
static double face_theta(const pgko *o, int g) { int f = -1 - g; return o->bc_th[f / 2][f % 2]; }

static double kappaR(const pgko *o, double rho, double theta)
{
    /* kappa_R = k_r kappa_T, kappa_T = 5 p tau / (2B), p = rho theta */
    return o->kr * 5.0 * rho * theta * o->tau / (2.0 * o->B);
}

/* ghost values beyond a bounded face f next to site s_adj: the face's
 * temperature, with the site's own density at a wall */
typedef struct { double th, rho, kap; } ghost;

static ghost ghost_of(const pgko *o, int f, int s_adj)
{
    ghost g;
    int a = f / 2, side = f % 2;
    double rho = o->bc[a][side] == BC_WALL ? o->rho[s_adj] : o->bc_rho[a][side];
    g.rho = rho;
    g.th = o->bc_th[a][side];
    g.kap = kappaR(o, rho, g.th);
    return g;
}

/* Steps 2-4 of the theta_R split on the half-relaxed field theta_hat:
 *   2. MacCormack advection  d theta/dt + u.grad theta = 0 with u^n:
 *        predictor  theta* = theta_hat - sum_a u_a (theta_hat(x+e_a) - theta_hat(x))
 *        corrector  theta^mc = 1/2 [theta_hat + theta* - sum_a u_a (theta*(x) - theta*(x-e_a))]
 *   3. FTCS diffusion  d theta/dt = (2/(rho delta)) div(kappa_R grad theta):
 *        CN : flux form with face conductivities 1/2 (kappa(x) + kappa(x+e));
 *        LIT: D_R lap(theta) with D_R = 2 kappa_R/(rho delta) at the site (as printed);
 *   4. second half of the relaxation:
 *        CN : explicit complement of the first half, theta += (R - r), so that
 *             the exchange with the translational energy is exact;
 *        LIT: backward Euler (theta + X theta_T)/(1+X) (as printed). */
static void transport(pgko *o)
{
    int ns = o->ns;
    double *ts = o->e1, *tm = o->e2;
    const double *th = o->ehat;
#pragma omp parallel for
    for (int s = 0; s < ns; s++) {
        double adv = 0.0;
        for (int a = 0; a < 3; a++) {
            int p = nb(o, s, a, +1);
            double tp = (p >= 0) ? th[p] : face_theta(o, p);
            adv += o->u[3 * s + a] * (tp - th[s]);
        }
        ts[s] = th[s] - adv;
    }
#pragma omp parallel for
    for (int s = 0; s < ns; s++) {
        double adv = 0.0;
        for (int a = 0; a < 3; a++) {
            int m = nb(o, s, a, -1);
            double tmv = (m >= 0) ? ts[m] : face_theta(o, m);
            adv += o->u[3 * s + a] * (ts[s] - tmv);
        }
        tm[s] = 0.5 * (th[s] + ts[s] - adv);
    }
    /* diffusion in nsub equal FTCS sub-steps (ping-pong between tm and ts) */
    double *cur = tm, *nxt = ts;
    double frac = 1.0 / o->nsub;
    for (int it = 0; it < o->nsub; it++) {
        int last = it == o->nsub - 1;
#pragma omp parallel for
        for (int s = 0; s < ns; s++) {
            double k_s = kappaR(o, o->rho[s], o->theta[s]);
            double flux = 0.0, lap = 0.0;
            for (int a = 0; a < 3; a++)
                for (int dir = -1; dir <= 1; dir += 2) {
                    int q = nb(o, s, a, dir);
                    double tq, kq;
                    if (q >= 0) {
                        tq = cur[q];
                        kq = kappaR(o, o->rho[q], o->theta[q]);
                    } else {
                        ghost gh = ghost_of(o, -1 - q, s);
                        tq = gh.th;
                        kq = gh.kap;
                    }
                    flux += 0.5 * (k_s + kq) * (tq - cur[s]);
                    lap += tq - cur[s];
                }
            double tdif;
            if (o->variant == VAR_CN) tdif = cur[s] + frac * 2.0 * flux / (o->rho[s] * o->delta);
            else tdif = cur[s] + frac * 2.0 * k_s / (o->rho[s] * o->delta) * lap;
            if (!last) {
                nxt[s] = tdif;
            } else if (o->variant == VAR_CN) {
                o->er[s] = tdif + o->d[s];                            /* second half, CN */
            } else {
                o->er[s] = (tdif + o->X * o->T[s]) / (1.0 + o->X);    /* second half, as printed */
            }
        }
        double *t = cur; cur = nxt; nxt = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Time step                                                                */
/* ------------------------------------------------------------------------ */
/* Number of equal FTCS sub-steps that keeps the explicit diffusion stable:
 * FTCS needs 2 dim D_R dt <= dx^2 with D_R = 2 kappa_R/(rho delta)
 * = 5 k_r theta tau/(B delta); evaluated at 1.5 times the largest of theta0
 * and the face temperatures.  One sub-step is the printed scheme. */
static int diffusion_substeps(const pgko *o)
{
    int dim = (o->nx > 1) + (o->ny > 1) + (o->nz > 1);
    double th = o->th0;
    for (int f = 0; f < 4; f++)
        if (o->bc[f / 2][f % 2] != BC_PERIODIC && o->bc_th[f / 2][f % 2] > th) th = o->bc_th[f / 2][f % 2];
    double DR = o->delta > 0 ? 5.0 * o->kr * th * o->tau / (o->B * o->delta) : 0.0;
    int n = (int)ceil(2.0 * dim * DR * 1.5);
    return n < 1 ? 1 : n;
}

int pgko_substeps(pgko *o) { return diffusion_substeps(o); }

int pgko_step(pgko *o, long nsteps)
{
    int ns = o->ns;
    o->nsub = diffusion_substeps(o);
    for (long n = 0; n < nsteps; n++) {
        int fail = 0;
#pragma omp parallel for reduction(+ : fail)
        for (int s = 0; s < ns; s++) {
            double gi[NQ], go[NQ];
            for (int i = 0; i < NQ; i++) gi[i] = o->g[(size_t)i * ns + s];
            site_state st;
            if (site_collide(o, gi, o->er[s], go, &st)) fail++;
            for (int i = 0; i < NQ; i++) o->gp[(size_t)i * ns + s] = go[i];
            o->rho[s] = st.rho;
            for (int a = 0; a < 3; a++) o->u[3 * s + a] = st.u[a];
            o->T[s] = st.T;
            o->theta[s] = st.theta;
            o->ehat[s] = st.R;           /* theta_R after the first half relaxation */
            o->d[s] = st.R - st.r;       /* its increment, repeated by the CN second half */
        }
        if (fail) { o->e2_fail += fail; return -2; }
        stream(o);
        transport(o);
    }
    return 0;
}

/* f-moments of the current state (time level n, before the collision):
 * rho, u[3][ns], theta_T(f), theta_R, pressure tensor P(f) [6][ns]. */
int pgko_moments(pgko *o, double *rho, double *u, double *thT, double *thR, double *P)
{
    int ns = o->ns;
#pragma omp parallel for
    for (int s = 0; s < ns; s++) {
        double gi[NQ];
        for (int i = 0; i < NQ; i++) gi[i] = o->g[(size_t)i * ns + s];
        site_state st;
        site_moments(o, gi, o->er[s], &st);
        if (rho) rho[s] = st.rho;
        if (u) for (int a = 0; a < 3; a++) u[(size_t)a * ns + s] = st.u[a];
        if (thT) thT[s] = st.T;
        if (thR) thR[s] = st.r;
        if (P) {
            P[0 * (size_t)ns + s] = st.P_f[0][0];
            P[1 * (size_t)ns + s] = st.P_f[1][1];
            P[2 * (size_t)ns + s] = st.P_f[2][2];
            P[3 * (size_t)ns + s] = st.P_f[0][1];
            P[4 * (size_t)ns + s] = st.P_f[0][2];
            P[5 * (size_t)ns + s] = st.P_f[1][2];
        }
    }
    return 0;
}

/* mass, momentum and total energy  sum(rho), sum(rho u), sum(1/2 sum g c^2 + E_R) */
int pgko_conserved(pgko *o, double *out)
{
    int ns = o->ns;
    double m = 0, jx = 0, jy = 0, jz = 0, e = 0;
#pragma omp parallel for reduction(+ : m, jx, jy, jz, e)
    for (int s = 0; s < ns; s++) {
        double r = 0, j[3] = {0, 0, 0}, c2 = 0;
        for (int i = 0; i < NQ; i++) {
            double gi = o->g[(size_t)i * ns + s];
            r += gi;
            for (int a = 0; a < 3; a++) j[a] += gi * o->c[i][a];
            c2 += gi * (o->c[i][0] * o->c[i][0] + o->c[i][1] * o->c[i][1] + o->c[i][2] * o->c[i][2]);
        }
        double er = 0.5 * o->delta * r * o->er[s];   /* E_R = delta rho theta_R / 2 */
        m += r; jx += j[0]; jy += j[1]; jz += j[2]; e += 0.5 * c2 + er;
    }
    out[0] = m; out[1] = jx; out[2] = jy; out[3] = jz; out[4] = e;
    return 0;
}

/* raw state access for the pins (populations [41][ns] and the rotational field) */
void pgko_get_state(const pgko *o, double *g, double *er)
{
    if (g) memcpy(g, o->g, sizeof(double) * NQ * (size_t)o->ns);
    if (er) memcpy(er, o->er, sizeof(double) * (size_t)o->ns);
}

void pgko_set_state(pgko *o, const double *g, const double *er)
{
    if (g) memcpy(o->g, g, sizeof(double) * NQ * (size_t)o->ns);
    if (er) memcpy(o->er, er, sizeof(double) * (size_t)o->ns);
}
