/*
 * FP64 CPU oracle for the D3Q19 lattice Boltzmann stream-collide update of
 * Bauer & Ruede, "An improved lattice Boltzmann D3Q19 method based on an
 * alternative equilibrium discretization" (arXiv:1803.04937).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library: every constant below is
 * written out here from the paper.
 *
 * Layout of every PDF array: dense structure of arrays, f[q * ncells + cell],
 * cell = (z * ny + y) * nx + x (x fastest).  All arithmetic is FP64.
 *
 * What each function follows:
 *   velocity sets, weights ....... Sec. 2.3 (D3Q19 and D3Q27 stencils, weights)
 *   standard equilibrium ......... Sec. 2.2, eq. discreteEquilibriumStandard,
 *                                  second-order part, rho0 from Sec. 2.3
 *   improved equilibrium ......... Sec. 3.2, eq. new_d3q19_equilibrium
 *   third-order D3Q19-I .......... Sec. 3.2 construction carried to O(u^3):
 *                                  the 19 kept Maxwellian moments, truncated
 *                                  at third order in u, solved for f^eq with
 *                                  the 19 x 19 moment matrix (Table 1, D3Q19-I
 *                                  column, lists these moments)
 *   D3Q27 equilibrium ............ Sec. 3.1: moment matching on D3Q27 gives
 *                                  the standard equilibrium with D3Q27
 *                                  weights, so D3Q27 uses that form
 *   forcing term ................. Sec. 2.3, F_q = w_q / c_s^2 c_q . a
 *   SRT update ................... Sec. 2.3, eq. lb_srt_with_forces
 *   macroscopic moments .......... Sec. 2.3, eqs. mass_conservation and
 *                                  macroscopic_vel_shift
 *   half-way bounce-back, periodic Sec. 5.1 (duct set-up)
 *   MRT collision ................ Sec. 3.2: C = -M^-1 S (M f - m_eq) in the
 *                                  space of the 19 kept monomial moments,
 *                                  m_eq = M f^eq (for D3Q19-I: the Maxwellian
 *                                  moments); rates: 2nd-order moments omega,
 *                                  3rd-order omega3, 4th-order omega4; force
 *                                  M^-1 (I - S/2) M F
 *   TRT collision ................ named in Sec. 1 and Sec. 3.3 but not
 *                                  defined there; the two-relaxation-time
 *                                  split into even and odd parts over
 *                                  opposite directions is used, with the
 *                                  force (odd) relaxed by omega_minus
 *   KBC collision ................ Sec. 3.3 (and the Re = 500 runs of
 *                                  Sec. 5.2): the entropic multi-relaxation
 *                                  collision of Karlin, Boesch and
 *                                  Chikatamarla (PRE 90, 031302, 2014; the
 *                                  KBC-N4 split of Boesch et al., PRE 92,
 *                                  043309, 2015) written in the 19 kept
 *                                  moments of Sec. 3.2 with the chosen
 *                                  equilibrium (Maxwellian moments for
 *                                  D3Q19-I), as Sec. 3.3 proposes
 *   inlet, outlet (Sec. 5.2) ..... open x faces: a prescribed inflow
 *                                  velocity by the moving-wall half-way
 *                                  bounce-back of Ladd (J. Fluid Mech. 271,
 *                                  285, 1994) and a constant outlet pressure
 *                                  by the anti-bounce-back of Ginzburg,
 *                                  Verhaeghe and d'Humieres (Commun. Comput.
 *                                  Phys. 3, 427, 2008)
 *   adjoint, objectives .......... not in the paper: the exact transpose of
 *                                  the discrete update above (SRT, TRT, MRT;
 *                                  periodic and wall boundaries)
 *
 * Parity pins: the test suite checks these functions against the moment
 * table of Sec. 3.1 (Table 1), an exact-rational moment-matching
 * construction from the Maxwellian moments (Sec. 3.1-3.2), streaming against
 * numpy.roll, conservation of mass and momentum, closed-form shear-wave
 * decay, the exact plane-Poiseuille solution, the duct projection property
 * behind Sec. 5.1, and finite differences for the adjoint.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NQ 27 /* array bound: D3Q27; D3Q19 uses the first 19 entries */

/* ------------------------------------------------------------------------ */
/* Velocity sets (Sec. 2.3).  Order: rest; the six axis directions; the      */
/* twelve edge directions (D3Q19 ends here); the eight corner directions     */
/* (D3Q27).  Opposite directions sit next to each other.                     */
/* ------------------------------------------------------------------------ */
static const int C[NQ][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1},
};

/* Number of directions of the configured stencil. */
#define QN(cfg) ((cfg)->stencil == 27 ? 27 : 19)

/* The direction with c_p = -c_q, found by search. */
static int opposite(int q)
{
    for (int p = 0; p < NQ; ++p)
        if (C[p][0] == -C[q][0] && C[p][1] == -C[q][1] && C[p][2] == -C[q][2]) return p;
    return -1;
}

typedef struct {
    int nx, ny, nz;
    int periodic[3];    /* 1: periodic axis; 0: half-way bounce-back walls   */
    int improved;       /* 0: D3Q19-S, 1: D3Q19-I, 2: D3Q19-I to O(u^3)     */
    int trt;            /* 0: SRT, 1: TRT                                    */
    int compressible;   /* 0: rho0 = 1 (the paper's choice), 1: rho0 = rho   */
    double omega;       /* SRT rate, or TRT even rate omega_plus             */
    double magic;       /* TRT Lambda = (1/w+ - 1/2)(1/w- - 1/2)             */
    double accel[3];    /* body acceleration a                               */
    int stencil;        /* 19 (D3Q19) or 27 (D3Q27)                          */
    int mrt;            /* 1: MRT (D3Q19), overrides trt                     */
    double omega3;      /* MRT rate of the third-order moments               */
    double omega4;      /* MRT rate of the fourth-order moments              */
    int kbc;            /* 1: KBC entropic collision (D3Q19), overrides the
                           others                                            */
    int kbc_fixed;      /* 0: entropic stabiliser; 1: the fixed value
                           kbc_gamma (for tests of the construction)         */
    double kbc_gamma;
    int open_x;         /* 1: inlet at the x = -1/2 face, outlet at x = nx - 1/2
                           (x must not be periodic); incompressible form     */
    double rho_out;     /* outlet density                                    */
    const double *inlet;/* inflow velocity [3][nz][ny] at the inlet cells    */
} oracle_cfg;

/* Weights by the squared length of c_q (Sec. 2.3).  D3Q19: 1/3, 1/18, 1/36.
 * D3Q27: 8/27, 2/27, 1/54, 1/216. */
static double weight_of(int stencil, int q)
{
    int n2 = C[q][0] * C[q][0] + C[q][1] * C[q][1] + C[q][2] * C[q][2];
    if (stencil == 27) {
        if (n2 == 0) return 8.0 / 27.0;
        if (n2 == 1) return 2.0 / 27.0;
        if (n2 == 2) return 1.0 / 54.0;
        return 1.0 / 216.0;
    }
    if (n2 == 0) return 1.0 / 3.0;
    if (n2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}
#define weight(q) weight_of(cfg->stencil, (q))

void oracle_velocity_set(int stencil, int *c_out, double *w_out, int *opp_out)
{
    int qn = stencil == 27 ? 27 : 19;
    for (int q = 0; q < qn; ++q) {
        for (int d = 0; d < 3; ++d) c_out[3 * q + d] = C[q][d];
        w_out[q] = weight_of(stencil, q);
        opp_out[q] = opposite(q);
    }
}

/* ------------------------------------------------------------------------ */
/* Equilibria, truncated at second order in u.                              */
/* ------------------------------------------------------------------------ */

/* Standard equilibrium: w rho + w rho0 [3 c_a u_a
 *                                      + 9/2 u_a u_b (c_a c_b - delta_ab/3)]. */
static double feq_standard(const oracle_cfg *cfg, int q, double rho, double rho0,
                           const double u[3])
{
    double first = 0.0, second = 0.0;
    for (int a = 0; a < 3; ++a) {
        first += C[q][a] * u[a];
        for (int b = 0; b < 3; ++b)
            second += u[a] * u[b] * (C[q][a] * C[q][b] - (a == b ? 1.0 / 3.0 : 0.0));
    }
    return weight(q) * rho + weight(q) * rho0 * (3.0 * first + 4.5 * second);
}

/* Improved equilibrium D3Q19-I, case by case on the type of c_q.  The edge
 * term -3/2 u_i^2 c_qi^2 is summed over i. */
static double feq_improved(const oracle_cfg *cfg, int q, double rho, double rho0,
                           const double u[3])
{
    int n2 = C[q][0] * C[q][0] + C[q][1] * C[q][1] + C[q][2] * C[q][2];
    double cu = 0.0, uu = 0.0, uc2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        cu += u[i] * C[q][i];
        uu += u[i] * u[i];
        uc2 += u[i] * u[i] * C[q][i] * C[q][i];
    }
    double bracket;
    if (n2 == 0)
        bracket = -uu;
    else if (n2 == 1)
        bracket = 3.0 * cu - 3.0 * uu + 6.0 * cu * cu;
    else
        bracket = 3.0 * cu - 1.5 * uc2 + 4.5 * cu * cu;
    return rho * weight(q) + weight(q) * rho0 * bracket;
}

/* Moment-matching construction (Sec. 3.1-3.2) at third order in u.  The
 * independent moments are xi_0^e0 xi_1^e1 xi_2^e2 with e_i in {0, 1, 2};
 * D3Q19 keeps the 19 that are not in eq. dropped_d3q19_moments. */
static int kept_exponents(int e[19][3])
{
    static const int dropped[8][3] = {{1, 2, 2}, {2, 1, 2}, {2, 2, 1}, {1, 1, 2},
                                      {1, 2, 1}, {2, 1, 1}, {1, 1, 1}, {2, 2, 2}};
    int n = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int is_dropped = 0;
                for (int k = 0; k < 8; ++k)
                    if (dropped[k][0] == a && dropped[k][1] == b && dropped[k][2] == c)
                        is_dropped = 1;
                if (!is_dropped) {
                    e[n][0] = a;
                    e[n][1] = b;
                    e[n][2] = c;
                    ++n;
                }
            }
    return n;
}

/* Inverse of the 19 x 19 moment matrix M[k][q] = prod_i c_qi^e_ki, by
 * Gauss-Jordan elimination with partial pivoting.  Computed by
 * oracle_prepare() before any parallel region reads it. */
static double Minv[19][19];
static int Mexp[19][3];
static int Minv_ready = 0;
static void moment_matrix_inverse(void)
{
    if (Minv_ready) return;
    kept_exponents(Mexp);
    double A[19][38];
    for (int k = 0; k < 19; ++k)
        for (int q = 0; q < 19; ++q) {
            double v = 1.0;
            for (int i = 0; i < 3; ++i)
                for (int t = 0; t < Mexp[k][i]; ++t) v *= C[q][i];
            A[k][q] = v;
            A[k][19 + q] = (k == q);
        }
    for (int col = 0; col < 19; ++col) {
        int piv = col;
        for (int r = col + 1; r < 19; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        for (int j = 0; j < 38; ++j) {
            double t = A[col][j];
            A[col][j] = A[piv][j];
            A[piv][j] = t;
        }
        double d = A[col][col];
        for (int j = 0; j < 38; ++j) A[col][j] /= d;
        for (int r = 0; r < 19; ++r)
            if (r != col) {
                double m = A[r][col];
                for (int j = 0; j < 38; ++j) A[r][j] -= m * A[col][j];
            }
    }
    for (int q = 0; q < 19; ++q)
        for (int k = 0; k < 19; ++k) Minv[q][k] = A[q][19 + k];
    Minv_ready = 1;
}

static double ipow(double x, int n)
{
    double r = 1.0;
    for (int i = 0; i < n; ++i) r *= x;
    return r;
}

/* Maxwellian moment of exponent e (variance c_s^2 = 1/3), truncated at
 * O(u^3): product of the one-dimensional moments 1, u, u^2 + 1/3, the
 * velocity-free part times rho, every other term times rho0. */
static void moment_coefs(const int e[3], double coef[3][3])
{
    /* coef[axis][power]: the one-dimensional moment of exponent e[axis] is
     * sum_power coef * u^power. */
    for (int i = 0; i < 3; ++i) {
        coef[i][0] = e[i] == 0 ? 1.0 : (e[i] == 2 ? 1.0 / 3.0 : 0.0);
        coef[i][1] = e[i] == 1 ? 1.0 : 0.0;
        coef[i][2] = e[i] == 2 ? 1.0 : 0.0;
    }
}

static double maxwellian_moment3(const int e[3], double rho, double rho0, const double u[3])
{
    double coef[3][3];
    moment_coefs(e, coef);
    double free = coef[0][0] * coef[1][0] * coef[2][0];
    double rest = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                if (a + b + c == 0 || a + b + c > 3) continue;
                rest += coef[0][a] * coef[1][b] * coef[2][c] * ipow(u[0], a) * ipow(u[1], b) *
                        ipow(u[2], c);
            }
    return free * rho + rest * rho0;
}

/* d/du_d of the moment above at fixed rho, rho0: the derivative of each
 * retained monomial u0^a u1^b u2^c. */
static double dmaxwellian_moment3_du(const int e[3], double rho0, const double u[3], int d)
{
    double coef[3][3];
    moment_coefs(e, coef);
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                int pw[3] = {a, b, c};
                if (a + b + c == 0 || a + b + c > 3 || pw[d] == 0) continue;
                double t = coef[0][a] * coef[1][b] * coef[2][c];
                for (int i = 0; i < 3; ++i)
                    t *= i == d ? pw[i] * ipow(u[i], pw[i] - 1) : ipow(u[i], pw[i]);
                s += t;
            }
    return s * rho0;
}

/* All 19 values f^eq = M^-1 m(rho, u). */
static void feq_improved3_all(double rho, double rho0, const double u[3], double out[19])
{
    double m[19];
    for (int k = 0; k < 19; ++k) m[k] = maxwellian_moment3(Mexp[k], rho, rho0, u);
    for (int q = 0; q < 19; ++q) {
        double v = 0.0;
        for (int k = 0; k < 19; ++k) v += Minv[q][k] * m[k];
        out[q] = v;
    }
}

static double feq(const oracle_cfg *cfg, int q, double rho, double rho0, const double u[3])
{
    if (cfg->stencil != 27 && cfg->improved == 2) {
        double all[19];
        feq_improved3_all(rho, rho0, u, all);
        return all[q];
    }
    if (cfg->stencil == 27) return feq_standard(cfg, q, rho, rho0, u);
    return cfg->improved ? feq_improved(cfg, q, rho, rho0, u) : feq_standard(cfg, q, rho, rho0, u);
}

static void feq_all(const oracle_cfg *cfg, double rho, double rho0, const double u[3],
                    double out[NQ])
{
    if (cfg->stencil != 27 && cfg->improved == 2) {
        feq_improved3_all(rho, rho0, u, out);
        return;
    }
    for (int q = 0; q < QN(cfg); ++q) out[q] = feq(cfg, q, rho, rho0, u);
}

/* d f^eq_q / d u_b at fixed rho and rho0, differentiated by hand from the two
 * forms above. */
static double dfeq_du(const oracle_cfg *cfg, int q, int b, double rho0, const double u[3])
{
    double cu = 0.0;
    for (int i = 0; i < 3; ++i) cu += u[i] * C[q][i];
    double cb = C[q][b];
    if (!cfg->improved || cfg->stencil == 27)
        return weight(q) * rho0 * (3.0 * cb + 9.0 * cu * cb - 3.0 * u[b]);
    int n2 = C[q][0] * C[q][0] + C[q][1] * C[q][1] + C[q][2] * C[q][2];
    if (n2 == 0) return weight(q) * rho0 * (-2.0 * u[b]);
    if (n2 == 1) return weight(q) * rho0 * (3.0 * cb - 6.0 * u[b] + 12.0 * cu * cb);
    return weight(q) * rho0 * (3.0 * cb - 3.0 * u[b] * cb * cb + 9.0 * cu * cb);
}

/* d f^eq_q / d u_b for all q: the hand-differentiated forms above, or for the
 * third-order D3Q19-I, M^-1 times the derivatives of its moments. */
static void dfeq_du_all(const oracle_cfg *cfg, double rho0, const double u[3], double D[NQ][3])
{
    if (cfg->stencil != 27 && cfg->improved == 2) {
        double dm[19][3];
        for (int k = 0; k < 19; ++k)
            for (int b = 0; b < 3; ++b) dm[k][b] = dmaxwellian_moment3_du(Mexp[k], rho0, u, b);
        for (int q = 0; q < 19; ++q)
            for (int b = 0; b < 3; ++b) {
                double v = 0.0;
                for (int k = 0; k < 19; ++k) v += Minv[q][k] * dm[k][b];
                D[q][b] = v;
            }
        return;
    }
    for (int q = 0; q < QN(cfg); ++q)
        for (int b = 0; b < 3; ++b) D[q][b] = dfeq_du(cfg, q, b, rho0, u);
}

/* Serial set-up before any parallel region (the third-order construction's
 * moment-matrix inverse). */
static void oracle_prepare(void) { moment_matrix_inverse(); }

void oracle_feq(const oracle_cfg *cfg, double rho, double rho0, const double *u, double *out)
{
    oracle_prepare();
    feq_all(cfg, rho, rho0, u, out);
}

void oracle_dfeq_du(const oracle_cfg *cfg, double rho0, const double *u, double *out /*[Q][3]*/)
{
    oracle_prepare();
    double D[NQ][3];
    dfeq_du_all(cfg, rho0, u, D);
    for (int q = 0; q < QN(cfg); ++q)
        for (int b = 0; b < 3; ++b) out[3 * q + b] = D[q][b];
}

/* Forcing term F_q = w_q / c_s^2 (c_q . a), c_s^2 = 1/3. */
static double force_term(const oracle_cfg *cfg, int q)
{
    double ca = 0.0;
    for (int d = 0; d < 3; ++d) ca += C[q][d] * cfg->accel[d];
    return weight(q) / (1.0 / 3.0) * ca;
}

/* MRT rate of kept moment k (Sec. 3.2): the conserved moments (order 0, 1)
 * relax at 1, which leaves them unchanged; order 2 at omega (the viscosity),
 * order 3 at omega3, order 4 at omega4. */
static double mrt_rate(const oracle_cfg *cfg, int k)
{
    int order = Mexp[k][0] + Mexp[k][1] + Mexp[k][2];
    return order <= 1 ? 1.0 : (order == 2 ? cfg->omega : (order == 3 ? cfg->omega3 : cfg->omega4));
}

/* TRT odd rate from Lambda = (1/w+ - 1/2)(1/w- - 1/2). */
static double omega_minus(const oracle_cfg *cfg)
{
    if (!cfg->trt) return cfg->omega;
    double tau_plus = 1.0 / cfg->omega - 0.5;
    return 1.0 / (0.5 + cfg->magic / tau_plus);
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                          */
/* ------------------------------------------------------------------------ */

static int64_t ncells_of(const oracle_cfg *cfg)
{
    return (int64_t)cfg->nx * cfg->ny * cfg->nz;
}

/* Cell index of x + s*c_q, or -1 if it lies outside a wall axis. */
static int64_t shifted_cell(const oracle_cfg *cfg, int x, int y, int z, int q, int s)
{
    int p[3] = {x + s * C[q][0], y + s * C[q][1], z + s * C[q][2]};
    int n[3] = {cfg->nx, cfg->ny, cfg->nz};
    for (int d = 0; d < 3; ++d) {
        if (p[d] < 0 || p[d] >= n[d]) {
            if (!cfg->periodic[d]) return -1;
            p[d] = ((p[d] % n[d]) + n[d]) % n[d];
        }
    }
    return ((int64_t)p[2] * cfg->ny + p[1]) * cfg->nx + p[0];
}

static int is_solid(const uint8_t *solid, int64_t cell)
{
    return cell < 0 || (solid != NULL && solid[cell] != 0);
}

static void feq_all(const oracle_cfg *cfg, double rho, double rho0, const double u[3],
                    double out[NQ]);

/* Pull gather with half-way bounce-back: g_q(x) = f_q(x - c_q), or
 * f_qbar(x) when x - c_q is a wall or a solid cell.  With open x faces, a
 * source beyond the inlet face (x - c_qx < 0) gives the moving-wall
 * bounce-back g_q = f_qbar(x) + 6 w_q c_q . u_in (the wall term of a wall
 * moving at the inflow velocity of the cell's row, rho0 = 1), and a source
 * beyond the outlet face gives the anti-bounce-back
 * g_q = -f_qbar(x) + 2 f^eq+_q(rho_out, u_b), with f^eq+ the even part of
 * the equilibrium, (f^eq_q + f^eq_qbar) / 2, and u_b the velocity of the
 * cell's own stored state (read-out sum_q c_q f_q(x) - a/2). */
static void gather(const oracle_cfg *cfg, const uint8_t *solid, const double *f,
                   int x, int y, int z, double g[NQ])
{
    int64_t n = ncells_of(cfg);
    int64_t here = ((int64_t)z * cfg->ny + y) * cfg->nx + x;
    double ub[3] = {0.0, 0.0, 0.0}, fe[NQ];
    int outlet_cell = cfg->open_x && x == cfg->nx - 1;
    if (outlet_cell) {
        for (int q = 0; q < QN(cfg); ++q)
            for (int d = 0; d < 3; ++d) ub[d] += C[q][d] * f[(int64_t)q * n + here];
        for (int d = 0; d < 3; ++d) ub[d] -= 0.5 * cfg->accel[d];
        feq_all(cfg, cfg->rho_out, 1.0, ub, fe);
    }
    for (int q = 0; q < QN(cfg); ++q) {
        int qb = opposite(q);
        int px = x - C[q][0];
        if (cfg->open_x && px < 0) {
            const double *uin = cfg->inlet;
            int64_t row = (int64_t)z * cfg->ny + y, nyz = (int64_t)cfg->ny * cfg->nz;
            double cu = 0.0;
            for (int d = 0; d < 3; ++d) cu += C[q][d] * uin[d * nyz + row];
            g[q] = f[(int64_t)qb * n + here] + 6.0 * weight(q) * cu;
            continue;
        }
        if (cfg->open_x && px >= cfg->nx) {
            g[q] = -f[(int64_t)qb * n + here] + (fe[q] + fe[qb]);
            continue;
        }
        int64_t src = shifted_cell(cfg, x, y, z, q, -1);
        if (is_solid(solid, src))
            g[q] = f[(int64_t)qb * n + here];
        else
            g[q] = f[(int64_t)q * n + src];
    }
}

/* rho, and the equilibrium velocity u = (sum_q c_q g_q + a/2) / rho0'. */
static void macroscopic(const oracle_cfg *cfg, const double g[NQ], double *rho, double *rho0,
                        double u[3])
{
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < QN(cfg); ++q) {
        r += g[q];
        for (int d = 0; d < 3; ++d) j[d] += C[q][d] * g[q];
    }
    *rho = r;
    *rho0 = cfg->compressible ? r : 1.0;
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * cfg->accel[d]) / *rho0;
}

static double monomial(int k, int q);

/* KBC collision of one cell (D3Q19).  The populations split by the 19 kept
 * monomial moments of Sec. 3.2 (moment k of f: m_k = sum_q M[k][q] f_q,
 * f_q = sum_k Minv[q][k] m_k) into a kinematic part (orders 0 and 1: mass
 * and momentum), a shear part s (orders 2 and 3: the stress tensor with its
 * trace and the third-order moments, the KBC-N4 choice) and a higher-order
 * part h (order 4).  With beta = omega / 2 and the parts of the
 * non-equilibrium g - f^eq written ds and dh,
 *   f*_q = g_q - beta (2 ds_q + gamma dh_q) + force,
 * so s relaxes at omega (the viscosity) and h at gamma beta.  gamma
 * minimises the entropy H = sum f ln(f / w) of f* to second order about
 * f^eq, i.e. the entropic norm <X|X> with <X|Y> = sum_q X_q Y_q / f^eq_q,
 * over 0 <= gamma <= 2: the higher-order part relaxes at most as fast as
 * the shear part (the stabiliser only adds damping to it).  That norm is
 * quadratic in gamma, so the minimiser is the unconstrained one,
 *   gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>,
 * clamped to [0, 2]; gamma = 2 (the single-rate value) when <dh|dh> = 0.
 * (With rates gamma beta up to 2, perturbations of the moments that dh
 * barely contains grow from step to step where the rate comes close to 2.)
 * The force enters
 * as in the MRT form M^-1 (I - S/2) M F: its kinematic part whole (those
 * moments are not relaxed), its shear part times (1 - beta), its
 * higher-order part (zero: F is odd) times (1 - gamma beta / 2).  Returns
 * gamma. */
static double kbc_collide(const oracle_cfg *cfg, const double g[NQ], const double fe[NQ],
                          double out[NQ])
{
    double dm[19], mF[19];
    for (int k = 0; k < 19; ++k) {
        dm[k] = mF[k] = 0.0;
        for (int q = 0; q < 19; ++q) {
            dm[k] += monomial(k, q) * (g[q] - fe[q]);
            mF[k] += monomial(k, q) * force_term(cfg, q);
        }
    }
    double ds[NQ], dh[NQ], Fk[NQ], Fs[NQ], Fh[NQ];
    for (int q = 0; q < 19; ++q) {
        ds[q] = dh[q] = Fk[q] = Fs[q] = Fh[q] = 0.0;
        for (int k = 0; k < 19; ++k) {
            int order = Mexp[k][0] + Mexp[k][1] + Mexp[k][2];
            if (order <= 1) {
                Fk[q] += Minv[q][k] * mF[k];
            } else if (order <= 3) {
                ds[q] += Minv[q][k] * dm[k];
                Fs[q] += Minv[q][k] * mF[k];
            } else {
                dh[q] += Minv[q][k] * dm[k];
                Fh[q] += Minv[q][k] * mF[k];
            }
        }
    }
    double beta = 0.5 * cfg->omega, sh = 0.0, hh = 0.0;
    for (int q = 0; q < 19; ++q) {
        sh += ds[q] * dh[q] / fe[q];
        hh += dh[q] * dh[q] / fe[q];
    }
    double gamma;
    if (cfg->kbc_fixed)
        gamma = cfg->kbc_gamma;
    else if (hh != 0.0)
        gamma = fmin(fmax(1.0 / beta - (2.0 - 1.0 / beta) * sh / hh, 0.0), 2.0);
    else
        gamma = 2.0;
    for (int q = 0; q < 19; ++q)
        out[q] = g[q] - beta * (2.0 * ds[q] + gamma * dh[q]) + Fk[q] + (1.0 - beta) * Fs[q] +
                 (1.0 - 0.5 * gamma * beta) * Fh[q];
    return gamma;
}

/* Collision of one cell: post-collision f* from the gathered g. */
static void collide(const oracle_cfg *cfg, const double g[NQ], double out[NQ])
{
    double rho, rho0, u[3], fe[NQ];
    macroscopic(cfg, g, &rho, &rho0, u);
    feq_all(cfg, rho, rho0, u, fe);
    if (cfg->kbc) {
        kbc_collide(cfg, g, fe, out);
        return;
    }
    double w = cfg->omega;
    if (cfg->mrt) {
        /* m = M g, m_eq = M f^eq, F moments; relax moment k with its rate. */
        double m[19], meq[19], mF[19], mnew[19];
        for (int k = 0; k < 19; ++k) {
            m[k] = meq[k] = mF[k] = 0.0;
            for (int q = 0; q < 19; ++q) {
                double mk = 1.0;
                for (int i = 0; i < 3; ++i)
                    for (int t = 0; t < Mexp[k][i]; ++t) mk *= C[q][i];
                m[k] += mk * g[q];
                meq[k] += mk * fe[q];
                mF[k] += mk * force_term(cfg, q);
            }
            double s = mrt_rate(cfg, k);
            mnew[k] = m[k] - s * (m[k] - meq[k]) + (1.0 - s / 2.0) * mF[k];
        }
        for (int q = 0; q < 19; ++q) {
            double v = 0.0;
            for (int k = 0; k < 19; ++k) v += Minv[q][k] * mnew[k];
            out[q] = v;
        }
        return;
    }
    if (!cfg->trt) {
        for (int q = 0; q < QN(cfg); ++q)
            out[q] = g[q] - w * (g[q] - fe[q]) + (1.0 - w / 2.0) * force_term(cfg, q);
        return;
    }
    double wm = omega_minus(cfg);
    for (int q = 0; q < QN(cfg); ++q) {
        int qb = opposite(q);
        double gp = 0.5 * (g[q] + g[qb]), gm = 0.5 * (g[q] - g[qb]);
        double ep = 0.5 * (fe[q] + fe[qb]), em = 0.5 * (fe[q] - fe[qb]);
        out[q] = g[q] - w * (gp - ep) - wm * (gm - em) + (1.0 - wm / 2.0) * force_term(cfg, q);
    }
}

/* ------------------------------------------------------------------------ */
/* Public forward API                                                        */
/* ------------------------------------------------------------------------ */

/* KBC collision of one gathered state g (no streaming): post-collision
 * populations and the stabiliser gamma. */
double oracle_kbc_collide(const oracle_cfg *cfg, const double *g, double *out)
{
    oracle_prepare();
    double rho, rho0, u[3], fe[NQ], gg[NQ], o[NQ];
    for (int q = 0; q < 19; ++q) gg[q] = g[q];
    macroscopic(cfg, gg, &rho, &rho0, u);
    feq_all(cfg, rho, rho0, u, fe);
    double gamma = kbc_collide(cfg, gg, fe, o);
    for (int q = 0; q < 19; ++q) out[q] = o[q];
    return gamma;
}

/* f = f^eq(rho_init, u_init) in fluid cells, w_q in solid cells.
 * u_init is [3][cells]. */
void oracle_init(const oracle_cfg *cfg, const uint8_t *solid, const double *rho_init,
                 const double *u_init, double *f)
{
    oracle_prepare();
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        if (solid && solid[c]) {
            for (int q = 0; q < QN(cfg); ++q) f[q * n + c] = weight(q);
            continue;
        }
        double u[3] = {u_init[c], u_init[n + c], u_init[2 * n + c]};
        double rho = rho_init ? rho_init[c] : 1.0;
        double rho0 = cfg->compressible ? rho : 1.0;
        double fe[NQ];
        feq_all(cfg, rho, rho0, u, fe);
        for (int q = 0; q < QN(cfg); ++q) f[q * n + c] = fe[q];
    }
}

/* One two-grid pull step, fin -> fout.  Solid cells keep their values. */
void oracle_step(const oracle_cfg *cfg, const uint8_t *solid, const double *fin, double *fout)
{
    oracle_prepare();
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int z = 0; z < cfg->nz; ++z)
        for (int y = 0; y < cfg->ny; ++y)
            for (int x = 0; x < cfg->nx; ++x) {
                int64_t c = ((int64_t)z * cfg->ny + y) * cfg->nx + x;
                if (solid && solid[c]) {
                    for (int q = 0; q < QN(cfg); ++q) fout[q * n + c] = fin[q * n + c];
                    continue;
                }
                double g[NQ], out[NQ];
                gather(cfg, solid, fin, x, y, z, g);
                collide(cfg, g, out);
                for (int q = 0; q < QN(cfg); ++q) fout[q * n + c] = out[q];
            }
}

void oracle_run(const oracle_cfg *cfg, const uint8_t *solid, double *f, double *tmp, int nsteps)
{
    int64_t bytes = ncells_of(cfg) * QN(cfg) * (int64_t)sizeof(double);
    for (int s = 0; s < nsteps; ++s) {
        oracle_step(cfg, solid, f, tmp);
        memcpy(f, tmp, (size_t)bytes);
    }
}

/* Post-step values at selected cells only (for sampled checks on large
 * grids): out[k * 19 + q] = f*_q at cells[k]. */
void oracle_step_cells(const oracle_cfg *cfg, const uint8_t *solid, const double *fin,
                       const int64_t *cells, int64_t ncell_list, double *out)
{
    oracle_prepare();
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ncell_list; ++k) {
        int64_t c = cells[k];
        int x = (int)(c % cfg->nx), y = (int)((c / cfg->nx) % cfg->ny),
            z = (int)(c / ((int64_t)cfg->nx * cfg->ny));
        if (solid && solid[c]) {
            for (int q = 0; q < QN(cfg); ++q) out[k * QN(cfg) + q] = fin[q * n + c];
            continue;
        }
        double g[NQ];
        gather(cfg, solid, fin, x, y, z, g);
        collide(cfg, g, out + k * QN(cfg));
    }
}

/* Density and velocity of a stored post-collision state:
 * rho = sum f*, u = (sum c f* - a/2) / rho0'.  Solid cells report 0. */
void oracle_moments(const oracle_cfg *cfg, const uint8_t *solid, const double *f, double *rho,
                    double *u)
{
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        if (solid && solid[c]) {
            rho[c] = 0.0;
            for (int d = 0; d < 3; ++d) u[d * n + c] = 0.0;
            continue;
        }
        double r = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < QN(cfg); ++q) {
            r += f[q * n + c];
            for (int d = 0; d < 3; ++d) j[d] += C[q][d] * f[q * n + c];
        }
        double rho0 = cfg->compressible ? r : 1.0;
        rho[c] = r;
        for (int d = 0; d < 3; ++d) u[d * n + c] = (j[d] - 0.5 * cfg->accel[d]) / rho0;
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint (exact transpose of oracle_step); incompressible form, SRT, TRT   */
/* and MRT, periodic and wall boundaries.                                     */
/* ------------------------------------------------------------------------ */

/* Full 19x19 Jacobian J[q][r] = d f*_q / d g_r of the collision of one cell,
 * and the derivatives of f* with respect to omega and a. */
/* Moment k of direction q: c_q^e_k (the MRT moment matrix M[k][q]). */
static double monomial(int k, int q)
{
    double v = 1.0;
    for (int i = 0; i < 3; ++i)
        for (int t = 0; t < Mexp[k][i]; ++t) v *= C[q][i];
    return v;
}

/* MRT (Sec. 3.2) written on the populations: R = M^-1 S M, and its
 * derivative with respect to omega, P2 = M^-1 diag(order == 2) M. */
static void mrt_relaxation(const oracle_cfg *cfg, double R[NQ][NQ], double P2[NQ][NQ])
{
    for (int q = 0; q < 19; ++q)
        for (int r = 0; r < 19; ++r) {
            double v = 0.0, p2 = 0.0;
            for (int k = 0; k < 19; ++k) {
                int order = Mexp[k][0] + Mexp[k][1] + Mexp[k][2];
                double mk = Minv[q][k] * monomial(k, r);
                v += mk * mrt_rate(cfg, k);
                p2 += order == 2 ? mk : 0.0;
            }
            R[q][r] = v;
            P2[q][r] = p2;
        }
}

static void collision_jacobian(const oracle_cfg *cfg, const double g[NQ], double J[NQ][NQ],
                               double dw[NQ], double da[NQ][3])
{
    double rho, rho0, u[3], fe[NQ], D[NQ][3], dfe_dg[NQ][NQ];
    macroscopic(cfg, g, &rho, &rho0, u);
    feq_all(cfg, rho, rho0, u, fe);
    dfeq_du_all(cfg, rho0, u, D);
    /* With rho0 = 1: d rho / d g_r = 1, d u_b / d g_r = c_rb, d u_b / d a_b = 1/2. */
    for (int q = 0; q < QN(cfg); ++q)
        for (int r = 0; r < QN(cfg); ++r) {
            double v = weight(q);
            for (int b = 0; b < 3; ++b) v += D[q][b] * C[r][b];
            dfe_dg[q][r] = v;
        }
    double wp = cfg->omega, wm = omega_minus(cfg);
    /* Relaxation matrix R = wp P+ + wm P-, P+- = (I +- reversal) / 2, or the
     * MRT one. */
    double R[NQ][NQ], P2[NQ][NQ];
    if (cfg->mrt) {
        mrt_relaxation(cfg, R, P2);
    } else {
        for (int q = 0; q < QN(cfg); ++q)
            for (int s = 0; s < QN(cfg); ++s) {
                double pp = 0.5 * ((q == s) + (opposite(q) == s));
                double pm = 0.5 * ((q == s) - (opposite(q) == s));
                R[q][s] = cfg->trt ? wp * pp + wm * pm : wp * (q == s);
            }
    }
    for (int q = 0; q < QN(cfg); ++q)
        for (int r = 0; r < QN(cfg); ++r) {
            double v = (q == r) - R[q][r];
            for (int s = 0; s < QN(cfg); ++s) v += R[q][s] * dfe_dg[s][r];
            J[q][r] = v;
        }
    double fm = cfg->trt ? wm : wp; /* rate multiplying the force */
    for (int q = 0; q < QN(cfg); ++q) {
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int s = 0; s < QN(cfg); ++s) v += R[q][s] * 0.5 * D[s][b];
            if (cfg->mrt) {
                /* force term M^-1 (I - S/2) M F = (I - R/2) F, F_s = 3 w_s c_s.a */
                v += 3.0 * weight(q) * C[q][b];
                for (int s = 0; s < 19; ++s) v -= 0.5 * R[q][s] * 3.0 * weight(s) * C[s][b];
                da[q][b] = v;
            } else {
                da[q][b] = v + (1.0 - fm / 2.0) * 3.0 * weight(q) * C[q][b];
            }
        }
    }
    /* d f* / d omega.  For TRT, omega_minus follows omega through fixed Lambda;
     * for MRT only the second-order moments' rate moves: -P2 (g - f^eq + F/2). */
    for (int q = 0; q < QN(cfg); ++q) {
        int qb = opposite(q);
        if (cfg->mrt) {
            double v = 0.0;
            for (int s = 0; s < 19; ++s)
                v -= P2[q][s] * (g[s] - fe[s] + 0.5 * force_term(cfg, s));
            dw[q] = v;
        } else if (!cfg->trt) {
            dw[q] = -(g[q] - fe[q]) - 0.5 * force_term(cfg, q);
        } else {
            double gp = 0.5 * (g[q] + g[qb]), gm = 0.5 * (g[q] - g[qb]);
            double ep = 0.5 * (fe[q] + fe[qb]), em = 0.5 * (fe[q] - fe[qb]);
            double d_plus = -(gp - ep);
            double d_minus = -(gm - em) - 0.5 * force_term(cfg, q);
            double tau_p = 1.0 / wp - 0.5;
            double dwm_dwp = -wm * wm * cfg->magic / (tau_p * tau_p * wp * wp);
            dw[q] = d_plus + d_minus * dwm_dwp;
        }
    }
}

/* lam_prev = (d step / d f_t)^T lam_next.  grad[0] += dJ/domega,
 * grad[1..3] += dJ/da (the contribution of this step).  Every stencil and
 * equilibrium, SRT, TRT and MRT; returns -1 for the compressible form, the
 * KBC collision and open faces, which have no adjoint here. */
int oracle_adjoint_step(const oracle_cfg *cfg, const uint8_t *solid, const double *f_t,
                        const double *lam_next, double *lam_prev, double *grad)
{
    if (cfg->compressible || cfg->kbc || cfg->open_x) return -1;
    oracle_prepare();
    int64_t n = ncells_of(cfg);
    double *plane = (double *)calloc((size_t)cfg->nz * 4, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < cfg->nz; ++z) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int y = 0; y < cfg->ny; ++y)
            for (int x = 0; x < cfg->nx; ++x) {
                int64_t c = ((int64_t)z * cfg->ny + y) * cfg->nx + x;
                if (solid && solid[c]) {
                    for (int q = 0; q < QN(cfg); ++q) lam_prev[q * n + c] = lam_next[q * n + c];
                    continue;
                }
                double g[NQ], J[NQ][NQ], dw[NQ], da[NQ][3], lam[NQ];
                gather(cfg, solid, f_t, x, y, z, g);
                collision_jacobian(cfg, g, J, dw, da);
                for (int q = 0; q < QN(cfg); ++q) lam[q] = lam_next[q * n + c];
                for (int q = 0; q < QN(cfg); ++q) {
                    acc[0] += lam[q] * dw[q];
                    for (int b = 0; b < 3; ++b) acc[1 + b] += lam[q] * da[q][b];
                }
                /* mu = J^T lam, pushed back along the pull: g_r(x) was read
                 * from f_r(x - c_r), or from f_rbar(x) at a wall. */
                for (int r = 0; r < QN(cfg); ++r) {
                    double mu = 0.0;
                    for (int q = 0; q < QN(cfg); ++q) mu += J[q][r] * lam[q];
                    int64_t src = shifted_cell(cfg, x, y, z, r, -1);
                    if (is_solid(solid, src))
                        lam_prev[(int64_t)opposite(r) * n + c] = mu;
                    else
                        lam_prev[(int64_t)r * n + src] = mu;
                }
            }
        for (int k = 0; k < 4; ++k) plane[4 * z + k] = acc[k];
    }
    for (int z = 0; z < cfg->nz; ++z)
        for (int k = 0; k < 4; ++k) grad[k] += plane[4 * z + k];
    free(plane);
    return 0;
}

/* The adjoint of selected cells only (for sampled checks on large grids):
 * mu[k * Q + r] = sum_q J_C[q][r] lam_next_q(x) at the fluid cell x =
 * cells[k], the value oracle_adjoint_step pushes to lam_prev[r][x - c_r]
 * (or to lam_prev[rbar][x] when x - c_r is a wall or solid).  Solid cells
 * report lam_next (copied through).  Returns -1 where oracle_adjoint_step
 * does. */
int oracle_adjoint_cells(const oracle_cfg *cfg, const uint8_t *solid, const double *f_t,
                         const double *lam_next, const int64_t *cells, int64_t ncell_list,
                         double *mu_out)
{
    if (cfg->compressible || cfg->kbc || cfg->open_x) return -1;
    oracle_prepare();
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ncell_list; ++k) {
        int64_t c = cells[k];
        int x = (int)(c % cfg->nx), y = (int)((c / cfg->nx) % cfg->ny),
            z = (int)(c / ((int64_t)cfg->nx * cfg->ny));
        double *mu = mu_out + k * QN(cfg);
        if (solid && solid[c]) {
            for (int q = 0; q < QN(cfg); ++q) mu[q] = lam_next[q * n + c];
            continue;
        }
        double g[NQ], J[NQ][NQ], dw[NQ], da[NQ][3];
        gather(cfg, solid, f_t, x, y, z, g);
        collision_jacobian(cfg, g, J, dw, da);
        for (int r = 0; r < QN(cfg); ++r) {
            double v = 0.0;
            for (int q = 0; q < QN(cfg); ++q) v += J[q][r] * lam_next[q * n + c];
            mu[r] = v;
        }
    }
    return 0;
}

/* Objectives of a stored state and their seeds lam_T = dJ / d f.
 * kind 0: kinetic energy E = 1/2 sum over fluid cells of |u|^2.
 * kind 1: outlet flux, sum of u_x over fluid cells of the plane x = nx - 1.
 * u is the stored-state velocity of oracle_moments (rho0 = 1).  dJda gets
 * the explicit derivative with respect to a (through u = sum c f - a/2). */
double oracle_objective(const oracle_cfg *cfg, const uint8_t *solid, int kind, const double *f,
                        double *lam_seed, double *dJda)
{
    int64_t n = ncells_of(cfg);
    double J = 0.0, da[3] = {0.0, 0.0, 0.0};
    for (int64_t c = 0; c < n; ++c) {
        int fluid = !(solid && solid[c]);
        double u[3] = {0.0, 0.0, 0.0};
        if (fluid) {
            for (int q = 0; q < QN(cfg); ++q)
                for (int d = 0; d < 3; ++d) u[d] += C[q][d] * f[q * n + c];
            for (int d = 0; d < 3; ++d) u[d] -= 0.5 * cfg->accel[d];
        }
        int on_outlet = (int)(c % cfg->nx) == cfg->nx - 1;
        for (int q = 0; q < QN(cfg); ++q) {
            double s = 0.0;
            if (fluid && kind == 0)
                s = C[q][0] * u[0] + C[q][1] * u[1] + C[q][2] * u[2];
            else if (fluid && kind == 1 && on_outlet)
                s = C[q][0];
            if (lam_seed) lam_seed[q * n + c] = s;
        }
        if (!fluid) continue;
        if (kind == 0) {
            J += 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int d = 0; d < 3; ++d) da[d] += -0.5 * u[d];
        } else if (on_outlet) {
            J += u[0];
            da[0] += -0.5;
        }
    }
    if (dJda)
        for (int d = 0; d < 3; ++d) dJda[d] = da[d];
    return J;
}

/* Gradient with respect to u_init of the initial state f = f^eq(rho_init,
 * u_init): grad_u[b][x] = sum_q lam0_q(x) d f^eq_q / d u_b. */
int oracle_init_vjp(const oracle_cfg *cfg, const uint8_t *solid, const double *u_init,
                    const double *lam0, double *grad_u)
{
    oracle_prepare();
    int64_t n = ncells_of(cfg);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) {
        if (solid && solid[c]) {
            for (int b = 0; b < 3; ++b) grad_u[b * n + c] = 0.0;
            continue;
        }
        double u[3] = {u_init[c], u_init[n + c], u_init[2 * n + c]};
        double D[NQ][3];
        dfeq_du_all(cfg, 1.0, u, D);
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int q = 0; q < QN(cfg); ++q) v += lam0[q * n + c] * D[q][b];
            grad_u[b * n + c] = v;
        }
    }
    return 0;
}
