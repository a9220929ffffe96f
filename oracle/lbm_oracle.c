/*
 * Plain FP64 CPU oracle of the lattice Boltzmann collide-and-stream step of
 * Latt, Coreixas & Beny, "Cross-platform programming model for many-core
 * lattice Boltzmann simulation" (arXiv:2010.11751).
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library. The GPU product path shares
 * no code, header, table or helper with it.
 *
 * Written for obviousness, not speed: one cell at a time, loops over the
 * discrete velocities, the paper's notation (f, f_out, pop, out, tmp, c_k,
 * t_k, k-bar), FP64 throughout. Build with -ffp-contract=off.
 *
 * Parity status of each part (what pins it lives in tests/test_oracle_*.py):
 *   lattice tables ............ pinned (isotropy identities, worked f_out_0 /
 *                               f_out_10 relation of Sec. 2.6)
 *   equilibrium, BGK, TRT ..... pinned (closed-form moments, Eq. symmetry_Ek,
 *                               conservation, fixed point, TRT->BGK limit,
 *                               Taylor-Green decay, Couette, Poiseuille)
 *   REG ....................... pinned (stress relation, w=1 -> equilibrium,
 *                               bulk knob reduces to single relaxation)
 *   moment-space models ....... pinned (relaxed moments of the output read
 *   (NW4, RM, HM, CM, CHM, K)   back by direct sums, worked f_out_0 / f_out_10
 *                               formula of Sec. 2.6, the identity of the
 *                               linear families at equal rates, Maxwellian
 *                               moments of the equilibrium, fixed point,
 *                               Taylor-Green decay)
 *   RR ........................ pinned (D3Q27 product-form equilibrium; the
 *                               Hermite coefficients of the output, recovered
 *                               by projection, follow the recursion in its
 *                               second-derivative form at every order). The
 *                               choice of this weighted recursive form for the
 *                               paper's RR is a reading of an absent reference.
 *   reference step, schemes ... pinned (np.roll brute force, bounce-back
 *                               permutation, mass conservation, schemes and
 *                               layouts agree bit for bit, shuffled order)
 *   per-cell reference step ... pinned (equals the whole-lattice reference
 *                               step cell by cell, bit for bit, in every
 *                               geometry, model and lattice)
 *   invariants ................ pinned (mass and kinetic energy of states
 *                               built from given rho and u fields equal
 *                               sum rho and 1/2 sum rho |u|^2 of those fields)
 *   curved walls .............. pinned (q = 1/2 is the half-way wall bit for
 *                               bit; plane Couette flow between walls at any
 *                               q is the exact straight line through the
 *                               wall positions; pull scheme = reference step)
 *   pressure walls ............ pinned (a fluid at rest at the walls' density
 *                               is a fixed point; a pressure-driven channel
 *                               takes the parabola of its density drop; the
 *                               schemes agree bit for bit)
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Configuration, as passed from Python (ctypes Structure of the same shape). */

enum { O_FLUID = 0, O_WALL = 1, O_LID = 2, O_PRESSURE = 3 };
enum { O_CAVITY = 0, O_PERIODIC = 1, O_CHANNEL = 2 };
enum { O_BGK = 0, O_TRT = 1, O_REG = 2, O_RR = 3,
       O_NW4 = 4, O_RM = 5, O_HM = 6, O_CM = 7, O_CHM = 8, O_K = 9 };
enum { O_SOA = 0, O_AOS = 1 };

typedef struct {
    int32_t q, nx, ny, nz;
    int32_t geometry; /* O_CAVITY, O_PERIODIC, O_CHANNEL                       */
    int32_t model;    /* O_BGK .. O_K                                          */
    int32_t layout;   /* O_SOA: pop[k][Ntot], O_AOS: pop[Ntot][Q]              */
    int32_t pad_;
    double omega;      /* shear relaxation frequency omega_nu                  */
    double trt_lambda; /* TRT "magic" parameter                                */
    double omega_bulk; /* bulk relaxation frequency omega_nu_b (REG, RR, MRT)  */
    double omega3;     /* third-order moments of the moment-space models       */
    double omega4;     /* fourth and higher orders of the moment-space models  */
    double u_lid[3];   /* velocity u_w of LID cells                            */
    double force[3];   /* test-only uniform body force; zero for the method    */
} ocfg;

/* ------------------------------------------------------------------------- */
/* Lattices (Sec. 2.1 refers to the textbook stencils; weights are the
 * standard D3Q19 / D3Q27 ones). Velocity order: first the velocities whose
 * first nonzero component is -1 (by number of nonzeros, then
 * lexicographically), then the rest velocity, then the negatives of the first
 * half in the same order; this is the order that puts c_0=(-1,0,0)=-c_10 as
 * the worked example of Sec. 2.6 requires. */

typedef struct {
    int q, rest;
    int c[27][3];
    double t[27];
    int opp[27];
} olat;

static const int Q19_HALF[9][3] = {
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 1}, {-1, 1, 0}, {0, -1, -1}, {0, -1, 1}};
static const int Q27_HALF[13][3] = {
    {-1, 0, 0}, {0, -1, 0}, {0, 0, -1},
    {-1, -1, 0}, {-1, 0, -1}, {-1, 0, 1}, {-1, 1, 0}, {0, -1, -1}, {0, -1, 1},
    {-1, -1, -1}, {-1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}};

static int make_lattice(int q, olat *L)
{
    int half, k, a;
    const int (*h)[3];
    if (q == 19) { half = 9; h = Q19_HALF; }
    else if (q == 27) { half = 13; h = Q27_HALF; }
    else return -1;
    L->q = q;
    L->rest = half;
    for (a = 0; a < 3; ++a) L->c[half][a] = 0;
    for (k = 0; k < half; ++k)
        for (a = 0; a < 3; ++a) {
            L->c[k][a] = h[k][a];
            L->c[k + half + 1][a] = -h[k][a];
        }
    for (k = 0; k < q; ++k) {
        int nnz = abs(L->c[k][0]) + abs(L->c[k][1]) + abs(L->c[k][2]);
        if (q == 19) L->t[k] = nnz == 0 ? 1.0 / 3.0 : nnz == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
        else L->t[k] = nnz == 0 ? 8.0 / 27.0 : nnz == 1 ? 2.0 / 27.0 : nnz == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
        L->opp[k] = k == half ? half : (k < half ? k + half + 1 : k - half - 1);
    }
    return 0;
}

/* Threads of the OpenMP loops (timing only; results do not depend on it). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_lattice(int q, int32_t *c, double *t, int32_t *opp)
{
    olat L;
    int k, a;
    if (make_lattice(q, &L)) return -1;
    for (k = 0; k < q; ++k) {
        for (a = 0; a < 3; ++a) c[3 * k + a] = L.c[k][a];
        t[k] = L.t[k];
        opp[k] = L.opp[k];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Indexing (Sec. 2.5): linear index i = (x*ny + y)*nz + z, z fastest.
 * Neighbour coordinates wrap modulo the box, which only matters for periodic
 * axes: in a cavity a fluid cell's neighbours are always inside the box. */

static int64_t cell_index(const ocfg *g, int64_t x, int64_t y, int64_t z)
{
    return (x * g->ny + y) * g->nz + z;
}

static void cell_xyz(const ocfg *g, int64_t i, int64_t *x, int64_t *y, int64_t *z)
{
    *x = i / ((int64_t)g->ny * g->nz);
    *y = (i % ((int64_t)g->ny * g->nz)) / g->nz;
    *z = i % g->nz;
}

static int64_t wrap(int64_t v, int64_t n) { return ((v % n) + n) % n; }

/* Index of the cell at x + s*c (s = +1 or -1). */
static int64_t neighbour(const ocfg *g, int64_t i, const int *c, int s)
{
    int64_t x, y, z;
    cell_xyz(g, i, &x, &y, &z);
    return cell_index(g, wrap(x + s * c[0], g->nx), wrap(y + s * c[1], g->ny),
                      wrap(z + s * c[2], g->nz));
}

static int64_t ntot(const ocfg *g) { return (int64_t)g->nx * g->ny * g->nz; }

/* Address of population k of cell i in the configured layout (Sec. 2.3). */
static int64_t at(const ocfg *g, int64_t i, int k)
{
    return g->layout == O_AOS ? i * g->q + k : (int64_t)k * ntot(g) + i;
}

int64_t oracle_neighbour_index(const ocfg *g, int64_t i, int k)
{
    olat L;
    if (make_lattice(g->q, &L)) return -1;
    return neighbour(g, i, L.c[k], +1);
}

/* ------------------------------------------------------------------------- */
/* Geometry. Cavity: fluid inside, one wall layer on every face, the whole
 * top layer z = nz-1 (edges and corners included) is the moving lid.
 * Periodic: every cell is fluid. Channel: periodic in x and y, a wall at
 * z = 0 and the lid at z = nz-1. */

void oracle_flags(const ocfg *g, uint8_t *flags)
{
    int64_t x, y, z;
    for (x = 0; x < g->nx; ++x)
        for (y = 0; y < g->ny; ++y)
            for (z = 0; z < g->nz; ++z) {
                uint8_t f = O_FLUID;
                if (g->geometry == O_CAVITY) {
                    int inside = x >= 1 && x <= g->nx - 2 && y >= 1 && y <= g->ny - 2 &&
                                 z >= 1 && z <= g->nz - 2;
                    if (!inside) f = (z == g->nz - 1) ? O_LID : O_WALL;
                } else if (g->geometry == O_CHANNEL) {
                    if (z == 0) f = O_WALL;
                    else if (z == g->nz - 1) f = O_LID;
                }
                flags[cell_index(g, x, y, z)] = f;
            }
}

/* Momentum-exchange term of Eq. momentum-exchange with rho_w = 1:
 * w_k = -6 t_k c_k . u_w, stored by wall cells (Eq. storage2). */
static double wall_term(const olat *L, const ocfg *g, uint8_t flag, int k)
{
    double uw[3] = {0.0, 0.0, 0.0};
    if (flag == O_LID) { uw[0] = g->u_lid[0]; uw[1] = g->u_lid[1]; uw[2] = g->u_lid[2]; }
    return -6.0 * L->t[k] * (L->c[k][0] * uw[0] + L->c[k][1] * uw[1] + L->c[k][2] * uw[2]);
}

/* Boundary extensions of the link-wise bounce-back (Sec. 1.1 notes that it
 * extends to curved walls while staying local; Eq. momentum-exchange has the
 * wall density rho_w).
 *
 * Pressure (density) walls: a cell of type O_PRESSURE reflects a population
 * with the opposite sign, f_kbar(x) = -f_out_k(x) + a_k, and stores
 * a_k = 2 t_k rho_w [1 + 9/2 (c_k . u_w)^2 - 3/2 |u_w|^2] in its slot k:
 * twice the even part of the equilibrium at (rho_w, u_w), so that the
 * density, not the velocity, is set at the half-way wall (anti-bounce-back).
 * Every bounce-back site reads the sign from the wall cell's type. */
static double reflected(uint8_t wall, double v) { return wall == O_PRESSURE ? -v : v; }

/* Curved walls: the wall crosses the link from fluid cell x to the wall cell
 * s = x - c_k at the fraction q of the link from x (0 < q <= 1; q = 1/2 is
 * the half-way wall). The population entering x in direction k is the linear
 * interpolated bounce-back, written with post-collision values only:
 *   q >= 1/2: [f_out_kbar(x) + (2q - 1) f_out_k(x) + w_kbar(s)] / (2q)
 *   q <  1/2: 2q f_out_kbar(x) + (1 - 2q) f_out_kbar(x + c_k) + w_kbar(s)
 * f_out_kbar(x + c_k) is the value that streams into x along the same line
 * from the other side (f_out_kbar(x) when x + c_k is not fluid). Both forms
 * give the half-way rule at q = 1/2, and both read only values that a cell
 * gathering its populations (the pull form) reads for itself. */
static double curved_link(double q, double fo_kbar_x, double fo_k_x, double fo_kbar_n, double w)
{
    if (q == 0.5) return fo_kbar_x + w;
    if (q > 0.5) return (fo_kbar_x + (2.0 * q - 1.0) * fo_k_x + w) / (2.0 * q);
    return 2.0 * q * fo_kbar_x + (1.0 - 2.0 * q) * fo_kbar_n + w;
}

/* ------------------------------------------------------------------------- */
/* Moments and equilibria. */

static void density_velocity(const olat *L, const double *f, double *rho, double u[3])
{
    int k, a;
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (k = 0; k < L->q; ++k) {
        r += f[k];
        for (a = 0; a < 3; ++a) j[a] += L->c[k][a] * f[k];
    }
    *rho = r;
    for (a = 0; a < 3; ++a) u[a] = j[a] / r;
}

/* BGK-W2 second-order weighted equilibrium (Sec. 2.6), with the |u|^2
 * coefficient 3/2 = 1/(2 c_s^2) that makes sum_k E_k = rho. */
static void equilibrium2(const olat *L, double rho, const double u[3], double *E)
{
    int k;
    double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (k = 0; k < L->q; ++k) {
        double cu = L->c[k][0] * u[0] + L->c[k][1] * u[1] + L->c[k][2] * u[2];
        E[k] = rho * L->t[k] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

/* Hermite machinery for the recursive-regularized model. A multi-index
 * n = (nx, ny, nz) with entries in {0,1,2}; per axis h_0 = 1, h_1(c) = c,
 * h_2(c) = c^2 - 1/3 (c_s^2 = 1/3); H_n(c) is the product over the axes and
 * its norm is N_n = nx! ny! nz! (1/3)^(nx+ny+nz). */
static double hermite_1d(int n, int c)
{
    return n == 0 ? 1.0 : n == 1 ? (double)c : (double)(c * c) - 1.0 / 3.0;
}

static double hermite(const int n[3], const int c[3])
{
    return hermite_1d(n[0], c[0]) * hermite_1d(n[1], c[1]) * hermite_1d(n[2], c[2]);
}

static double hermite_norm(const int n[3])
{
    double v = 1.0;
    int a, m;
    for (a = 0; a < 3; ++a)
        for (m = 0; m < n[a]; ++m) v *= (m + 1) / 3.0;
    return v;
}

/* Supported Hermite set S: all of {0,1,2}^3 on D3Q27; on D3Q19 every n of
 * order <= 2 plus the six permutations of (2,1,0). */
static int in_support(int q, const int n[3])
{
    int order = n[0] + n[1] + n[2];
    int twos = (n[0] == 2) + (n[1] == 2) + (n[2] == 2);
    int ones = (n[0] == 1) + (n[1] == 1) + (n[2] == 1);
    if (q == 27) return 1;
    if (order <= 2) return 1;
    return order == 3 && twos == 1 && ones == 1;
}

/* Equilibrium of the recursive-regularized model: the Hermite expansion of
 * the Maxwellian restricted to S, E_k = t_k rho sum_n H_n(c_k) u^n / N_n. */
static void equilibrium_rr(const olat *L, double rho, const double u[3], double *E)
{
    int k, n[3];
    for (k = 0; k < L->q; ++k) {
        double s = 0.0;
        for (n[0] = 0; n[0] <= 2; ++n[0])
            for (n[1] = 0; n[1] <= 2; ++n[1])
                for (n[2] = 0; n[2] <= 2; ++n[2]) {
                    if (!in_support(L->q, n)) continue;
                    s += hermite(n, L->c[k]) * pow(u[0], n[0]) * pow(u[1], n[1]) *
                         pow(u[2], n[2]) / hermite_norm(n);
                }
        E[k] = L->t[k] * rho * s;
    }
}

static void equilibrium_nw4(const olat *L, double rho, const double u[3], double *E);

void oracle_equilibrium(int q, int model, double rho, const double *u, double *E)
{
    olat L;
    if (make_lattice(q, &L)) return;
    if (model == O_RR) equilibrium_rr(&L, rho, u, E);
    else if (model >= O_NW4) equilibrium_nw4(&L, rho, u, E);
    else equilibrium2(&L, rho, u, E);
}

/* ------------------------------------------------------------------------- */
/* Collision models (Sec. 2.2, Sec. 2.6). */

/* TRT antisymmetric rate from the magic parameter
 * Lambda = (1/omega_plus - 1/2)(1/omega_minus - 1/2). */
static double trt_omega_minus(double omega_plus, double lambda)
{
    return 1.0 / (0.5 + lambda / (1.0 / omega_plus - 0.5));
}

/* Relaxed second-order non-equilibrium stress. The bulk-viscosity knob of
 * Eq. bulk, read with (M - M^eq) in place of the printed (M^eq - M^eq): the
 * deviatoric part relaxes with omega_nu, the trace with omega_nu_b. */
static void relaxed_stress(double omega, double omega_bulk, double P[3][3])
{
    int a, b;
    double tr3 = (P[0][0] + P[1][1] + P[2][2]) / 3.0;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) {
            double dev = P[a][b] - (a == b ? tr3 : 0.0);
            P[a][b] = (1.0 - omega) * dev + (a == b ? (1.0 - omega_bulk) * tr3 : 0.0);
        }
}

static void noneq_stress(const olat *L, const double *f, const double *E, double P[3][3])
{
    int k, a, b;
    for (a = 0; a < 3; ++a)
        for (b = 0; b < 3; ++b) P[a][b] = 0.0;
    for (k = 0; k < L->q; ++k)
        for (a = 0; a < 3; ++a)
            for (b = 0; b < 3; ++b) P[a][b] += L->c[k][a] * L->c[k][b] * (f[k] - E[k]);
}

/* Non-equilibrium Hermite coefficient a1_n for |n| >= 2 by the pair-sum
 * recursion: a1_{a1..am} = sum over pairs l<j of (prod of u over the other
 * indices) * Pi*_{al aj}; at order 2 this is just Pi*_{ab}. */
static double a1_coefficient(const int n[3], const double u[3], double P[3][3])
{
    int idx[6], m = 0, a, r, l, j;
    double s = 0.0;
    for (a = 0; a < 3; ++a)
        for (r = 0; r < n[a]; ++r) idx[m++] = a;
    for (l = 0; l < m; ++l)
        for (j = l + 1; j < m; ++j) {
            double prod = P[idx[l]][idx[j]];
            for (r = 0; r < m; ++r)
                if (r != l && r != j) prod *= u[idx[r]];
            s += prod;
        }
    return s;
}

/* ------------------------------------------------------------------------- */
/* Moment-space collision models (Sec. 2.2, Sec. 2.6): BGK with the
 * non-weighted fourth-order equilibrium (BGK-NW4), and the multi-relaxation-
 * time models in raw (RM), Hermite (HM), central (CM) and central Hermite
 * (CHM) moments and in cumulants (K), all in the non-weighted formulation:
 * a set of Q populations corresponds one-to-one with its Q moments over the
 * basis B of multi-indices n in {0,1,2}^3 whose monomial c^n does not vanish
 * on every lattice velocity (D3Q19: at most two nonzero entries, 19 indices;
 * D3Q27: all 27).
 *
 * Each moment family is a product over the axes of a polynomial p_{n_a}:
 *   raw              1, c,     c^2
 *   Hermite          1, c,     c^2 - c_s^2
 *   central          1, c - u, (c - u)^2
 *   central Hermite  1, c - u, (c - u)^2 - c_s^2
 * and X_n = (1/rho) sum_k P_n(c_k) f_k (Eq. RM, with the 1/rho the worked
 * f_out_0 example of Sec. 2.6 needs). The equilibria are the same moments of
 * the continuous Maxwellian (density 1, mean u, variance c_s^2 per axis):
 * raw 1, u, u^2 + c_s^2; Hermite 1, u, u^2; central 1, 0, c_s^2; central
 * Hermite 1, 0, 0 (products over the axes).
 *
 * Relaxation (Eq. RMcoll): X*_n = X_n - w_n (X_n - X^eq_n), with w = omega_nu
 * for the off-diagonal second-order moments, the mixing of Eq. bulk for the
 * diagonal ones, omega_3 at third order and omega_4 at orders four and up.
 * The cumulant model replaces the fourth-order central moments by the
 * cumulants C_220 = k_220 - k_200 k_020 - 2 k_110^2 (and permutations) and
 * relaxes those. The outgoing populations are the solution of
 * sum_k P_n(c_k) f_out_k = rho X*_n for every n in B. */

enum { FAM_RAW = 0, FAM_HERMITE = 1, FAM_CENTRAL = 2, FAM_CHERMITE = 3 };

static int moment_basis(int q, int nb[27][3])
{
    int a, b, e, n = 0;
    for (a = 0; a <= 2; ++a)
        for (b = 0; b <= 2; ++b)
            for (e = 0; e <= 2; ++e) {
                if (q == 19 && a > 0 && b > 0 && e > 0) continue;
                nb[n][0] = a;
                nb[n][1] = b;
                nb[n][2] = e;
                ++n;
            }
    return n;
}

static double axis_poly(int fam, int n, double c, double u)
{
    double x = (fam == FAM_CENTRAL || fam == FAM_CHERMITE) ? c - u : c;
    if (n == 0) return 1.0;
    if (n == 1) return x;
    return (fam == FAM_HERMITE || fam == FAM_CHERMITE) ? x * x - 1.0 / 3.0 : x * x;
}

static double axis_maxwellian(int fam, int n, double u)
{
    if (n == 0) return 1.0;
    switch (fam) {
    case FAM_RAW: return n == 1 ? u : u * u + 1.0 / 3.0;
    case FAM_HERMITE: return n == 1 ? u : u * u;
    case FAM_CENTRAL: return n == 1 ? 0.0 : 1.0 / 3.0;
    default: return 0.0;
    }
}

/* T[n][k] = P_n(c_k) of a family at velocity u. */
static void moment_matrix(const olat *L, int fam, const double u[3], int nb[27][3], int nm,
                          double T[27][27])
{
    int n, k, a;
    for (n = 0; n < nm; ++n)
        for (k = 0; k < L->q; ++k) {
            double v = 1.0;
            for (a = 0; a < 3; ++a) v *= axis_poly(fam, nb[n][a], L->c[k][a], u[a]);
            T[n][k] = v;
        }
}

/* Solve T x = b (m x m) by Gauss-Jordan elimination with partial pivoting. */
static void solve(int m, double T[27][27], const double *b, double *x)
{
    double A[27][28];
    int r, c, p;
    for (r = 0; r < m; ++r) {
        for (c = 0; c < m; ++c) A[r][c] = T[r][c];
        A[r][m] = b[r];
    }
    for (c = 0; c < m; ++c) {
        int piv = c;
        for (r = c + 1; r < m; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (piv != c)
            for (p = 0; p <= m; ++p) { double t = A[c][p]; A[c][p] = A[piv][p]; A[piv][p] = t; }
        for (r = 0; r < m; ++r) {
            double fct;
            if (r == c) continue;
            fct = A[r][c] / A[c][c];
            for (p = c; p <= m; ++p) A[r][p] -= fct * A[c][p];
        }
    }
    for (r = 0; r < m; ++r) x[r] = A[r][m] / A[r][r];
}

/* X*_n from X_n and X^eq_n for the orders and rates described above. */
static void relax_moments(const ocfg *g, int nb[27][3], int nm, const double *X, const double *Xeq,
                          double *Xs)
{
    double wm = (g->omega_bulk - g->omega) / 3.0, wp = wm + g->omega;
    int n, m, a;
    for (n = 0; n < nm; ++n) {
        int ord = nb[n][0] + nb[n][1] + nb[n][2];
        int diag = -1;
        for (a = 0; a < 3; ++a)
            if (nb[n][a] == 2 && ord == 2) diag = a;
        if (ord <= 1) {
            Xs[n] = X[n];
        } else if (diag >= 0) {
            /* Eq. bulk: X*_aa = X_aa - w+ (X_aa - eq) - w- sum_{b != a} (X_bb - eq) */
            Xs[n] = X[n] - wp * (X[n] - Xeq[n]);
            for (m = 0; m < nm; ++m) {
                int om = nb[m][0] + nb[m][1] + nb[m][2];
                if (m != n && om == 2 && (nb[m][0] == 2 || nb[m][1] == 2 || nb[m][2] == 2))
                    Xs[n] -= wm * (X[m] - Xeq[m]);
            }
        } else if (ord == 2) {
            Xs[n] = X[n] - g->omega * (X[n] - Xeq[n]);
        } else if (ord == 3) {
            Xs[n] = X[n] - g->omega3 * (X[n] - Xeq[n]);
        } else {
            Xs[n] = X[n] - g->omega4 * (X[n] - Xeq[n]);
        }
    }
}

static int find_index(int nb[27][3], int nm, int a, int b, int e)
{
    int n;
    for (n = 0; n < nm; ++n)
        if (nb[n][0] == a && nb[n][1] == b && nb[n][2] == e) return n;
    return -1;
}

/* BGK-NW4 equilibrium: the populations whose raw moments over B are the
 * Maxwellian ones. */
static void equilibrium_nw4(const olat *L, double rho, const double u[3], double *E)
{
    int nb[27][3], nm = moment_basis(L->q, nb), n, a;
    double T[27][27], Meq[27];
    double zero[3] = {0.0, 0.0, 0.0};
    moment_matrix(L, FAM_RAW, zero, nb, nm, T);
    for (n = 0; n < nm; ++n) {
        double v = rho;
        for (a = 0; a < 3; ++a) v *= axis_maxwellian(FAM_RAW, nb[n][a], u[a]);
        Meq[n] = v;
    }
    solve(nm, T, Meq, E);
}

static void collide_moment_space(const olat *L, const ocfg *g, double rho, const double u[3],
                                 const double *f, double *fout)
{
    int nb[27][3], nm = moment_basis(L->q, nb), n, k, a;
    double T[27][27], X[27], Xeq[27], Xs[27], b[27];
    int fam = g->model == O_HM ? FAM_HERMITE : g->model == O_CHM ? FAM_CHERMITE
            : (g->model == O_CM || g->model == O_K) ? FAM_CENTRAL : FAM_RAW;

    if (g->model == O_NW4) {
        double E[27];
        equilibrium_nw4(L, rho, u, E);
        for (k = 0; k < L->q; ++k) fout[k] = f[k] - g->omega * (f[k] - E[k]);
        return;
    }
    if (g->model == O_K && L->q != 19) {
        for (k = 0; k < L->q; ++k) fout[k] = NAN;
        return;
    }
    moment_matrix(L, fam, u, nb, nm, T);
    for (n = 0; n < nm; ++n) {
        double s = 0.0, e = 1.0;
        for (k = 0; k < L->q; ++k) s += T[n][k] * f[k];
        X[n] = s / rho;
        for (a = 0; a < 3; ++a) e *= axis_maxwellian(fam, nb[n][a], u[a]);
        Xeq[n] = e;
    }
    if (g->model == O_K) {
        /* Orders two and three: cumulants equal central moments. Order four
         * (D3Q19: 220, 202, 022): relax C = k_aabb - k_aa k_bb - 2 k_ab^2
         * towards 0 and rebuild k*_aabb from C* and the relaxed second order. */
        int p, axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        double Xtmp[27];
        ocfg g2 = *g;
        g2.omega4 = 0.0; /* fourth order handled below */
        relax_moments(&g2, nb, nm, X, Xeq, Xtmp);
        for (n = 0; n < nm; ++n) Xs[n] = Xtmp[n];
        for (p = 0; p < 3; ++p) {
            int d[3] = {0, 0, 0}, e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0}, o[3] = {0, 0, 0};
            int i4, i1, i2, io;
            double C, Cs;
            d[axes[p][0]] = 2; d[axes[p][1]] = 2;
            e1[axes[p][0]] = 2;
            e2[axes[p][1]] = 2;
            o[axes[p][0]] = 1; o[axes[p][1]] = 1;
            i4 = find_index(nb, nm, d[0], d[1], d[2]);
            i1 = find_index(nb, nm, e1[0], e1[1], e1[2]);
            i2 = find_index(nb, nm, e2[0], e2[1], e2[2]);
            io = find_index(nb, nm, o[0], o[1], o[2]);
            C = X[i4] - X[i1] * X[i2] - 2.0 * X[io] * X[io];
            Cs = (1.0 - g->omega4) * C;
            Xs[i4] = Cs + Xs[i1] * Xs[i2] + 2.0 * Xs[io] * Xs[io];
        }
    } else {
        relax_moments(g, nb, nm, X, Xeq, Xs);
    }
    for (n = 0; n < nm; ++n) b[n] = rho * Xs[n];
    solve(nm, T, b, fout);
}

static void collide(const olat *L, const ocfg *g, const double *f, double *fout)
{
    int k, a, b;
    double rho, u[3], E[27];
    density_velocity(L, f, &rho, u);

    if (g->model == O_BGK) {
        equilibrium2(L, rho, u, E);
        for (k = 0; k < L->q; ++k) fout[k] = f[k] - g->omega * (f[k] - E[k]);
    } else if (g->model == O_TRT) {
        double wp = g->omega, wm = trt_omega_minus(g->omega, g->trt_lambda);
        equilibrium2(L, rho, u, E);
        for (k = 0; k < L->q; ++k) {
            int kb = L->opp[k];
            double fp = 0.5 * (f[k] + f[kb]), fm = 0.5 * (f[k] - f[kb]);
            double ep = 0.5 * (E[k] + E[kb]), em = 0.5 * (E[k] - E[kb]);
            fout[k] = f[k] - wp * (fp - ep) - wm * (fm - em);
        }
    } else if (g->model == O_REG) {
        double P[3][3];
        equilibrium2(L, rho, u, E);
        noneq_stress(L, f, E, P);
        relaxed_stress(g->omega, g->omega_bulk, P);
        for (k = 0; k < L->q; ++k) {
            double s = 0.0;
            for (a = 0; a < 3; ++a)
                for (b = 0; b < 3; ++b)
                    s += (L->c[k][a] * L->c[k][b] - (a == b ? 1.0 / 3.0 : 0.0)) * P[a][b];
            fout[k] = E[k] + L->t[k] * 4.5 * s;
        }
    } else if (g->model >= O_NW4) {
        collide_moment_space(L, g, rho, u, f, fout);
    } else { /* O_RR */
        double P[3][3];
        int n[3];
        equilibrium_rr(L, rho, u, E);
        noneq_stress(L, f, E, P);
        relaxed_stress(g->omega, g->omega_bulk, P);
        for (k = 0; k < L->q; ++k) {
            double s = 0.0;
            for (n[0] = 0; n[0] <= 2; ++n[0])
                for (n[1] = 0; n[1] <= 2; ++n[1])
                    for (n[2] = 0; n[2] <= 2; ++n[2]) {
                        if (n[0] + n[1] + n[2] < 2 || !in_support(L->q, n)) continue;
                        s += hermite(n, L->c[k]) * a1_coefficient(n, u, P) / hermite_norm(n);
                    }
            fout[k] = E[k] + L->t[k] * s;
        }
    }

    /* Test-only body force (not part of the paper's method): first-order
     * source 3 t_k c_k . F added to the outgoing populations. */
    if (g->force[0] != 0.0 || g->force[1] != 0.0 || g->force[2] != 0.0)
        for (k = 0; k < L->q; ++k)
            fout[k] += 3.0 * L->t[k] *
                       (L->c[k][0] * g->force[0] + L->c[k][1] * g->force[1] +
                        L->c[k][2] * g->force[2]);
}

int oracle_collide(const ocfg *g, const double *f, double *fout)
{
    olat L;
    if (make_lattice(g->q, &L)) return -1;
    collide(&L, g, f, fout);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* State set-up: wall cells hold their momentum-exchange terms in every slot
 * (Eq. storage2; pressure cells their anti-bounce-back terms), fluid cells
 * hold E(rho, u) (Eq. storage1). rho and u may be
 * NULL (rho = 1, u = 0); u is given as u[3][Ntot]. The equilibrium is the
 * model's own (E^S for RR, the NW4 equilibrium for the moment-space models). */
int oracle_init_state_ex(const ocfg *g, const uint8_t *flags, const double *rho, const double *u,
                         const double *wall_u, const double *wall_rho, double *pop)
{
    olat L;
    int64_t i, n = ntot(g);
    int k;
    if (make_lattice(g->q, &L)) return -1;
    for (i = 0; i < n; ++i) {
        if (flags[i] != O_FLUID) {
            /* Eq. storage2 with the cell's own wall velocity and density when
             * given: -6 t_k rho_w c_k . u_w. */
            for (k = 0; k < L.q; ++k) {
                if (flags[i] == O_PRESSURE) {
                    double uw[3] = {0.0, 0.0, 0.0}, rw = wall_rho ? wall_rho[i] : 1.0, cu, uu;
                    if (wall_u) { uw[0] = wall_u[i]; uw[1] = wall_u[n + i]; uw[2] = wall_u[2 * n + i]; }
                    cu = L.c[k][0] * uw[0] + L.c[k][1] * uw[1] + L.c[k][2] * uw[2];
                    uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
                    pop[at(g, i, k)] = 2.0 * L.t[k] * rw * (1.0 + 4.5 * cu * cu - 1.5 * uu);
                } else if (wall_u || wall_rho) {
                    double uw[3] = {0.0, 0.0, 0.0}, rw = wall_rho ? wall_rho[i] : 1.0;
                    if (wall_u) { uw[0] = wall_u[i]; uw[1] = wall_u[n + i]; uw[2] = wall_u[2 * n + i]; }
                    pop[at(g, i, k)] = -6.0 * L.t[k] * rw *
                                       (L.c[k][0] * uw[0] + L.c[k][1] * uw[1] + L.c[k][2] * uw[2]);
                } else {
                    pop[at(g, i, k)] = wall_term(&L, g, flags[i], k);
                }
            }
        } else {
            double r = rho ? rho[i] : 1.0, v[3] = {0.0, 0.0, 0.0}, E[27];
            if (u) { v[0] = u[i]; v[1] = u[n + i]; v[2] = u[2 * n + i]; }
            if (g->model == O_RR) equilibrium_rr(&L, r, v, E);
            else if (g->model >= O_NW4) equilibrium_nw4(&L, r, v, E);
            else equilibrium2(&L, r, v, E);
            for (k = 0; k < L.q; ++k) pop[at(g, i, k)] = E[k];
        }
    }
    return 0;
}

int oracle_init_state(const ocfg *g, const uint8_t *flags, const double *rho,
                      const double *u, double *pop)
{
    return oracle_init_state_ex(g, flags, rho, u, NULL, NULL, pop);
}

/* ------------------------------------------------------------------------- */
/* Reference step, free of any memory-access scheme (Sec. 2.1):
 * collide every fluid cell, then every fluid cell x gathers population k from
 * its upstream neighbour s = x - c_k; if s is not fluid the link is bounced
 * back at the half-way wall, f_k(x) = f_out_kbar(x) + w_kbar(s)
 * (Eq. momentum-exchange with k and k-bar exchanged), w_kbar(s) being the
 * term the wall cell s stores in its slot k-bar (Eq. storage2); a pressure
 * cell reflects with the opposite sign, and a link with a wall distance
 * qlink[k][x] other than 1/2 takes the curved-wall rule (qlink may be NULL:
 * every wall half-way). The rest population stays. Wall cells keep their
 * stored terms. fnew must not alias f. */
int oracle_reference_step_ex(const ocfg *g, const uint8_t *flags, const double *f, const double *qlink,
                             double *fnew)
{
    olat L;
    int64_t i, n = ntot(g);
    double *fo;
    if (make_lattice(g->q, &L)) return -1;
    fo = (double *)malloc(sizeof(double) * (size_t)n * L.q);
    if (!fo) return -2;

#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        double cell[27], out[27];
        int k;
        if (flags[i] != O_FLUID) continue;
        for (k = 0; k < L.q; ++k) cell[k] = f[at(g, i, k)];
        collide(&L, g, cell, out);
        for (k = 0; k < L.q; ++k) fo[at(g, i, k)] = out[k];
    }

#pragma omp parallel for schedule(static)
    for (i = 0; i < n; ++i) {
        int k;
        if (flags[i] != O_FLUID) {
            for (k = 0; k < L.q; ++k) fnew[at(g, i, k)] = f[at(g, i, k)];
            continue;
        }
        for (k = 0; k < L.q; ++k) {
            int64_t s;
            if (k == L.rest) { fnew[at(g, i, k)] = fo[at(g, i, k)]; continue; }
            s = neighbour(g, i, L.c[k], -1);
            if (flags[s] == O_FLUID) {
                fnew[at(g, i, k)] = fo[at(g, s, k)];
            } else if (flags[s] == O_PRESSURE || !qlink) {
                fnew[at(g, i, k)] = reflected(flags[s], fo[at(g, i, L.opp[k])]) + f[at(g, s, L.opp[k])];
            } else {
                int64_t nb = neighbour(g, i, L.c[k], +1);
                double fo_n = flags[nb] == O_FLUID ? fo[at(g, nb, L.opp[k])] : fo[at(g, i, L.opp[k])];
                fnew[at(g, i, k)] = curved_link(qlink[(int64_t)k * n + i], fo[at(g, i, L.opp[k])],
                                                fo[at(g, i, k)], fo_n, f[at(g, s, L.opp[k])]);
            }
        }
    }
    free(fo);
    return 0;
}

int oracle_reference_step(const ocfg *g, const uint8_t *flags, const double *f, double *fnew)
{
    return oracle_reference_step_ex(g, flags, f, NULL, fnew);
}

/* The reference step for a list of cells only: new populations of cell
 * cells[j] written to fnew[j*Q + k]. Same definition as above, evaluated one
 * cell at a time so that large lattices can be checked on samples. */
int oracle_reference_cells(const ocfg *g, const uint8_t *flags, const double *f,
                           const int64_t *cells, int64_t ncells, double *fnew)
{
    olat L;
    int64_t j;
    if (make_lattice(g->q, &L)) return -1;
    for (j = 0; j < ncells; ++j) {
        int64_t i = cells[j];
        double cell[27], out[27], own[27];
        int k, m;
        if (flags[i] != O_FLUID) {
            for (k = 0; k < L.q; ++k) fnew[j * L.q + k] = f[at(g, i, k)];
            continue;
        }
        for (m = 0; m < L.q; ++m) cell[m] = f[at(g, i, m)];
        collide(&L, g, cell, own);
        for (k = 0; k < L.q; ++k) {
            int64_t s;
            if (k == L.rest) { fnew[j * L.q + k] = own[k]; continue; }
            s = neighbour(g, i, L.c[k], -1);
            if (flags[s] == O_FLUID) {
                for (m = 0; m < L.q; ++m) cell[m] = f[at(g, s, m)];
                collide(&L, g, cell, out);
                fnew[j * L.q + k] = out[k];
            } else {
                fnew[j * L.q + k] = reflected(flags[s], own[L.opp[k]]) + f[at(g, s, L.opp[k])];
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The three memory-access schemes of Table 1, executed on fluid cells in the
 * order given by `order` (a permutation of 0..Ntot-1; NULL = natural order).
 * Order independence is what makes them thread safe (Sec. 2.3). */

static int64_t pick(const int64_t *order, int64_t j) { return order ? order[j] : j; }

/* Double-population scheme: collide pop, stream into out; the caller then
 * exchanges the two arrays. Both arrays hold the wall terms in wall cells. */
int oracle_2pop_step(const ocfg *g, const uint8_t *flags, const double *pop, double *out,
                     const int64_t *order)
{
    olat L;
    int64_t j, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        int64_t i = pick(order, j);
        double cell[27], fo[27];
        int k;
        if (flags[i] != O_FLUID) continue;
        for (k = 0; k < L.q; ++k) cell[k] = pop[at(g, i, k)];
        collide(&L, g, cell, fo);
        for (k = 0; k < L.q; ++k) {
            int64_t nb;
            if (k == L.rest) { out[at(g, i, k)] = fo[k]; continue; }
            nb = neighbour(g, i, L.c[k], +1);
            if (flags[nb] == O_FLUID) out[at(g, nb, k)] = fo[k];              /* nb_out_k <- pop_k        */
            else out[at(g, i, L.opp[k])] = reflected(flags[nb], fo[k]) + pop[at(g, nb, k)]; /* out_kbar <- pop_k + nb_pop_k */
        }
    }
    return 0;
}

/* Swap algorithm, split into a collision sweep and a streaming sweep over the
 * nine (thirteen on D3Q27) directions k < rest. The wall cells' duty of the
 * Table 1 caption is read as an accumulation nb_pop_k += pop_kbar, which is
 * the only reading that keeps the fluid population it would otherwise
 * discard. */
int oracle_swap_step(const ocfg *g, const uint8_t *flags, double *pop, const int64_t *order)
{
    olat L;
    int64_t j, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;

#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        int64_t i = pick(order, j);
        double cell[27], fo[27];
        int k;
        if (flags[i] != O_FLUID) continue;
        for (k = 0; k < L.q; ++k) cell[k] = pop[at(g, i, k)];
        collide(&L, g, cell, fo);
        for (k = 0; k < L.q; ++k) pop[at(g, i, L.opp[k])] = fo[k];           /* pop_kbar <- Omega_k(pop) */
    }

#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        int64_t i = pick(order, j);
        int k;
        for (k = 0; k < L.rest; ++k) {
            int64_t nb = neighbour(g, i, L.c[k], +1);
            if (flags[i] == O_FLUID) {
                if (flags[nb] == O_FLUID) {                                  /* pop_kbar <-> nb_pop_k */
                    double tmp = pop[at(g, i, L.opp[k])];
                    pop[at(g, i, L.opp[k])] = pop[at(g, nb, k)];
                    pop[at(g, nb, k)] = tmp;
                } else {                                                     /* pop_kbar += nb_pop_k */
                    pop[at(g, i, L.opp[k])] = reflected(flags[nb], pop[at(g, i, L.opp[k])]) + pop[at(g, nb, k)];
                }
            } else if (flags[nb] == O_FLUID) {                               /* wall: nb_pop_k += pop_kbar */
                pop[at(g, nb, k)] = reflected(flags[i], pop[at(g, nb, k)]) + pop[at(g, i, L.opp[k])];
            }
        }
    }
    return 0;
}

/* AA-pattern. Even step: purely local, post-collision values at opposite
 * slots. Odd step: pull f_k(x) from pop_kbar(x - c_k) (the streaming equation
 * fixes the upstream cell), or pop_k(x) + pop_kbar(x - c_k) across a wall;
 * collide; push f_out_k to pop_k(x + c_k), or pop_kbar(x) <- f_out_k +
 * pop_k(x + c_k) across a wall. The rest population stays local. */
int oracle_aa_step(const ocfg *g, const uint8_t *flags, double *pop, int odd, const int64_t *order)
{
    olat L;
    int64_t j, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        int64_t i = pick(order, j);
        double tmp[27], fo[27];
        int k;
        if (flags[i] != O_FLUID) continue;
        if (!odd) {
            for (k = 0; k < L.q; ++k) tmp[k] = pop[at(g, i, k)];
            collide(&L, g, tmp, fo);
            for (k = 0; k < L.q; ++k) pop[at(g, i, L.opp[k])] = fo[k];
            continue;
        }
        for (k = 0; k < L.q; ++k) {
            int64_t s;
            if (k == L.rest) { tmp[k] = pop[at(g, i, k)]; continue; }
            s = neighbour(g, i, L.c[k], -1);
            if (flags[s] == O_FLUID) tmp[k] = pop[at(g, s, L.opp[k])];
            else tmp[k] = reflected(flags[s], pop[at(g, i, k)]) + pop[at(g, s, L.opp[k])];
        }
        collide(&L, g, tmp, fo);
        for (k = 0; k < L.q; ++k) {
            int64_t nb;
            if (k == L.rest) { pop[at(g, i, k)] = fo[k]; continue; }
            nb = neighbour(g, i, L.c[k], +1);
            if (flags[nb] == O_FLUID) pop[at(g, nb, k)] = fo[k];
            else pop[at(g, i, L.opp[k])] = reflected(flags[nb], fo[k]) + pop[at(g, nb, k)];
        }
    }
    return 0;
}

/* Double-population scheme in pull form (Table 1's 2Pop pushes instead).
 * Between steps both arrays hold post-collision values at opposite slots,
 * as the AA array after an even step; the entry step from a pre-collision
 * state is the AA even step. A step gathers f_k(x) from pop_kbar(x - c_k),
 * or pop_k(x) + pop_kbar(x - c_k) across a wall, collides, and stores f_out_k
 * at out_kbar(x); the caller then exchanges the arrays. Both arrays hold the
 * wall terms in wall cells. */
int oracle_pull_step_ex(const ocfg *g, const uint8_t *flags, const double *pop, const double *qlink, double *out,
                        const int64_t *order)
{
    olat L;
    int64_t j, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;
#pragma omp parallel for schedule(static)
    for (j = 0; j < n; ++j) {
        int64_t i = pick(order, j);
        double tmp[27], fo[27];
        int k;
        if (flags[i] != O_FLUID) continue;
        for (k = 0; k < L.q; ++k) {
            int64_t s;
            if (k == L.rest) { tmp[k] = pop[at(g, i, k)]; continue; }
            s = neighbour(g, i, L.c[k], -1);
            if (flags[s] == O_FLUID) {
                tmp[k] = pop[at(g, s, L.opp[k])];
            } else if (flags[s] == O_PRESSURE || !qlink) {
                tmp[k] = reflected(flags[s], pop[at(g, i, k)]) + pop[at(g, s, L.opp[k])];
            } else {  /* slot k of a cell holds f_out_kbar: see curved_link */
                int64_t nb = neighbour(g, i, L.c[k], +1);
                tmp[k] = curved_link(qlink[(int64_t)k * n + i], pop[at(g, i, k)], pop[at(g, i, L.opp[k])],
                                     pop[at(g, flags[nb] == O_FLUID ? nb : i, k)], pop[at(g, s, L.opp[k])]);
            }
        }
        collide(&L, g, tmp, fo);
        for (k = 0; k < L.q; ++k) out[at(g, i, L.opp[k])] = fo[k];
    }
    return 0;
}

int oracle_pull_step(const ocfg *g, const uint8_t *flags, const double *pop, double *out,
                     const int64_t *order)
{
    return oracle_pull_step_ex(g, flags, pop, NULL, out, order);
}

/* Natural pre-collision populations of an AA array left by an even step:
 * the odd-step pull without the collision. Wall cells copy their terms. */
int oracle_aa_natural_ex(const ocfg *g, const uint8_t *flags, const double *pop, const double *qlink, double *f)
{
    olat L;
    int64_t i, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;
    for (i = 0; i < n; ++i) {
        int k;
        for (k = 0; k < L.q; ++k) {
            int64_t s;
            if (flags[i] != O_FLUID || k == L.rest) { f[at(g, i, k)] = pop[at(g, i, k)]; continue; }
            s = neighbour(g, i, L.c[k], -1);
            if (flags[s] == O_FLUID) {
                f[at(g, i, k)] = pop[at(g, s, L.opp[k])];
            } else if (flags[s] == O_PRESSURE || !qlink) {
                f[at(g, i, k)] = reflected(flags[s], pop[at(g, i, k)]) + pop[at(g, s, L.opp[k])];
            } else {
                int64_t nb = neighbour(g, i, L.c[k], +1);
                f[at(g, i, k)] = curved_link(qlink[(int64_t)k * n + i], pop[at(g, i, k)], pop[at(g, i, L.opp[k])],
                                             pop[at(g, flags[nb] == O_FLUID ? nb : i, k)], pop[at(g, s, L.opp[k])]);
            }
        }
    }
    return 0;
}

int oracle_aa_natural(const ocfg *g, const uint8_t *flags, const double *pop, double *f)
{
    return oracle_aa_natural_ex(g, flags, pop, NULL, f);
}

/* ------------------------------------------------------------------------- */
/* Read-outs. Density and velocity of every fluid cell (0 on wall cells);
 * u is written as u[3][Ntot]. */
int oracle_macroscopic(const ocfg *g, const uint8_t *flags, const double *f, double *rho, double *u)
{
    olat L;
    int64_t i, n = ntot(g);
    if (make_lattice(g->q, &L)) return -1;
    for (i = 0; i < n; ++i) {
        double cell[27], r, v[3];
        int k;
        if (flags[i] != O_FLUID) { rho[i] = 0.0; u[i] = u[n + i] = u[2 * n + i] = 0.0; continue; }
        for (k = 0; k < L.q; ++k) cell[k] = f[at(g, i, k)];
        density_velocity(&L, cell, &r, v);
        rho[i] = r;
        u[i] = v[0]; u[n + i] = v[1]; u[2 * n + i] = v[2];
    }
    return 0;
}

/* Global mass sum_fluid sum_k f_k and kinetic energy 1/2 sum_fluid rho |u|^2,
 * accumulated in long double in index order. */
int oracle_invariants(const ocfg *g, const uint8_t *flags, const double *f, double *mass, double *ke)
{
    olat L;
    int64_t i, n = ntot(g);
    long double m = 0.0L, e = 0.0L;
    if (make_lattice(g->q, &L)) return -1;
    for (i = 0; i < n; ++i) {
        double cell[27], r, v[3];
        int k;
        if (flags[i] != O_FLUID) continue;
        for (k = 0; k < L.q; ++k) { cell[k] = f[at(g, i, k)]; m += cell[k]; }
        density_velocity(&L, cell, &r, v);
        e += 0.5L * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    }
    *mass = (double)m;
    *ke = (double)e;
    return 0;
}
