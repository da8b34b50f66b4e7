/*
 * oracle.c -- plain FP64 CPU oracle of one time step of the two-component
 * Shan-Chen lattice Boltzmann model on D3Q19 of Otomo et al., "Multi-component
 * lattice Boltzmann models for accurate simulation of flows with wide viscosity
 * variation" (arXiv:1711.03254), Section 2, Eqs. (1)-(11).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU baseline of
 * the benchmark do.  It shares no code, header, table or constant with the GPU
 * library: the lattice below is typed out here on its own.
 *
 * It is written for a reader holding the paper: every field is computed over
 * the whole lattice, one equation at a time, in the order Section 2 states
 * them, with no fusion, blocking or reordering.  Every floating-point value is
 * an IEEE double; the file is compiled without fused multiply-add and without
 * fast-math.  Loops over sites may run on several OpenMP threads; each site's
 * result is computed by one thread from read-only inputs, so results do not
 * depend on the thread count.
 *
 * Readings of the paper that this file fixes (the paper is silent or leaves a
 * choice open; each is listed with its reason in the design notes):
 *   - pseudo-potential psi = rho (Eq. 7 uses the densities themselves);
 *   - mixture weight p = rho_1 / rho in Eq. (6) (the density-weighted viscosity
 *     named for the layered Poiseuille comparison in Section 3.2);
 *   - forcing term (Section 2, "following Li et al. 2012"): the equilibrium is
 *     taken at the force-shifted velocity u_F of Eq. (8); the forcing term is
 *     Guo's, rewritten for the regularized non-equilibrium (forcing_term()):
 *     F_i = w_i (c_i . F) / (2 T0) + (1 - 1/(2 tau)) Phi : (u_F F + F u_F).
 *     The first moment of the post-collision populations is then rho u + F,
 *     so u_F is the average of the pre- and post-collision velocities, as
 *     Eq. (8) states; the second-order part gives the viscous stress
 *     rho nu (grad u + grad u^T) where the density varies (interfaces);
 *   - regularization Phi : Pi of Eq. (10): the second-order Hermite projection
 *     f'_i = w_i / (2 T0^2) (c_i c_i - T0 I) : Pi, with Pi the second moment of
 *     f - f_eq;
 *   - friction wall (Section 2, volumetric boundary): the voxel special case,
 *     halfway bounce-back on a solid mask;
 *   - wettability (Eq. 11): on solid sites rho'_beta is the wall density
 *     rho^s_beta, with rho^s_1 = max(-rho^s, 0) and rho^s_2 = max(rho^s, 0)
 *     from the single parameter rho^s (rho_0 = 1);
 *   - body force: a uniform acceleration g acting on each component as
 *     rho_alpha g (the gravity of Section 3.2);
 *   - the state held between steps is the post-streaming distribution
 *     f_i(x, t) of Eq. (1); sites are indexed s = x + nx (y + ny z) and the
 *     populations as f[(alpha * 19 + i) * N + s]; solid sites carry no
 *     populations (their entries are left at zero).
 *
 * Parity status of each exported function is stated next to it; all of them
 * are pinned by the CPU tests against closed forms, invariants and an
 * independent linear analysis (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Lattice temperature T0 = 1/3 (Section 2, after Eq. 3). */
static const double T0 = 1.0 / 3.0;

/* D3Q19 velocities (Qian et al. 1992, cited in Section 2): the rest velocity,
 * the six face neighbours and the twelve edge neighbours, in the fixed order
 * rest; +x -x +y -y +z -z; then the xy, xz and yz diagonals. */
static const int CV[Q][3] = {
    { 0, 0, 0},
    { 1, 0, 0}, {-1, 0, 0}, { 0, 1, 0}, { 0,-1, 0}, { 0, 0, 1}, { 0, 0,-1},
    { 1, 1, 0}, {-1,-1, 0}, { 1,-1, 0}, {-1, 1, 0},
    { 1, 0, 1}, {-1, 0,-1}, { 1, 0,-1}, {-1, 0, 1},
    { 0, 1, 1}, { 0,-1,-1}, { 0, 1,-1}, { 0,-1, 1},
};

/* Isotropic D3Q19 weights: 1/3 at rest, 1/18 for speed 1, 1/36 for speed
 * sqrt(2).  The weight follows from |c|^2, so it is computed, not tabulated. */
static double weight_of(int i)
{
    int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Index of the velocity opposite to c_i, found by search. */
static int opposite_of(int i)
{
    for (int j = 0; j < Q; ++j)
        if (CV[j][0] == -CV[i][0] && CV[j][1] == -CV[i][1] && CV[j][2] == -CV[i][2])
            return j;
    return -1;
}

/* Both are evaluated once for all 19 directions before first use. */
static double W_TABLE[Q];
static int OPP_TABLE[Q];
static int tables_ready = 0;
static void make_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) { W_TABLE[i] = weight_of(i); OPP_TABLE[i] = opposite_of(i); }
    tables_ready = 1;
}
static double weight(int i) { return W_TABLE[i]; }
static int opposite(int i) { return OPP_TABLE[i]; }

typedef struct {
    int32_t nx, ny, nz;
    int32_t eq_kind;     /* 0: Eq. (3) as printed; 1: with the second-order terms */
    int32_t force_kind;  /* 0: forcing with its second-order part (default); 1: first order only */
    int32_t wall_kind;   /* 0: wall force as Eq. (11) gives it (W1); 1: minus its share of the
                            mixture's net wall force (W2) */
    double tau[2];       /* tau_alpha > 1/2; nu_alpha = T0 (tau_alpha - 1/2) */
    double G;            /* Eq. (7); G < 0 is repulsive */
    double g[3];         /* body acceleration */
    double rho_s;        /* single wall-potential parameter */
    const uint8_t *solid;/* N bytes, nonzero = solid; may be NULL (no solids) */
} ora_params;

static int64_t nsites(const ora_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

static int is_solid(const ora_params *p, int64_t s) { return p->solid && p->solid[s]; }

static int64_t site_index(const ora_params *p, int x, int y, int z) { return x + (int64_t)p->nx * (y + (int64_t)p->ny * z); }

/* Neighbour of site s displaced by d (periodic in every direction). */
static int64_t shifted(const ora_params *p, int64_t s, int dx, int dy, int dz)
{
    int x = (int)(s % p->nx);
    int y = (int)((s / p->nx) % p->ny);
    int z = (int)(s / ((int64_t)p->nx * p->ny));
    x += dx; y += dy; z += dz;   /* |d| <= 1 in each direction */
    if (x < 0) x += p->nx; else if (x >= p->nx) x -= p->nx;
    if (y < 0) y += p->ny; else if (y >= p->ny) y -= p->ny;
    if (z < 0) z += p->nz; else if (z >= p->nz) z -= p->nz;
    return site_index(p, x, y, z);
}

/* ------------------------------------------------------------------------- */
/* Single-site building blocks.                                              */
/* ------------------------------------------------------------------------- */

/* Eq. (3): equilibrium of one component at density rho and velocity u.  With
 * eq_kind = 0 it is the Stokes-flow form printed in the paper (no terms of
 * second order in u); with eq_kind = 1 the second-order terms of the full
 * third-order expansion are included as well. */
void ora_feq(int eq_kind, double rho, const double u[3], double out[Q])
{
    make_tables();
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        double bracket = 1.0 + cu / T0 + (cu * cu * cu) / (6.0 * T0 * T0 * T0)
                         - cu * uu / (2.0 * T0 * T0);
        if (eq_kind == 1)
            bracket += (cu * cu) / (2.0 * T0 * T0) - uu / (2.0 * T0);
        out[i] = rho * weight(i) * bracket;
    }
}

/* Eq. (10): regularized non-equilibrium part f' = Phi : Pi.  Pi is the
 * non-equilibrium momentum flux, the second moment of f - f_eq; Phi projects
 * it back on the second-order Hermite polynomial c_i c_i - T0 I with weight
 * w_i / (2 T0^2).  Pi is returned as the full 3x3 matrix (row-major). */
void ora_regularize(const double f[Q], const double feq[Q], double fprime[Q], double Pi[9])
{
    make_tables();
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double sum = 0.0;
            for (int i = 0; i < Q; ++i)
                sum += CV[i][a] * CV[i][b] * (f[i] - feq[i]);
            Pi[3 * a + b] = sum;
        }
    for (int i = 0; i < Q; ++i) {
        double contraction = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double hermite = CV[i][a] * CV[i][b] - (a == b ? T0 : 0.0);
                contraction += hermite * Pi[3 * a + b];
            }
        fprime[i] = weight(i) / (2.0 * T0 * T0) * contraction;
    }
}

/* Wall densities rho^s_1, rho^s_2 from the single parameter rho^s (Section 2,
 * after Eq. 11): rho^s_1 = -rho_0 rho^s Theta(-rho^s),
 * rho^s_2 = rho_0 rho^s Theta(rho^s), with rho_0 = 1. */
static double wall_density(double rho_s, int alpha)
{
    if (alpha == 0) return rho_s < 0.0 ? -rho_s : 0.0;
    return rho_s > 0.0 ? rho_s : 0.0;
}

/* Forcing term of Eq. (9) for one component (Section 2, "following Li et al.
 * 2012", whose scheme is of Guo's type).  Guo's term, written for the
 * shifted velocity u_F, has a first-order Hermite part w_i c_i.F / T0 and a
 * second-order part w_i (c_i c_i - T0 I):(u_F F) / T0^2, both weighted by
 * (1 - 1/(2 tau)), and it acts on the BGK non-equilibrium f - f_eq(u_F),
 * whose first moment is -F/2.  The regularized f' of Eq. (10) keeps only the
 * second-order part of that non-equilibrium, so its dropped first-order part
 * (1 - 1/tau)(-F/2) is folded into the forcing term: the first-order part
 * becomes w_i c_i.F / (2 T0) for every tau, and the second-order part is
 * (1 - 1/(2 tau)) Phi : (u_F F + F u_F) with the projection Phi of Eq. (10).
 * force_kind = 1 keeps the first-order part only. */
static void forcing_term(int force_kind, double tau_mix, const double u[3], const double F[3], double out[Q])
{
    double S[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            S[3 * a + b] = (1.0 - 1.0 / (2.0 * tau_mix)) * (u[a] * F[b] + F[a] * u[b]);
    for (int i = 0; i < Q; ++i) {
        double cF = CV[i][0] * F[0] + CV[i][1] * F[1] + CV[i][2] * F[2];
        double first = weight(i) * cF / (2.0 * T0);
        double second = 0.0;
        if (force_kind == 0) {
            double contraction = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double hermite = CV[i][a] * CV[i][b] - (a == b ? T0 : 0.0);
                    contraction += hermite * S[3 * a + b];
                }
            second = weight(i) / (2.0 * T0 * T0) * contraction;
        }
        out[i] = first + second;
    }
}

/* ------------------------------------------------------------------------- */
/* Whole-lattice fields, one equation at a time.                             */
/* ------------------------------------------------------------------------- */

/* Eq. (4): component densities rho_alpha = sum_i f_i and momenta
 * j_alpha = sum_i c_i f_i at every fluid site. */
static void field_moments(const ora_params *p, const double *f, double *rho, double *j)
{
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        for (int a = 0; a < 2; ++a) {
            double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            if (!is_solid(p, s)) {
                for (int i = 0; i < Q; ++i) {
                    double fi = f[(a * Q + i) * N + s];
                    r += fi;
                    jx += CV[i][0] * fi;
                    jy += CV[i][1] * fi;
                    jz += CV[i][2] * fi;
                }
            }
            rho[a * N + s] = r;
            j[(a * 3 + 0) * N + s] = jx;
            j[(a * 3 + 1) * N + s] = jy;
            j[(a * 3 + 2) * N + s] = jz;
        }
    }
}

/* Eqs. (7) and (11): interaction force on component alpha from component
 * beta != alpha, F = G rho_alpha(x) sum_i w_i c_i rho'_beta(x + c_i), where
 * rho' is the fluid density on fluid sites and the wall density on solid
 * sites; plus the body force rho_alpha g. */
static void field_force(const ora_params *p, const double *rho, double *F)
{
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        /* per component: the fluid-fluid part of Eq. (7) and the wall part of
         * Eq. (11) (neighbours on solid sites carry the wall density) */
        double ff[2][3] = {{0, 0, 0}, {0, 0, 0}}, fw[2][3] = {{0, 0, 0}, {0, 0, 0}};
        if (!is_solid(p, s)) {
            for (int a = 0; a < 2; ++a) {
                int b = 1 - a;
                for (int i = 0; i < Q; ++i) {
                    int64_t n = shifted(p, s, CV[i][0], CV[i][1], CV[i][2]);
                    for (int d = 0; d < 3; ++d) {
                        if (is_solid(p, n))
                            fw[a][d] += weight(i) * CV[i][d] * wall_density(p->rho_s, b);
                        else
                            ff[a][d] += weight(i) * CV[i][d] * rho[b * N + n];
                    }
                }
                for (int d = 0; d < 3; ++d) {
                    ff[a][d] *= p->G * rho[a * N + s];
                    fw[a][d] *= p->G * rho[a * N + s];
                }
            }
        }
        for (int a = 0; a < 2; ++a) {
            for (int d = 0; d < 3; ++d) {
                double v = 0.0;
                if (!is_solid(p, s)) {
                    double wall = fw[a][d];
                    if (p->wall_kind == 1) {
                        /* W2: each component gives up its density share of the
                         * mixture's net wall force, so that the walls push the
                         * components apart but not the mixture */
                        double rho_mix = rho[s] + rho[N + s];
                        wall -= rho[a * N + s] / rho_mix * (fw[0][d] + fw[1][d]);
                    }
                    v = ff[a][d] + wall + rho[a * N + s] * p->g[d];
                }
                F[(a * 3 + d) * N + s] = v;
            }
        }
    }
}

/* Eq. (8): u = (j_1 + j_2) / rho; g = sum_alpha g_alpha rho_alpha / rho with
 * g_alpha = F_alpha / rho_alpha, i.e. g = (F_1 + F_2) / rho (written without
 * dividing by a component density, which may be zero); u_F = u + g / 2. */
static void field_velocity(const ora_params *p, const double *rho, const double *j,
                           const double *F, double *uF)
{
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        for (int d = 0; d < 3; ++d) {
            double v = 0.0;
            if (!is_solid(p, s)) {
                double rho_mix = rho[0 * N + s] + rho[1 * N + s];
                double u = (j[(0 * 3 + d) * N + s] + j[(1 * 3 + d) * N + s]) / rho_mix;
                double g = (F[(0 * 3 + d) * N + s] + F[(1 * 3 + d) * N + s]) / rho_mix;
                v = u + g / 2.0;
            }
            uF[d * N + s] = v;
        }
    }
}

/* Eqs. (5)-(6): tau_mix = nu_mix / T0 + 1/2 with nu_mix = p nu_1 + (1-p) nu_2
 * and p = rho_1 / rho. */
static void field_tau(const ora_params *p, const double *rho, double *tau_mix)
{
    int64_t N = nsites(p);
    double nu1 = T0 * (p->tau[0] - 0.5);
    double nu2 = T0 * (p->tau[1] - 0.5);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        double t = 0.0;
        if (!is_solid(p, s)) {
            double frac = rho[0 * N + s] / (rho[0 * N + s] + rho[1 * N + s]);
            double nu_mix = frac * nu1 + (1.0 - frac) * nu2;
            t = nu_mix / T0 + 0.5;
        }
        tau_mix[s] = t;
    }
}

/* Eq. (9) with Eqs. (3) and (10): post-collision populations
 * f* = f_eq(rho_alpha, u_F) + (1 - 1/tau_mix) f' + F_i, with the forcing term
 * F_i of forcing_term() for the component's force F_alpha. */
static void field_collide(const ora_params *p, const double *f, const double *rho,
                          const double *uF, const double *tau_mix, const double *F,
                          double *fstar)
{
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        if (is_solid(p, s)) continue;
        double u[3] = {uF[0 * N + s], uF[1 * N + s], uF[2 * N + s]};
        for (int a = 0; a < 2; ++a) {
            double fs[Q], feq[Q], fprime[Q], Pi[9], forcing[Q];
            double Fa[3] = {F[(a * 3 + 0) * N + s], F[(a * 3 + 1) * N + s], F[(a * 3 + 2) * N + s]};
            for (int i = 0; i < Q; ++i) fs[i] = f[(a * Q + i) * N + s];
            ora_feq(p->eq_kind, rho[a * N + s], u, feq);
            ora_regularize(fs, feq, fprime, Pi);
            forcing_term(p->force_kind, tau_mix[s], u, Fa, forcing);
            for (int i = 0; i < Q; ++i)
                fstar[(a * Q + i) * N + s] = feq[i] + (1.0 - 1.0 / tau_mix[s]) * fprime[i] + forcing[i];
        }
    }
}

/* Eq. (1) streaming, f_i(x + c_i, t + 1) = f*_i(x, t), written as a pull
 * f_i(x, t+1) = f*_i(x - c_i, t); when x - c_i is solid the population that
 * left x towards the wall returns reversed (halfway bounce-back):
 * f_i(x, t+1) = f*_opp(i)(x, t). */
static void field_stream(const ora_params *p, const double *fstar, double *fout)
{
    int64_t N = nsites(p);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        for (int a = 0; a < 2; ++a)
            for (int i = 0; i < Q; ++i) {
                double v = 0.0;
                if (!is_solid(p, s)) {
                    int64_t src = shifted(p, s, -CV[i][0], -CV[i][1], -CV[i][2]);
                    v = is_solid(p, src) ? fstar[(a * Q + opposite(i)) * N + s]
                                         : fstar[(a * Q + i) * N + src];
                }
                fout[(a * Q + i) * N + s] = v;
            }
    }
}

/* ------------------------------------------------------------------------- */
/* Exported entry points.                                                    */
/* ------------------------------------------------------------------------- */

/* Velocities, weights and opposite indices, for the lattice pins. */
void ora_lattice(int32_t c[Q * 3], double w[Q], int32_t opp[Q])
{
    make_tables();
    for (int i = 0; i < Q; ++i) {
        for (int d = 0; d < 3; ++d) c[3 * i + d] = CV[i][d];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Initial state: f = f_eq(rho_alpha, u) at every fluid site (the paper does
 * not state the initial populations; the non-equilibrium part starts at 0).
 * u may be NULL (fluid at rest). */
void ora_init(const ora_params *p, const double *rho1, const double *rho2, const double *u, double *f)
{
    make_tables();
    int64_t N = nsites(p);
    memset(f, 0, sizeof(double) * 2 * Q * N);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < N; ++s) {
        if (is_solid(p, s)) continue;
        double us[3] = {0.0, 0.0, 0.0};
        if (u) for (int d = 0; d < 3; ++d) us[d] = u[d * N + s];
        double feq[Q];
        ora_feq(p->eq_kind, rho1[s], us, feq);
        for (int i = 0; i < Q; ++i) f[(0 * Q + i) * N + s] = feq[i];
        ora_feq(p->eq_kind, rho2[s], us, feq);
        for (int i = 0; i < Q; ++i) f[(1 * Q + i) * N + s] = feq[i];
    }
}

/* Current macroscopic fields (Eqs. 4, 7, 8, 11): rho_1, rho_2 and the
 * velocity u_F (stored as uF[d * N + s]).  Solid sites report zeros. */
int ora_moments(const ora_params *p, const double *f, double *rho1, double *rho2, double *uF)
{
    make_tables();
    int64_t N = nsites(p);
    double *rho = malloc(sizeof(double) * 2 * N);
    double *j = malloc(sizeof(double) * 6 * N);
    double *F = malloc(sizeof(double) * 6 * N);
    if (!rho || !j || !F) { free(rho); free(j); free(F); return -1; }
    field_moments(p, f, rho, j);
    field_force(p, rho, F);
    field_velocity(p, rho, j, F, uF);
    memcpy(rho1, rho, sizeof(double) * N);
    memcpy(rho2, rho + N, sizeof(double) * N);
    free(rho); free(j); free(F);
    return 0;
}

/* One time step, f(t) -> f(t+1), both in post-streaming form. */
int ora_step(const ora_params *p, const double *f, double *fout)
{
    make_tables();
    int64_t N = nsites(p);
    double *rho = malloc(sizeof(double) * 2 * N);
    double *j = malloc(sizeof(double) * 6 * N);
    double *F = malloc(sizeof(double) * 6 * N);
    double *uF = malloc(sizeof(double) * 3 * N);
    double *tau_mix = malloc(sizeof(double) * N);
    double *fstar = calloc((size_t)2 * Q * N, sizeof(double));
    int rc = 0;
    if (!rho || !j || !F || !uF || !tau_mix || !fstar) { rc = -1; goto done; }
    field_moments(p, f, rho, j);              /* Eq. (4)        */
    field_force(p, rho, F);                   /* Eqs. (7), (11) */
    field_velocity(p, rho, j, F, uF);         /* Eq. (8)        */
    field_tau(p, rho, tau_mix);               /* Eqs. (5), (6)  */
    field_collide(p, f, rho, uF, tau_mix, F, fstar); /* Eqs. (3), (9), (10) */
    field_stream(p, fstar, fout);             /* Eq. (1)        */
done:
    free(rho); free(j); free(F); free(uF); free(tau_mix); free(fstar);
    return rc;
}

/* n time steps in place. */
int ora_run(const ora_params *p, double *f, int64_t n)
{
    int64_t N = nsites(p);
    double *tmp = malloc(sizeof(double) * 2 * Q * N);
    if (!tmp) return -1;
    for (int64_t t = 0; t < n; ++t) {
        if (ora_step(p, f, tmp)) { free(tmp); return -1; }
        memcpy(f, tmp, sizeof(double) * 2 * Q * N);
    }
    free(tmp);
    return 0;
}

/* Sums over fluid sites of rho_1, rho_2 and rho u_F (three components). */
int ora_reduce(const ora_params *p, const double *f, double out[5])
{
    make_tables();
    int64_t N = nsites(p);
    double *r1 = malloc(sizeof(double) * N), *r2 = malloc(sizeof(double) * N);
    double *uF = malloc(sizeof(double) * 3 * N);
    if (!r1 || !r2 || !uF) { free(r1); free(r2); free(uF); return -1; }
    ora_moments(p, f, r1, r2, uF);
    for (int k = 0; k < 5; ++k) out[k] = 0.0;
    for (int64_t s = 0; s < N; ++s) {
        if (is_solid(p, s)) continue;
        out[0] += r1[s];
        out[1] += r2[s];
        for (int d = 0; d < 3; ++d) out[2 + d] += (r1[s] + r2[s]) * uF[d * N + s];
    }
    free(r1); free(r2); free(uF);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* One step evaluated at chosen sites only, for spot checks on lattices too  */
/* large to step whole.  Same equations, in the same order, applied to the   */
/* few sites that the requested outputs depend on: f(x, t+1) needs f* at x   */
/* and at x - c_i, and each of those needs rho at its own neighbours.  Its   */
/* results equal ora_step's bit for bit (pinned by the CPU tests).           */
/* ------------------------------------------------------------------------- */

static void site_moments(const ora_params *p, const double *f, int64_t s, double rho[2], double j[2][3])
{
    int64_t N = nsites(p);
    for (int a = 0; a < 2; ++a) {
        rho[a] = 0.0; j[a][0] = j[a][1] = j[a][2] = 0.0;
        for (int i = 0; i < Q; ++i) {
            double fi = f[(a * Q + i) * N + s];
            rho[a] += fi;
            for (int d = 0; d < 3; ++d) j[a][d] += CV[i][d] * fi;
        }
    }
}

static double site_density(const ora_params *p, const double *f, int64_t s, int a)
{
    int64_t N = nsites(p);
    double r = 0.0;
    for (int i = 0; i < Q; ++i) r += f[(a * Q + i) * N + s];
    return r;
}

/* Eqs. (7) and (11) with the body force, at the fluid site s: the same sums
 * in the same order as field_force(), with the neighbours' densities summed
 * on the spot (the fluid-fluid part and the wall part of each component's
 * force apart, then the wall kind's combination). */
static void site_force(const ora_params *p, const double *f, int64_t s, const double rho[2], double F[2][3])
{
    double ff[2][3] = {{0, 0, 0}, {0, 0, 0}}, fw[2][3] = {{0, 0, 0}, {0, 0, 0}};
    for (int a = 0; a < 2; ++a) {
        int b = 1 - a;
        for (int i = 0; i < Q; ++i) {
            int64_t n = shifted(p, s, CV[i][0], CV[i][1], CV[i][2]);
            int wall = is_solid(p, n);
            double rho_b = wall ? 0.0 : site_density(p, f, n, b);
            for (int d = 0; d < 3; ++d) {
                if (wall)
                    fw[a][d] += weight(i) * CV[i][d] * wall_density(p->rho_s, b);
                else
                    ff[a][d] += weight(i) * CV[i][d] * rho_b;
            }
        }
        for (int d = 0; d < 3; ++d) {
            ff[a][d] *= p->G * rho[a];
            fw[a][d] *= p->G * rho[a];
        }
    }
    for (int a = 0; a < 2; ++a)
        for (int d = 0; d < 3; ++d) {
            double wall = fw[a][d];
            if (p->wall_kind == 1) {
                double rho_mix = rho[0] + rho[1];
                wall -= rho[a] / rho_mix * (fw[0][d] + fw[1][d]);
            }
            F[a][d] = ff[a][d] + wall + rho[a] * p->g[d];
        }
}

/* Post-collision populations of the fluid site s (Eqs. 3-11), computed as
 * field_moments() ... field_collide() compute them for that site. */
static void site_collide(const ora_params *p, const double *f, int64_t s, double fstar[2][Q])
{
    int64_t N = nsites(p);
    double rho[2], j[2][3], F[2][3];
    site_moments(p, f, s, rho, j);
    site_force(p, f, s, rho, F);
    double rho_mix = rho[0] + rho[1];
    double u[3];
    for (int d = 0; d < 3; ++d) {
        double bare = (j[0][d] + j[1][d]) / rho_mix;
        double g = (F[0][d] + F[1][d]) / rho_mix;
        u[d] = bare + g / 2.0;
    }
    double nu1 = T0 * (p->tau[0] - 0.5), nu2 = T0 * (p->tau[1] - 0.5);
    double frac = rho[0] / (rho[0] + rho[1]);
    double nu_mix = frac * nu1 + (1.0 - frac) * nu2;
    double tau_mix = nu_mix / T0 + 0.5;
    for (int a = 0; a < 2; ++a) {
        double fs[Q], feq[Q], fprime[Q], Pi[9], forcing[Q];
        for (int i = 0; i < Q; ++i) fs[i] = f[(a * Q + i) * N + s];
        ora_feq(p->eq_kind, rho[a], u, feq);
        ora_regularize(fs, feq, fprime, Pi);
        forcing_term(p->force_kind, tau_mix, u, F[a], forcing);
        for (int i = 0; i < Q; ++i)
            fstar[a][i] = feq[i] + (1.0 - 1.0 / tau_mix) * fprime[i] + forcing[i];
    }
}

/* out[(k * 2 + alpha) * 19 + i] = f_i^alpha(sites[k], t + 1); sites must be
 * fluid.  Returns -1 if a requested site is solid. */
int ora_step_sites(const ora_params *p, const double *f, int64_t nreq, const int64_t *sites, double *out)
{
    make_tables();
    for (int64_t k = 0; k < nreq; ++k)
        if (is_solid(p, sites[k])) return -1;
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < nreq; ++k) {
        int64_t s = sites[k];
        double here[2][Q], there[2][Q];
        site_collide(p, f, s, here);
        for (int i = 0; i < Q; ++i) {
            int64_t src = shifted(p, s, -CV[i][0], -CV[i][1], -CV[i][2]);
            int wall = is_solid(p, src);
            if (!wall) site_collide(p, f, src, there);
            for (int a = 0; a < 2; ++a)
                out[(k * 2 + a) * Q + i] = wall ? here[a][opposite(i)] : there[a][i];
        }
    }
    return 0;
}

/* Thread count of the OpenMP loops (0 or less leaves the default). */
#ifdef _OPENMP
#include <omp.h>
void ora_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int ora_get_threads(void) { return omp_get_max_threads(); }
#else
void ora_set_threads(int n) { (void)n; }
int ora_get_threads(void) { return 1; }
#endif
