/*
 * Test-infrastructure oracle for the regularized colour-gradient (RCG) lattice
 * Boltzmann step of arXiv:1711.02003, Sec. II.  Plain FP64 C, built with
 * -ffp-contract=off.  Not part of the product: only tests, the smoke check and
 * the benchmark's CPU-baseline leg use it.  It shares no code with the GPU
 * library.
 *
 * One time step, in the paper's order (Eq. (4) read as the composition
 * recolour o (perturb o collide), then streaming, Eq. (1)):
 *   1. colour densities rho^k (Eq. 2), total momentum rho*u (Eq. 3),
 *      phase field psi = (rho^R - rho^B) / rho;
 *   2. colour gradient F = grad psi with the isotropic stencil
 *      (1/c_s^2) sum_i w_i c_i psi(x + c_i);
 *   3. regularized relaxation (Eqs. 5, 6, 7, 11) at the node's relaxation
 *      time tau (below): the post-collision population is the sum of the
 *      colour equilibria plus (1 - 1/tau) times the second-order Hermite
 *      projection of the non-equilibrium momentum flux of both colours; or
 *      plain BGK (Eq. 5) on the total population at the same rate; or
 *      Eq. (5) as it is written, each colour relaxed towards its own
 *      equilibrium at its own rate 1/tau_k, when requested;
 *   4. perturbation (Eq. 9): add sum_k (A_k/2)|F| [w_i (F.c_i)^2/|F|^2 - B_i];
 *   5. recolouring (Eq. 10) of the total f_i into the two colours;
 *   6. streaming (Eq. 1) in push form with the boundary rules below.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - one relaxation time per node: Eq. (5) gives each component its own
 *     rate and Eq. (11) a single tau; a node holding both colours relaxes
 *     at tau = nu / c_s^2 + 1/2 with 1/nu = sum_k (rho^k / rho) / nu_k and
 *     nu_k = c_s^2 (tau_k - 1/2) (the harmonic mean of the component
 *     viscosities; the pure components keep their own tau_k);
 *   - B_i = w_i (|c_i|^2 - (D-1) c_s^2), which makes the perturbation
 *     mass-conserving with a traceless-in-the-normal stress;
 *   - D3Q19 phi_i^k: rest alpha_k, moving (1 - alpha_k) w_i / (1 - w_0),
 *     the same rule that gives Eq. (7) for D2Q9;
 *   - cos(phi_0) = 0 for the rest direction; for |F| <= eps_F the
 *     perturbation is skipped and all cosines are zero;
 *   - walls: half-way bounce-back of each colour; psi seen by the gradient =
 *     psi of the fluid node itself (neutral wetting, mask code 1) or the
 *     wall's own phase value psi_w (wetting walls, codes 64..127);
 *   - inlets: moving-wall bounce-back injecting colour k with density
 *     rho_w^k, psi seen by the gradient = psi of the inlet densities;
 *   - outlets: anti-bounce-back pressure boundary per colour: a population
 *     that would enter the outlet comes back reversed as minus itself plus
 *     twice the even part of the colour equilibrium at the outlet density
 *     (split into colours by the sending node's colour fractions) and the
 *     sending node's velocity, both taken from that node's own
 *     post-collision populations; psi seen by the gradient = psi of the
 *     node itself;
 *   - every axis wraps periodically; geometry comes only from the mask.
 */
#include "rcg_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19
#define CS2 (1.0 / 3.0)

typedef struct {
    int Q, D;
    int c[QMAX][3];
    double w[QMAX];
    double B[QMAX];
    int opp[QMAX];
    double cnorm[QMAX];
} lat_t;

/* Build the velocity set: D2Q9 in the order rest, then counter-clockwise
 * starting at +x, alternating axis and diagonal (Eq. (7) numbering shifted to
 * start at zero); D3Q19 as rest, the six axis vectors, the twelve face
 * diagonals. */
static void build_lattice(int lattice, lat_t *L)
{
    memset(L, 0, sizeof(*L));
    if (lattice == ORC_D2Q9) {
        static const int c2[9][2] = {{0, 0},  {1, 0},   {1, 1},  {0, 1}, {-1, 1},
                                     {-1, 0}, {-1, -1}, {0, -1}, {1, -1}};
        L->Q = 9;
        L->D = 2;
        for (int i = 0; i < 9; ++i) {
            L->c[i][0] = c2[i][0];
            L->c[i][1] = c2[i][1];
            L->c[i][2] = 0;
        }
    } else {
        int n = 0;
        L->Q = 19;
        L->D = 3;
        L->c[n][0] = L->c[n][1] = L->c[n][2] = 0;
        ++n;
        for (int a = 0; a < 3; ++a)
            for (int s = 1; s >= -1; s -= 2) {
                L->c[n][0] = L->c[n][1] = L->c[n][2] = 0;
                L->c[n][a] = s;
                ++n;
            }
        for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b)
                for (int sa = 1; sa >= -1; sa -= 2)
                    for (int sb = 1; sb >= -1; sb -= 2) {
                        L->c[n][0] = L->c[n][1] = L->c[n][2] = 0;
                        L->c[n][a] = sa;
                        L->c[n][b] = sb;
                        ++n;
                    }
    }
    for (int i = 0; i < L->Q; ++i) {
        int c2 = L->c[i][0] * L->c[i][0] + L->c[i][1] * L->c[i][1] + L->c[i][2] * L->c[i][2];
        if (L->D == 2)
            L->w[i] = (c2 == 0) ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        else
            L->w[i] = (c2 == 0) ? 1.0 / 3.0 : (c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        L->B[i] = L->w[i] * ((double)c2 - (double)(L->D - 1) * CS2);
        L->cnorm[i] = sqrt((double)c2);
        for (int j = 0; j < L->Q; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
                L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    }
}

/* phi_i(alpha) of Eq. (7): alpha for the rest population, the rest shared
 * among the moving ones in proportion to w_i. */
static double phi_of(const lat_t *L, int i, double alpha)
{
    if (i == 0) return alpha;
    return (1.0 - alpha) * L->w[i] / (1.0 - L->w[0]);
}

/* sum_i phi_i c_ix^2: the isotropic part of the equilibrium momentum flux per
 * unit density (Eq. (8) gives 3(1-alpha)/5 for D2Q9). */
static double phat_of(const lat_t *L, double alpha)
{
    double s = 0.0;
    for (int i = 0; i < L->Q; ++i) s += phi_of(L, i, alpha) * L->c[i][0] * L->c[i][0];
    return s;
}

static double alpha_or_default(const lat_t *L, double a)
{
    return (a > 0.0) ? a : L->w[0];
}

int orc_lattice(int lattice, double alpha, int *c, double *w, double *phi, double *B,
                int *opp)
{
    lat_t L;
    if (lattice != ORC_D2Q9 && lattice != ORC_D3Q19) return -1;
    build_lattice(lattice, &L);
    alpha = alpha_or_default(&L, alpha);
    for (int i = 0; i < L.Q; ++i) {
        if (c)
            for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        if (w) w[i] = L.w[i];
        if (phi) phi[i] = phi_of(&L, i, alpha);
        if (B) B[i] = L.B[i];
        if (opp) opp[i] = L.opp[i];
    }
    return L.Q;
}

/* Equilibrium of colour k, Eq. (6). */
static double feq(const lat_t *L, int i, double rho_k, double alpha_k, const double u[3])
{
    double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return rho_k * (phi_of(L, i, alpha_k) +
                    L->w[i] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
}

static int check_params(const orc_params *p, lat_t *L)
{
    if (!p) return -1;
    if (p->lattice != ORC_D2Q9 && p->lattice != ORC_D3Q19) return -1;
    if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return -1;
    if (p->lattice == ORC_D2Q9 && p->nz != 1) return -1;
    if (p->tau[0] <= 0.5 || p->tau[1] <= 0.5) return -1;
    if (p->collision < ORC_REGULARIZED || p->collision > ORC_BGK_COLOUR) return -1;
    build_lattice(p->lattice, L);
    if (p->mask) {
        long N = (long)p->nx * p->ny * p->nz;
        for (long n = 0; n < N; ++n) {
            int m = p->mask[n];
            if (m >= ORC_INLET0 && m < ORC_WALL0 && m - ORC_INLET0 >= p->n_inlets) return -1;
            if (m >= ORC_WALL0 && m < ORC_OUTLET0 && m - ORC_WALL0 >= p->n_walls) return -1;
            if (m >= ORC_OUTLET0 && m - ORC_OUTLET0 >= p->n_outlets) return -1;
        }
    }
    return 0;
}

/* Periodic wrap of a coordinate that is at most a few nodes outside [0, n). */
static inline long wrap(long a, long n)
{
    while (a < 0) a += n;
    while (a >= n) a -= n;
    return a;
}

static inline long node_at(const orc_params *p, long x, long y, long z)
{
    return wrap(x, p->nx) + p->nx * (wrap(y, p->ny) + p->ny * wrap(z, p->nz));
}

static inline int mask_of(const orc_params *p, long n)
{
    return p->mask ? p->mask[n] : 0;
}

#ifdef _OPENMP
#define OMP_FOR _Pragma("omp parallel for schedule(static)")
#else
#define OMP_FOR
#endif

static void set_threads(const orc_params *p)
{
#ifdef _OPENMP
    if (p->n_threads > 0) omp_set_num_threads(p->n_threads);
#else
    (void)p;
#endif
}

int orc_init(const orc_params *p, const double *rhoR, const double *rhoB, const double *u,
             double *f)
{
    lat_t L;
    if (check_params(p, &L)) return -1;
    set_threads(p);
    const long N = (long)p->nx * p->ny * p->nz;
    const int Q = L.Q;
    const double aR = alpha_or_default(&L, p->alpha[0]);
    const double aB = alpha_or_default(&L, p->alpha[1]);
    OMP_FOR
    for (long n = 0; n < N; ++n) {
        double un[3] = {0.0, 0.0, 0.0};
        if (u) {
            un[0] = u[n];
            un[1] = u[N + n];
            un[2] = u[2 * N + n];
        }
        for (int i = 0; i < Q; ++i) {
            f[(n * 2 + 0) * Q + i] = feq(&L, i, rhoR[n], aR, un);
            f[(n * 2 + 1) * Q + i] = feq(&L, i, rhoB[n], aB, un);
        }
    }
    return 0;
}

/* Eq. (2) and Eq. (3) at one node. */
static void node_moments(const lat_t *L, const double *fn, double *rR, double *rB, double j[3])
{
    double r0 = 0.0, r1 = 0.0;
    j[0] = j[1] = j[2] = 0.0;
    for (int i = 0; i < L->Q; ++i) {
        r0 += fn[i];
        r1 += fn[L->Q + i];
        for (int a = 0; a < 3; ++a) j[a] += (fn[i] + fn[L->Q + i]) * L->c[i][a];
    }
    *rR = r0;
    *rB = r1;
}

int orc_fields(const orc_params *p, const double *f, double *rhoR, double *rhoB, double *u,
               double *psi)
{
    lat_t L;
    if (check_params(p, &L)) return -1;
    set_threads(p);
    const long N = (long)p->nx * p->ny * p->nz;
    const int Q = L.Q;
    OMP_FOR
    for (long n = 0; n < N; ++n) {
        double rR = 0.0, rB = 0.0, j[3] = {0.0, 0.0, 0.0};
        if (mask_of(p, n) == 0) node_moments(&L, f + n * 2 * Q, &rR, &rB, j);
        double rho = rR + rB;
        if (rhoR) rhoR[n] = rR;
        if (rhoB) rhoB[n] = rB;
        for (int a = 0; a < 3; ++a)
            if (u) u[a * N + n] = (mask_of(p, n) == 0) ? j[a] / rho : 0.0;
        if (psi) psi[n] = (mask_of(p, n) == 0) ? (rR - rB) / rho : 0.0;
    }
    return 0;
}

/* Phase field psi = (rho^R - rho^B)/(rho^R + rho^B) of every fluid node. */
static void phase_field(const orc_params *p, const lat_t *L, const double *f, double *psi)
{
    const long N = (long)p->nx * p->ny * p->nz;
    OMP_FOR
    for (long n = 0; n < N; ++n) {
        if (mask_of(p, n) != 0) {
            psi[n] = 0.0;
            continue;
        }
        double rR, rB, j[3];
        node_moments(L, f + n * 2 * L->Q, &rR, &rB, j);
        psi[n] = (rR - rB) / (rR + rB);
    }
}

/* Colour gradient at fluid node (x,y,z): F = (1/c_s^2) sum_i w_i c_i psi~(x+c_i),
 * psi~ = psi at fluid neighbours, psi(x) at neutral walls and outlets, the
 * inlet's own phase value at inlets, psi_w at wetting walls. */
static void gradient_at(const orc_params *p, const lat_t *L, const double *psi, long x, long y,
                        long z, double F[3])
{
    long n = node_at(p, x, y, z);
    F[0] = F[1] = F[2] = 0.0;
    for (int i = 1; i < L->Q; ++i) {
        long m = node_at(p, x + L->c[i][0], y + L->c[i][1], z + L->c[i][2]);
        int code = mask_of(p, m);
        double ps;
        if (code == 0)
            ps = psi[m];
        else if (code >= ORC_INLET0 && code < ORC_WALL0) {
            const orc_inlet *in = &p->inlets[code - ORC_INLET0];
            ps = (in->rho_w[0] - in->rho_w[1]) / (in->rho_w[0] + in->rho_w[1]);
        } else if (code >= ORC_WALL0 && code < ORC_OUTLET0)
            ps = p->walls[code - ORC_WALL0].psi;
        else
            ps = psi[n];
        for (int a = 0; a < 3; ++a) F[a] += L->w[i] * L->c[i][a] * ps / CS2;
    }
}

int orc_gradient(const orc_params *p, const double *f, double *F)
{
    lat_t L;
    if (check_params(p, &L)) return -1;
    set_threads(p);
    const long N = (long)p->nx * p->ny * p->nz;
    double *psi = (double *)malloc(sizeof(double) * N);
    if (!psi) return -2;
    phase_field(p, &L, f, psi);
    OMP_FOR
    for (long n = 0; n < N; ++n) {
        long x = n % p->nx, y = (n / p->nx) % p->ny, z = n / ((long)p->nx * p->ny);
        double Fn[3] = {0.0, 0.0, 0.0};
        if (mask_of(p, n) == 0) gradient_at(p, &L, psi, x, y, z, Fn);
        for (int a = 0; a < 3; ++a) F[a * N + n] = Fn[a];
    }
    free(psi);
    return 0;
}

int orc_diagnostics(const orc_params *p, const double *f, orc_diag *d)
{
    lat_t L;
    if (check_params(p, &L) || !d) return -1;
    const long N = (long)p->nx * p->ny * p->nz;
    const int Q = L.Q;
    /* Eq. (8): the colour pressure is phat_k rho^k, phat_k the isotropic part
     * of the equilibrium momentum flux per unit density (3(1 - alpha_k)/5 for
     * D2Q9, 1/3 for alpha_k = w_0). */
    const double phat[2] = {phat_of(&L, alpha_or_default(&L, p->alpha[0])),
                            phat_of(&L, alpha_or_default(&L, p->alpha[1]))};
    double sum_in = 0.0, sum_out = 0.0;
    memset(d, 0, sizeof(*d));
    for (long n = 0; n < N; ++n) {
        if (mask_of(p, n) != 0) continue;
        d->fluid_nodes += 1;
        double rR, rB, j[3];
        node_moments(&L, f + n * 2 * Q, &rR, &rB, j);
        if (!(isfinite(rR) && isfinite(rB) && isfinite(j[0]) && isfinite(j[1]) && isfinite(j[2]))) {
            d->nonfinite += 1;
            continue;
        }
        const double rho = rR + rB;
        const double psi = (rR - rB) / rho;
        const double speed = sqrt(j[0] * j[0] + j[1] * j[1] + j[2] * j[2]) / rho;
        const double pres = phat[0] * rR + phat[1] * rB;
        d->mass[0] += rR;
        d->mass[1] += rB;
        for (int a = 0; a < 3; ++a) d->momentum[a] += j[a];
        if (speed > d->max_u) d->max_u = speed;
        if (psi > 0.99) {
            sum_in += pres;
            d->n_in += 1;
        } else if (psi < -0.99) {
            sum_out += pres;
            d->n_out += 1;
        }
        d->vol_R += 0.5 * (1.0 + psi);
    }
    d->p_in = d->n_in > 0 ? sum_in / (double)d->n_in : 0.0;
    d->p_out = d->n_out > 0 ? sum_out / (double)d->n_out : 0.0;
    const double pi = 3.14159265358979323846;
    d->R_eff = L.D == 2 ? sqrt(d->vol_R / pi) : cbrt(3.0 * d->vol_R / (4.0 * pi));
    return 0;
}

/* Collision, perturbation and recolouring at one node (steps 3-5). */
static void collide(const orc_params *p, const lat_t *L, const double *fin, const double F[3],
                    double *fout, double *f2out)
{
    const int Q = L->Q;
    const double alpha[2] = {alpha_or_default(L, p->alpha[0]), alpha_or_default(L, p->alpha[1])};
    double rho_k[2] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
    node_moments(L, fin, &rho_k[0], &rho_k[1], j);
    const double rho = rho_k[0] + rho_k[1];
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = j[a] / rho;

    /* Step 3: relaxation at the node's rate; the colour equilibria are
     * summed, so only the total momentum flux enters. */
    double inv_nu = 0.0;
    for (int k = 0; k < 2; ++k) inv_nu += (rho_k[k] / rho) / (CS2 * (p->tau[k] - 0.5));
    const double omega = 1.0 / (1.0 / (CS2 * inv_nu) + 0.5);
    double feq_sum[QMAX];
    for (int i = 0; i < Q; ++i)
        feq_sum[i] = feq(L, i, rho_k[0], alpha[0], u) + feq(L, i, rho_k[1], alpha[1], u);
    double f1[QMAX];
    if (p->collision == ORC_BGK) {
        /* Eq. (5) on the total population. */
        for (int i = 0; i < Q; ++i) {
            const double f = fin[i] + fin[Q + i];
            f1[i] = f - omega * (f - feq_sum[i]);
        }
    } else if (p->collision == ORC_BGK_COLOUR) {
        /* Eq. (5) as written: colour k relaxes towards its own equilibrium
         * at its own rate omega_k = 1/tau_k, and the colours are summed. */
        for (int i = 0; i < Q; ++i) {
            f1[i] = 0.0;
            for (int k = 0; k < 2; ++k) {
                const double fk = fin[k * Q + i];
                f1[i] += fk - (1.0 / p->tau[k]) * (fk - feq(L, i, rho_k[k], alpha[k], u));
            }
        }
    } else {
        /* Eq. (11): keep only rho^k, u and the momentum flux.  Pi^{neq} =
         * sum_i f_i c_i c_i - sum_k rho^k (phat_k I + u u), the equilibrium
         * flux of Eq. (6) summed over the colours. */
        const double phat[2] = {phat_of(L, alpha[0]), phat_of(L, alpha[1])};
        double Pi[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        for (int a = 0; a < L->D; ++a)
            for (int b = 0; b < L->D; ++b) {
                double s = 0.0;
                for (int i = 0; i < Q; ++i) s += (fin[i] + fin[Q + i]) * L->c[i][a] * L->c[i][b];
                for (int k = 0; k < 2; ++k) s -= rho_k[k] * ((a == b ? phat[k] : 0.0) + u[a] * u[b]);
                Pi[a][b] = s;
            }
        for (int i = 0; i < Q; ++i) {
            /* (c_i c_i - c_s^2 I) : Pi^{neq} */
            double qpi = 0.0;
            for (int a = 0; a < L->D; ++a)
                for (int b = 0; b < L->D; ++b)
                    qpi += (L->c[i][a] * L->c[i][b] - (a == b ? CS2 : 0.0)) * Pi[a][b];
            f1[i] = feq_sum[i] + (1.0 - omega) * L->w[i] / (2.0 * CS2 * CS2) * qpi;
        }
    }

    /* Step 4: perturbation, Eq. (9), summed over the two colours. */
    const double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    const int hasF = Fn > p->eps_F;
    double f2[QMAX];
    for (int i = 0; i < Q; ++i) {
        f2[i] = f1[i];
        if (hasF) {
            double Fc = F[0] * L->c[i][0] + F[1] * L->c[i][1] + F[2] * L->c[i][2];
            for (int k = 0; k < 2; ++k)
                f2[i] += 0.5 * p->A[k] * Fn * (L->w[i] * Fc * Fc / (Fn * Fn) - L->B[i]);
        }
    }
    if (f2out)
        for (int i = 0; i < Q; ++i) f2out[i] = f2[i];

    /* Step 5: recolouring, Eq. (10).  The zero-velocity equilibria give
     * sum_k rho^k phi_i^k. */
    const double seg = p->beta * rho_k[0] * rho_k[1] / (rho * rho);
    for (int i = 0; i < Q; ++i) {
        double cosp = 0.0;
        if (hasF && i != 0) {
            double Fc = F[0] * L->c[i][0] + F[1] * L->c[i][1] + F[2] * L->c[i][2];
            cosp = Fc / (Fn * L->cnorm[i]);
        }
        const double zero_u[3] = {0.0, 0.0, 0.0};
        double e0 = feq(L, i, rho_k[0], alpha[0], zero_u) + feq(L, i, rho_k[1], alpha[1], zero_u);
        fout[i] = rho_k[0] / rho * f2[i] + seg * cosp * e0;
        fout[Q + i] = rho_k[1] / rho * f2[i] - seg * cosp * e0;
    }
}

int orc_collide_node(const orc_params *p, const double *fin, const double *F, double *fout,
                     double *f2)
{
    lat_t L;
    if (!p) return -1;
    if (p->lattice != ORC_D2Q9 && p->lattice != ORC_D3Q19) return -1;
    build_lattice(p->lattice, &L);
    collide(p, &L, fin, F, fout, f2);
    return 0;
}

int orc_step(const orc_params *p, double *f, int nsteps)
{
    lat_t L;
    if (check_params(p, &L)) return -1;
    if (nsteps < 0) return -1;
    set_threads(p);
    const long N = (long)p->nx * p->ny * p->nz;
    const int Q = L.Q;
    double *psi = (double *)malloc(sizeof(double) * N);
    double *post = (double *)malloc(sizeof(double) * N * 2 * Q);
    if (!psi || !post) {
        free(psi);
        free(post);
        return -2;
    }
    for (int step = 0; step < nsteps; ++step) {
        /* Step 1: phase field of the current (pre-collision) state. */
        phase_field(p, &L, f, psi);

        /* Steps 2-5 at every fluid node. */
        OMP_FOR
        for (long n = 0; n < N; ++n) {
            if (mask_of(p, n) != 0) continue;
            long x = n % p->nx, y = (n / p->nx) % p->ny, z = n / ((long)p->nx * p->ny);
            double F[3];
            gradient_at(p, &L, psi, x, y, z, F);
            collide(p, &L, f + n * 2 * Q, F, post + n * 2 * Q, NULL);
        }

        /* Step 6: streaming, Eq. (1), push form.  Each fluid node sends its
         * post-collision populations along c_i.  A population that would enter
         * a wall of either kind comes back reversed to the sender (half-way
         * bounce-back); one
         * entering an inlet comes back reversed with the moving-wall momentum
         * term; one entering an outlet comes back by anti-bounce-back.  Every
         * fluid slot has exactly one writer, so the loop is race-free. */
        OMP_FOR
        for (long n = 0; n < N; ++n) {
            if (mask_of(p, n) != 0) continue;
            long x = n % p->nx, y = (n / p->nx) % p->ny, z = n / ((long)p->nx * p->ny);
            const double *pn = post + n * 2 * Q;
            for (int i = 0; i < Q; ++i) {
                long m = node_at(p, x + L.c[i][0], y + L.c[i][1], z + L.c[i][2]);
                int code = mask_of(p, m);
                const int io = L.opp[i];
                if (code == 0) {
                    for (int k = 0; k < 2; ++k) f[(m * 2 + k) * Q + i] = pn[k * Q + i];
                } else if (code == 1 || (code >= ORC_WALL0 && code < ORC_OUTLET0)) {
                    for (int k = 0; k < 2; ++k) f[(n * 2 + k) * Q + io] = pn[k * Q + i];
                } else if (code < ORC_WALL0) {
                    const orc_inlet *in = &p->inlets[code - ORC_INLET0];
                    double cu = L.c[i][0] * in->u[0] + L.c[i][1] * in->u[1] + L.c[i][2] * in->u[2];
                    for (int k = 0; k < 2; ++k)
                        f[(n * 2 + k) * Q + io] = pn[k * Q + i] - 2.0 * L.w[i] * in->rho_w[k] * cu / CS2;
                } else {
                    const orc_outlet *o = &p->outlets[code - ORC_OUTLET0];
                    double rP[2], jP[3], uP[3];
                    node_moments(&L, pn, &rP[0], &rP[1], jP);
                    for (int a = 0; a < 3; ++a) uP[a] = jP[a] / (rP[0] + rP[1]);
                    double cu = L.c[i][0] * uP[0] + L.c[i][1] * uP[1] + L.c[i][2] * uP[2];
                    double uu = uP[0] * uP[0] + uP[1] * uP[1] + uP[2] * uP[2];
                    for (int k = 0; k < 2; ++k) {
                        double rho_w = o->rho * rP[k] / (rP[0] + rP[1]);
                        double alpha_k = alpha_or_default(&L, p->alpha[k]);
                        double even = rho_w * (phi_of(&L, i, alpha_k) +
                                               L.w[i] * (cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
                        f[(n * 2 + k) * Q + io] = -pn[k * Q + i] + 2.0 * even;
                    }
                }
            }
        }
    }
    free(psi);
    free(post);
    return 0;
}
