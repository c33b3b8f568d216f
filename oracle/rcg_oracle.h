/*
 * Test-infrastructure oracle: plain, slow, FP64 CPU implementation of the
 * regularized colour-gradient (RCG) two-component lattice Boltzmann step of
 * Montessori, Lauricella, Tirelli, Succi, "Regularized lattice Boltzmann
 * multicomponent models for low Capillary and Reynolds microfluidics flows"
 * (arXiv:1711.02003), Sec. II, Eqs. (1)-(11).
 *
 * This code exists only to check the GPU implementation.  Only the tests,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It
 * shares no code, header, table or helper with the GPU library.
 *
 * State layout (array-of-structures, the oracle's own choice):
 *     f[((node * 2) + k) * Q + i],   node = x + nx * (y + ny * z),
 *     k = 0 (red, "zeta", dispersed) or 1 (blue, "xi", continuous),
 *     i = 0..Q-1 with i = 0 the rest velocity.
 * The stored state is the pre-collision population S_t (after streaming).
 */
#ifndef RCG_ORACLE_H
#define RCG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };
/* Relaxation: Eq. (11) at the node's rate; Eq. (5) on the total population at
 * the node's rate; Eq. (5) as written, each colour at its own rate 1/tau_k. */
enum { ORC_REGULARIZED = 0, ORC_BGK = 1, ORC_BGK_COLOUR = 2 };

/* Mask codes: 0 fluid, 1 neutral wall (half-way bounce-back; the colour
 * gradient sees the node's own psi there), 2..63 inlet number (code - 2),
 * 64..127 wetting wall number (code - 64; bounce-back, the gradient sees the
 * wall's psi_w), 128..255 outlet number (code - 128). */
#define ORC_INLET0 2
#define ORC_WALL0 64
#define ORC_OUTLET0 128

typedef struct {
    double u[3];      /* inlet velocity (lattice units) */
    double rho_w[2];  /* injected density of each colour */
} orc_inlet;

typedef struct {
    double rho;       /* prescribed total density (pressure rho/3) */
} orc_outlet;

typedef struct {
    double psi;       /* phase value psi_w the colour gradient sees at the wall */
} orc_wall;

typedef struct {
    int lattice;            /* ORC_D2Q9 or ORC_D3Q19 */
    int collision;          /* ORC_REGULARIZED, ORC_BGK or ORC_BGK_COLOUR */
    int nx, ny, nz;         /* nz = 1 for D2Q9 */
    double tau[2];          /* relaxation times of the pure components, Eq. (5) */
    double A[2];            /* surface-tension parameters A_k, Eq. (9) */
    double alpha[2];        /* density-ratio parameters alpha_k, Eq. (7) */
    double beta;            /* recolouring parameter, Eq. (10) */
    double eps_F;           /* |F| at or below which F is treated as zero */
    const uint8_t *mask;    /* nx*ny*nz codes, NULL = every node fluid */
    int n_inlets;
    const orc_inlet *inlets;
    int n_outlets;
    const orc_outlet *outlets;
    int n_walls;
    const orc_wall *walls;
    int n_threads;          /* OpenMP threads, <= 0 = library default */
} orc_params;

/* FP64 diagnostics of a pre-collision state, summed over fluid nodes in node
 * order.  A fluid node whose colour densities or momentum (Eqs. (2), (3)) are
 * not finite is counted in nonfinite and left out of every other sum. */
typedef struct {
    double mass[2];         /* sum of rho^R, rho^B (Eq. (2)) */
    double momentum[3];     /* sum of rho u (Eq. (3)) */
    double max_u;           /* max |u| */
    double p_in, p_out;     /* mean colour pressure sum_k phat_k rho^k (Eq. (8))
                               over nodes with psi > 0.99 and psi < -0.99 */
    long n_in, n_out;       /* node counts behind p_in and p_out */
    double vol_R;           /* sum (1 + psi)/2 */
    double R_eff;           /* sqrt(vol_R/pi) (2-D), (3 vol_R/(4 pi))^(1/3) (3-D) */
    long nonfinite;
    long fluid_nodes;
} orc_diag;

/* Lattice tables as the oracle builds them (for pins in tests).
 * c: Q*3 ints, w, phi (for given alpha), B: Q doubles each. Returns Q. */
int orc_lattice(int lattice, double alpha, int *c, double *w, double *phi,
                double *B, int *opp);

/* S_0 = colour equilibria f^{k,eq}(rho^k, u) of Eq. (6); rhoR, rhoB: N,
 * u: 3N (component-major, u[a*N + node]) or NULL for rest. */
int orc_init(const orc_params *p, const double *rhoR, const double *rhoB,
             const double *u, double *f);

/* Advance f (pre-collision state) by nsteps.  Returns 0 on success. */
int orc_step(const orc_params *p, double *f, int nsteps);

/* Moments of the pre-collision state: rho^R, rho^B (N each), u (3N,
 * component-major), psi (N).  Non-fluid nodes get zeros.  Any pointer may be
 * NULL. */
int orc_fields(const orc_params *p, const double *f, double *rhoR,
               double *rhoB, double *u, double *psi);

/* Colour gradient F (3N, component-major) of the pre-collision state. */
int orc_gradient(const orc_params *p, const double *f, double *F);

/* Diagnostics of the pre-collision state f (see orc_diag). */
int orc_diagnostics(const orc_params *p, const double *f, orc_diag *d);

/* Collision at one node, exposed for closed-form pins: fin = 2*Q
 * pre-collision values [k][i], F = colour gradient, fout = 2*Q
 * post-recolouring values [k][i].  Also returns (optionally) f2 = the Q
 * total post-perturbation values before recolouring. */
int orc_collide_node(const orc_params *p, const double *fin, const double *F,
                     double *fout, double *f2);

#ifdef __cplusplus
}
#endif
#endif
