/*
 * lbcg — regularized colour-gradient two-component lattice Boltzmann on
 * AMD MI355X (gfx950).
 *
 * The method is the one of Montessori, Lauricella, Tirelli and Succi,
 * "Regularized lattice Boltzmann multicomponent models for low Capillary and
 * Reynolds microfluidics flows" (arXiv:1711.02003), Sec. II: two colour
 * distributions f_i^R, f_i^B (Eq. (1)), colour densities (Eq. (2)), a common
 * velocity (Eq. (3)), a composite collision (Eq. (4)) made of a relaxation
 * towards the sum of the colour equilibria (Eqs. (5)-(7)) in its regularized
 * form (Eq. (11)), at one rate per node taken from the mixture viscosity, a
 * surface-tension perturbation driven by the colour gradient (Eq. (9)) and a
 * recolouring step (Eq. (10)), followed by streaming (Eq. (1)).
 *
 * Conventions used by every call:
 *   - a lattice has dims[0] x dims[1] x dims[2] = nx x ny x nz nodes
 *     (nz = 1 for D2Q9), node index n = x + nx * (y + ny * z), x fastest;
 *     all axes wrap periodically, geometry comes from the mask;
 *   - colour R ("red") is the dispersed component, B ("blue") the continuous
 *     one;
 *   - host arrays are plain C arrays owned by the caller; the library copies
 *     what it needs before returning and never keeps a host pointer;
 *   - every call returns LBCG_OK (0) or a negative LBCG_E_* code; on error
 *     the outputs are left untouched and the handle stays valid; no C++
 *     exception crosses this interface;
 *   - calls on one handle are not thread-safe; different handles are
 *     independent.  Work is queued on the handle's HIP stream; calls that
 *     return host data synchronize that stream.
 */
#ifndef LBCG_H
#define LBCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBCG_OK 0
#define LBCG_E_INVAL (-1)    /* invalid argument (dims, tau <= 1/2, mask code, sizes) */
#define LBCG_E_NOMEM (-2)    /* device memory exhausted or caller buffer too small */
#define LBCG_E_DEVICE (-3)   /* HIP runtime error, or no usable gfx950 device */
#define LBCG_E_UNSTABLE (-4) /* non-finite values found by the diagnostics */
#define LBCG_E_STATE (-5)    /* call made in the wrong order (e.g. step before init) */

/* Lattices: D2Q9 as written in the paper (Eq. (7)); D3Q19 for 3-D runs. */
#define LBCG_D2Q9 0
#define LBCG_D3Q19 1

/* Storage precision of the populations.  Arithmetic is FP64 for LBCG_F64
 * and FP32 otherwise; LBCG_F16 stores FP16 and computes in FP32. */
#define LBCG_F64 0
#define LBCG_F32 1
#define LBCG_F16 2

/* Relaxation: the regularized form of Eq. (11) (default) or the plain BGK
 * form of Eq. (5), both at the node's rate (see tau_B below), or Eq. (5) as
 * it is written, each colour relaxed towards its own equilibrium at its own
 * rate 1/tau_k (the literal baseline of Fig. 1; it does not keep momentum
 * where tau_R != tau_B).  Both BGK forms run on the generic kernel and,
 * with F32 or F16 storage, on the fused sweeps: the D3Q19 column sweep
 * (tiles of 8 rows, tile[0] 0 or 8) and the D2Q9 strip sweep; not on the
 * split step of D3Q19 lattices with geometry, the compact state or the
 * batched sweeps. */
#define LBCG_REGULARIZED 0
#define LBCG_BGK 1
#define LBCG_BGK_COLOUR 2

/* Kernel choice: automatic, the two-pass generic kernel (every lattice,
 * precision, collision and boundary) or the fused single-pass kernel (F32 or
 * F16 storage, state buffers below 4 GiB; D3Q19 or D2Q9, any collision
 * form, any geometry).  Automatic picks the fused kernel where it applies.
 *
 * LBCG_KERNEL_COMPACT (never picked automatically): the fused sweeps on a
 * compact state, regularized collision: for periodic lattices D3Q19 with F32
 * or F16 storage and tiles of 8 rows (tile[0] 0 or 8), or D2Q9 with F32
 * storage; with a geometry mask D3Q19 with F32 or F16 storage on the split
 * step of the fused kernel (launch shape fixed, tile all 0; a link from a
 * wall brings back the node's own population, a link from an inlet or an
 * outlet reads the pair that the boundary kernel stores in the pair
 * buffer); the pair state (2Q x 4 x pitch bytes for F32, 2Q x 2 x pitch for
 * F16) below 4 GiB (pitch = node count rounded up to 64).  Eq. (10) splits
 * every population of a node with coefficients that depend only on that
 * node and on the speed class of the direction, so each node stores its Q
 * total populations and its colour scalars (its minority share and one
 * vector per speed class) and the receiver of a population splits it: 192
 * bytes of memory traffic per node and step instead of 304 (D3Q19), 104
 * instead of 144 (D2Q9).  F16 storage keeps the totals (over w_i), the axis
 * vector and the diagonal ratio in F16, rounded stochastically, and the
 * minority share in F32: 100 bytes per node and step instead of the F16
 * pair state's 152.  Results agree with the pair-state kernels up to
 * rounding.  The first step after lbcg_init_fields or lbcg_set_state reads
 * the pair state; the calls that read the state (fields, populations,
 * diagnostics, lbcg_get_state) first convert the compact state to a pair
 * state in the handle's pair buffer, which the compact steps leave unused
 * but for those inlet and outlet values (one extra kernel, no change to the
 * trajectory).  lbcg_footprint adds the two compact buffers (2 x 96 x pitch
 * bytes for D3Q19 F32, 2 x 50 x pitch for D3Q19 F16, 2 x 52 x pitch for
 * D2Q9). */
#define LBCG_KERNEL_AUTO 0
#define LBCG_KERNEL_GENERIC 1
#define LBCG_KERNEL_FUSED 2
#define LBCG_KERNEL_COMPACT 3

/* Mask codes (one byte per node): 0 fluid; 1 neutral wall (half-way
 * bounce-back; the colour gradient sees the fluid node's own phase value
 * there); 2 + j inlet j, j < 62 (moving-wall velocity inlet); 64 + j wetting
 * wall j, j < 64 (half-way bounce-back; the colour gradient sees the wall's
 * phase value psi_w); 128 + j outlet j (pressure outlet).  The paper states
 * no boundary rule (its devices, Figs. 2 and 5, have walls, inlets and an
 * outlet); these are this library's.  Non-fluid nodes hold no fluid and are
 * never collided; their storage holds the boundary values that neighbouring
 * fluid nodes pull, and every export reports zeros for them. */
#define LBCG_FLUID 0
#define LBCG_WALL 1
#define LBCG_INLET0 2
#define LBCG_WALL0 64
#define LBCG_OUTLET0 128

/* Velocity inlet: populations leaving a fluid node towards the inlet node come
 * back reversed plus the moving-wall momentum term with velocity u; colour k
 * is injected with density rho_R / rho_B.  The colour gradient sees the
 * phase value (rho_R - rho_B) / (rho_R + rho_B) at inlet nodes. */
typedef struct {
    double u[3];
    double rho_R;
    double rho_B;
} lbcg_inlet;

/* Pressure outlet (anti-bounce-back): populations leaving towards the outlet
 * come back as minus themselves plus twice the even part of the colour
 * equilibrium at total density rho (split by the sending node's colour
 * fractions) and the sending node's velocity. */
typedef struct {
    double rho;
} lbcg_outlet;

/* Wetting wall: psi in [-1, 1] is the phase value (rho^R - rho^B)/rho the
 * colour gradient of a neighbouring fluid node sees at the wall.  +1 makes
 * colour R wet the wall, -1 colour B; a neutral wall is mask code 1. */
typedef struct {
    double psi;
} lbcg_wall;

typedef struct {
    int32_t lattice;     /* LBCG_D2Q9 or LBCG_D3Q19 */
    int32_t precision;   /* LBCG_F64, LBCG_F32 or LBCG_F16 */
    int32_t collision;   /* LBCG_REGULARIZED, LBCG_BGK or LBCG_BGK_COLOUR */
    int32_t kernel;      /* LBCG_KERNEL_* */
    int64_t dims[3];     /* nx, ny, nz (nz = 1 for D2Q9); each >= 1 */
    const uint8_t *mask; /* host, nx*ny*nz codes; NULL = every node fluid */
    double tau_R;        /* relaxation time of pure colour R (Eq. (5)), > 1/2 */
    double tau_B;        /* relaxation time of pure colour B, > 1/2; a node
                            holding both relaxes at tau = 3 nu + 1/2 with
                            1/nu = sum_k (rho^k/rho) / nu_k, nu_k = (tau_k - 1/2)/3 */
    double A_R;          /* surface-tension parameter A_R (Eq. (9)) */
    double A_B;          /* surface-tension parameter A_B (Eq. (9)) */
    double beta;         /* recolouring parameter (Eq. (10)), in [0, 1] */
    double alpha_R;      /* density-ratio parameter alpha_R (Eq. (7)); 0 = w_0 */
    double alpha_B;      /* density-ratio parameter alpha_B; 0 = w_0 */
    double eps_F;        /* |F| at or below which F counts as zero; < 0 = 1e-8 */
    int32_t n_inlets;    /* entries in inlets (<= 62) */
    int32_t n_outlets;   /* entries in outlets (<= 128) */
    const lbcg_inlet *inlets;   /* host, copied */
    const lbcg_outlet *outlets; /* host, copied */
    int32_t n_walls;     /* entries in walls (<= 64) */
    const lbcg_wall *walls;     /* host, copied */
    int32_t tile[3];     /* fused-kernel launch shape: rows per block (4 or 8;
                            D3Q19 only), z chunks (D2Q9: row chunks; <= 4096),
                            tile width (64; the compact D3Q19 sweep also 32:
                            256-thread blocks, several per compute unit);
                            0 = automatic.  With a geometry mask on D3Q19,
                            rows and z chunks both automatic pick the split
                            step (reported as rows 0) when at most half the
                            nodes are fluid, else the column sweep */
} lbcg_params;

/* FP64 diagnostics of the current state S_t (pre-collision), summed over fluid
 * nodes in a fixed order (bitwise reproducible for a given lattice).  Each
 * node's colour populations are decoded as lbcg_populations exports them and
 * its moments summed in FP64 (Eqs. (2), (3), (8)).  A fluid node whose
 * densities or momentum are not finite counts in `nonfinite` and is left out
 * of every other sum. */
typedef struct {
    double mass_R, mass_B;  /* sum of rho^R, rho^B (Eq. (2)) */
    double momentum[3];     /* sum of rho u (Eq. (3)) */
    double max_u;           /* max |u| (spurious currents at rest) */
    double p_in, p_out;     /* mean pressure sum_k phat_k rho^k (Eq. (8)) over
                               nodes with psi > 0.99 and psi < -0.99 */
    double vol_R;           /* sum (1 + psi)/2: volume of colour R */
    double R_eff;           /* sqrt(vol_R/pi) (2-D), (3 vol_R/(4 pi))^(1/3) (3-D) */
    int64_t nonfinite;      /* nodes whose moments are not finite */
    int64_t n_in, n_out;    /* node counts behind p_in and p_out */
    int64_t fluid_nodes;
    int64_t step;           /* time steps taken since initialisation */
} lbcg_diag;

typedef struct lbcg_sim lbcg_sim;

/* Device bytes lbcg_create needs for these parameters (two state buffers, the
 * phase-field scratch, the mask and link words, reduction scratch, a field
 * staging area, the two compact buffers of the compact kernel and, for a
 * D3Q19 F32 or F16 lattice with geometry, the split step's scratch: 12
 * collision moments and a node-list entry per node, and per-block lists).
 * Used for admission by footprint. */
int lbcg_footprint(const lbcg_params *p, size_t *bytes);

/* Create a simulation on the current HIP device.  dev_buf: NULL = the library
 * allocates (and frees) its memory; otherwise a device buffer of at least
 * lbcg_footprint bytes owned by the caller, which must outlive the handle.
 * hip_stream: the hipStream_t to queue work on; NULL = a stream the library
 * creates and owns.  Fails with LBCG_E_DEVICE if the device is not gfx950. */
int lbcg_create(const lbcg_params *p, void *dev_buf, size_t bytes, void *hip_stream,
                lbcg_sim **out);

/* Set the state to the colour equilibria of Eq. (6) at the given fields:
 * rhoR, rhoB (N doubles each), u (3N doubles, component-major, NULL = rest).
 * Resets the step counter. */
int lbcg_init_fields(lbcg_sim *s, const double *rhoR, const double *rhoB, const double *u);

/* Queue n >= 0 time steps (asynchronous).  One time step is Eq. (1): the
 * composite collision of Eq. (4) at every fluid node - relaxation (Eq. (11),
 * or Eq. (5) with a BGK collision), the perturbation of Eq. (9) driven by the
 * colour gradient of the phase field, the recolouring of Eq. (10) - followed
 * by streaming with the boundary rules of the mask.  Device faults surface at
 * the next synchronizing call. */
int lbcg_step(lbcg_sim *s, int64_t n);

/* Fields of the current state S_t: the colour densities rho^R, rho^B of
 * Eq. (2), the phase field psi = (rho^R - rho^B)/(rho^R + rho^B) (N doubles
 * each) and the common velocity u of Eq. (3) (3N doubles, component-major).
 * Output pointers select the fields (NULL = skip).  Non-fluid nodes read 0.
 * Synchronizes. */
int lbcg_fields(lbcg_sim *s, double *rhoR, double *rhoB, double *u, double *psi);

/* Pre-collision populations f_i^k of S_t (the distributions of Eq. (1)) in
 * canonical order f[k][i][n] (k = R, B; i as in the lattice numbering;
 * 2*Q*N doubles).  Synchronizes. */
int lbcg_populations(lbcg_sim *s, double *f);

/* Pre-collision populations of S_t at count listed nodes (node indices in
 * [0, N)): f[(j * 2 + k) * Q + i] for node j, colour k, direction i.  Lets a
 * caller check sampled nodes of a large lattice without copying it all.
 * Synchronizes. */
int lbcg_populations_at(lbcg_sim *s, const int64_t *nodes, int64_t count, double *f);

/* FP64 diagnostics (see lbcg_diag).  Returns LBCG_E_UNSTABLE, with *out
 * filled, when a non-finite value is found.  Synchronizes. */
int lbcg_diagnostics(lbcg_sim *s, lbcg_diag *out);

/* Raw state for checkpoint/restart: lbcg_state_bytes gives the size; get
 * copies it to host memory, set restores it (same parameters required).
 * A restored state continues bitwise-identically.  Synchronizes.  Layout: 8
 * int64 header words (magic, lattice, precision, nx, ny, nz, post-collision
 * flag, step), then Q arrays, one per direction, of N value pairs (total
 * deviation, minority share with the majority flag in its lowest bit) in
 * the storage precision. */
int lbcg_state_bytes(lbcg_sim *s, size_t *bytes);
int lbcg_get_state(lbcg_sim *s, void *host, size_t bytes);
int lbcg_set_state(lbcg_sim *s, const void *host, size_t bytes);

/* Wait for all queued work of the handle. */
int lbcg_synchronize(lbcg_sim *s);

/* Queue the handle's later work on another HIP stream (hip_stream; NULL = the
 * stream the library created for the handle, LBCG_E_INVAL if it created
 * none).  Nothing is synchronized here: the caller orders the work already
 * queued on the old stream before the handle's later work (by waiting for
 * the old stream or for an event recorded on it).  A batch keeps the stream
 * it was created with.  Lets one thread prepare or read back handles on one
 * stream while others compute on another (the served form). */
int lbcg_set_stream(lbcg_sim *s, void *hip_stream);

/* Release library-owned device memory and stream; never frees caller memory. */
void lbcg_destroy(lbcg_sim *s);

/* Static description of an LBCG_* status code. */
const char *lbcg_strerror(int status);

/* Launch shape chosen for the handle: kernel kind (LBCG_KERNEL_GENERIC,
 * LBCG_KERNEL_FUSED or LBCG_KERNEL_COMPACT), rows per block, z chunks, tile
 * width (64; or 32 on the compact D3Q19 sweep).  rows 0 on the fused kernel:
 * the split step of a D3Q19 lattice with geometry (one kernel pulls and
 * writes every fluid node's psi and collision moments, a second forms the
 * gradient, collides and stores, a third stores inlet and outlet values;
 * bitwise the column sweep's results, without the sweep's recomputed tile
 * ring and chunk halo, which dominate where the fluid fills few tiles).
 * NULL outputs are skipped. */
int lbcg_launch_info(lbcg_sim *s, int32_t *kernel, int32_t *rows, int32_t *zchunks, int32_t *tile_width);

/* Choose the fused (or compact) kernel's launch shape for this handle by
 * timing candidate shapes on the handle's own lattice (D3Q19: rows 4 or 8,
 * 8 only for the compact kernel, which also tries 32-wide tiles, and with a
 * geometry mask the split step; z splits
 * that fill the device once, twice or four times and chunks of 2 to 64
 * planes; D2Q9: row chunks of 8 to 512 rows), stepping the current state
 * into the spare buffer so the state does not change (the compact kernel is
 * timed on a compact state also before the handle's first compact step).  Keeps
 * the fastest shape for later steps and reports it.  No effect on the
 * generic kernel.  Synchronizes. */
int lbcg_tune(lbcg_sim *s, int32_t *rows, int32_t *zchunks);

/* Batched form (the paper's method applied to many independent lattices at
 * once): one fused launch per time level covers every lattice that still has
 * steps left, with runs of 32 levels replayed from HIP graphs.  A batch
 * refers to existing handles; it does not own them, and they must outlive
 * it.  Requirements: every handle initialised, all on the fused kernel
 * (D3Q19, F32 or F16 storage, regularized collision; geometry and periodic
 * lattices may mix) or all on the compact kernel (periodic D3Q19, F32 or
 * F16 storage), one storage precision, one stream, no handle listed twice.
 * tile: {rows per block (4 or 8; 8 on the compact kernel), z planes per
 * chunk (>= 1)}; NULL or {0, 0}
 * = choose by timing candidate shapes on the batch (the states do not
 * change).  Errors: LBCG_E_INVAL for a violated requirement, LBCG_E_NOMEM /
 * LBCG_E_DEVICE for allocation or HIP failures.  The batch allocates its
 * own small descriptor tables (device and pinned host memory).
 *
 * lbcg_batch_step advances lattice j by nsteps[j] >= 0 steps (n entries),
 * asynchronously on the shared stream.  Results per lattice are bitwise those
 * of lbcg_step on the handle alone.  Between batch steps the handles may be
 * used directly (fields, diagnostics, lbcg_step): a batch has no field call
 * of its own, since every member is an ordinary handle. */
typedef struct lbcg_batch lbcg_batch;
int lbcg_batch_create(lbcg_sim *const *sims, int32_t n, const int32_t *tile, lbcg_batch **out);
int lbcg_batch_step(lbcg_batch *b, const int64_t *nsteps);
/* Launch shape of the batch: rows per block, z planes per chunk, total blocks
 * of one level over all lattices. */
int lbcg_batch_launch_info(lbcg_batch *b, int32_t *rows, int32_t *zplanes, int64_t *blocks);
/* Waits for the batch's queued work, then releases its tables. */
void lbcg_batch_destroy(lbcg_batch *b);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the batched step of
 * lbcg_batch_step without a batch object, allocating nothing - no device or
 * host memory, no pinned staging, no HIP graph.  Advances sims[j] by
 * nsteps[j] >= 0 steps (n entries) with the launch shape tile = {rows per
 * block (4 or 8; 8 on the compact kernel), z planes per chunk (>= 1)}; the
 * requirements on the handles are those of lbcg_batch_create, and all must
 * belong to the device current at the call.  Results per lattice are bitwise
 * those of lbcg_batch_step and lbcg_step.
 * The descriptors and block tables live in one fixed area of device memory
 * that the library holds per device until the process ends (about 1.1 MB),
 * written by small kernels queued on the handles' stream: at most
 * LBCG_NOALLOC_MAX_LATTICES lattices per call and LBCG_NOALLOC_MAX_BLOCKS
 * blocks per level for each of the periodic and the geometry groups; larger
 * calls fail with LBCG_E_INVAL before queuing anything.  The area keeps the
 * last call's contents; calls on one stream are ordered, while calls whose
 * work overlaps on one device (different streams) race on it.  Asynchronous
 * like lbcg_batch_step.  Errors: LBCG_E_INVAL (requirements, sizes, another
 * device), LBCG_E_DEVICE (HIP errors). */
#define LBCG_NOALLOC_MAX_LATTICES 256
#define LBCG_NOALLOC_MAX_BLOCKS 65536
int lbcg_batch_step_noalloc(lbcg_sim *const *sims, int32_t n, const int32_t *tile, const int64_t *nsteps);

#ifdef __cplusplus
}
#endif
#endif
