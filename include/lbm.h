/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the two-component
 * Shan-Chen lattice Boltzmann model on D3Q19 of Otomo et al., "Multi-component
 * lattice Boltzmann models for accurate simulation of flows with wide
 * viscosity variation" (arXiv:1711.03254), Section 2.
 *
 * One time step (Eqs. 1-11): pull-streaming with halfway bounce-back on a
 * voxel solid mask, component densities and momenta (Eq. 4), the 18-neighbour
 * Shan-Chen force with the wall densities of the wettability condition
 * (Eqs. 7 and 11), the force-shifted velocity u_F (Eq. 8), the mixture
 * relaxation time (Eqs. 5-6), the third-order equilibrium (Eq. 3), the
 * regularized non-equilibrium part (Eq. 10) and the forcing term, combined as
 * in Eq. (9).
 *
 * Conventions shared by every call
 * --------------------------------
 *  Lattice: nx * ny * nz sites, periodic in every direction; walls come only
 *  from the solid mask.  Site index s = x + nx * (y + ny * z) (x fastest).
 *  Scalar fields are arrays of N = nx*ny*nz doubles indexed by s.  Vector
 *  fields are 3*N doubles, component-major: v[d * N + s], d = 0,1,2 = x,y,z.
 *  Populations are 2*19*N doubles, p[(alpha * 19 + i) * N + s], alpha = 0,1
 *  the component and i the D3Q19 direction in this fixed order:
 *     i = 0        rest (0,0,0)
 *     i = 1..6     (+1,0,0) (-1,0,0) (0,+1,0) (0,-1,0) (0,0,+1) (0,0,-1)
 *     i = 7..10    (+1,+1,0) (-1,-1,0) (+1,-1,0) (-1,+1,0)
 *     i = 11..14   (+1,0,+1) (-1,0,-1) (+1,0,-1) (-1,0,+1)
 *     i = 15..18   (0,+1,+1) (0,-1,-1) (0,+1,-1) (0,-1,+1)
 *  so the opposite of i >= 1 is i + 1 for odd i and i - 1 for even i.
 *  Weights: 1/3 (rest), 1/18 (i = 1..6), 1/36 (i = 7..18); T0 = 1/3.
 *  The populations exchanged through this ABI are the post-streaming
 *  distribution f_i(x, t) of Eq. (1); how the library stores them internally
 *  is its own affair.  Solid sites carry no populations: they read back as 0.
 *
 *  Pointers: "host" arguments are ordinary CPU memory; when an on_device flag
 *  (or inputs_on_device) is 1 they are device pointers in the same HIP
 *  context (e.g. torch tensors' data_ptr()), used on the context's stream.
 *  Input arrays are borrowed for the duration of the call only (copied);
 *  output arrays belong to the caller and must hold the sizes stated.
 *
 *  Errors: every call returns LBM_OK (0) or a negative code; no exception or
 *  signal crosses the ABI.  lbm_last_error() gives a text for the last
 *  failure of a context.  A context is not thread-safe; distinct contexts
 *  are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

/* Storage precision of the populations.  Arithmetic is FP64 for LBM_FP64
 * and FP32 otherwise.  FP16S / BF16S store each population as the 16-bit
 * deviation f_i - w_i * rho_ref[a] (shifted storage; rho_ref in lbm_params). */
typedef enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16S = 2, LBM_BF16S = 3 } lbm_prec;

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* invalid argument: see lbm_last_error */
    LBM_ENOMEM = -2,       /* device or host allocation failed */
    LBM_EDEVICE = -3,      /* a HIP call failed (its text in lbm_last_error) */
    LBM_ENONFINITE = -4,   /* the periodic check found a NaN or infinity */
    LBM_EMASSDRIFT = -5    /* the periodic check found a component mass off by more than mass_tol */
};

typedef struct {
    int32_t nx, ny, nz;          /* lattice size, each >= 1 */
    int32_t prec;                /* lbm_prec */
    double tau[2];               /* per-component relaxation times, > 1/2; nu_a = T0 (tau_a - 1/2) (Eq. 5) */
    double G;                    /* Shan-Chen coupling of Eq. (7), the paper's sign: G < 0 repels */
    double g[3];                 /* body acceleration; component a feels rho_a * g */
    double rho_s;                /* wall parameter rho^s: wall densities rho^s_1 = max(-rho^s, 0),
                                    rho^s_2 = max(rho^s, 0) on solid sites (Eq. 11 and after) */
    int32_t eq_kind;             /* 0: Eq. (3) as printed (no second-order terms); 1: with them */
    int32_t force_kind;          /* 0: forcing term with its second-order part (default);
                                    1: first-order part only */
    int32_t check_every;         /* every k steps lbm_step checks masses and finiteness in FP64 (0 = never) */
    int32_t inputs_on_device;    /* 1: solid, rho_init, u_init are device pointers */
    double mass_tol;             /* relative mass drift allowed by the check; 0 = a default per precision */
    double rho_ref[2];           /* per-component shift reference of FP16S / BF16S storage:
                                    stored value = f_i - w_i * rho_ref[a].  0 = the component's mean
                                    initial density over fluid sites; < 0 = no shift */
    const uint8_t *solid;        /* N bytes, nonzero = solid; NULL = no solids */
    const double *rho_init[2];   /* N each: initial component densities (>= 0, sum > 0 on fluid sites) */
    const double *u_init;        /* 3N (component-major) initial velocity, or NULL for rest */
    void *stream;                /* hipStream_t to run on; NULL = a stream the library creates */
    int32_t tile_x, tile_y;      /* x-y tile of the step kernel (0 = library default; 64x4, 32x8,
                                    16x16, 8x32, 64x8, 32x16 or 64x16; FP64 takes the first four
                                    only, others give LBM_EINVAL) */
    int32_t zchunk;              /* z planes per block; 0 (default): the library cuts each tile
                                    column into work items of balanced cost (dense columns into
                                    more, shorter items), one round of resident blocks */
    int32_t wall_kind;           /* 0: the wall force of Eq. (11) as it stands (W1, default);
                                    1: each component gives up its density share of the mixture's
                                    net wall force, so that the walls separate the components
                                    without pushing the mixture (W2, the momentum-balanced wall
                                    interaction of Section 2 after Eq. 11, used in
                                    Section 3.5) */
    double tau_crit;             /* FP32 and 16-bit storage: sites whose mixture relaxation time
                                    (Eqs. 5-6) is below tau_crit accumulate the second moments of
                                    the collision (the non-equilibrium flux of Eq. 10) in FP64:
                                    near tau = 1/2 (low viscosity) that flux is a small difference
                                    of sums of size rho / 3.  0 = never (default); FP64 storage
                                    computes everything in FP64 and ignores it */
} lbm_params;

/* Creates a context: validates p, allocates the device state and sets the
 * populations to the equilibrium f = f_eq(rho_init, u_init) (Eq. 3; the
 * paper does not state the initial populations).  Records the initial
 * component masses for the periodic check.  On failure *out is NULL.
 * Size limits (LBM_EINVAL): fewer than 2^30 sites, and 11 of the 19
 * directions of the fluid sites' populations below 4 GiB (about 24 M fluid
 * sites at FP64, 48 M at FP32, 97 M with 16-bit storage); with 32- or 16-bit
 * storage also nz (tile_x + 4)(tile_y + 4) x 4 bytes below 4 GiB (the index
 * tiles of one tile column: nz < 789 516 at 64 x 16 tiles).  Device memory:
 * two population buffers of about 2 x 22 x n_fluid x storage bytes (the 19
 * directions are stored in two halves of 11 direction slots), plus 8 bytes
 * per site for the link mask and the site index, plus at 32 and 16 bits
 * the step's index tiles, 4 (tile_x + 4)(tile_y + 4) / (tile_x tile_y)
 * bytes per site of the padded lattice (5.3 at 64 x 16). */
int lbm_init(const lbm_params *p, lbm_ctx **out);

/* Advances n >= 0 time steps (Eqs. 1-11).  Every check_every steps the step
 * also sums the masses in FP64 and flags non-finite values; a failed check
 * stops the advance and returns LBM_ENONFINITE or LBM_EMASSDRIFT.  Runs of
 * 16 plain steps replay a HIP graph captured on first use.  Asynchronous
 * except at check steps: later calls on the context are ordered after it. */
int lbm_step(lbm_ctx *c, int64_t n);

/* Macroscopic fields of the current state (Eqs. 4, 7, 8, 11): rho1, rho2 (N
 * each) and the velocity u_F of Eq. (8) (3N, component-major).  Any pointer
 * may be NULL to skip that field.  Solid sites report 0.  Returns after the
 * data is in place (synchronizes the context's stream). */
int lbm_moments(lbm_ctx *c, double *rho1, double *rho2, double *uF, int on_device);

/* FP64 sums over fluid sites of the current state: out = [sum rho1,
 * sum rho2, sum rho u_F,x, sum rho u_F,y, sum rho u_F,z] (host array of 5). */
int lbm_reduce(lbm_ctx *c, double out[5]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, allocation-free serving loops): the sums of lbm_reduce, written
 * to out_dev, a device array of 5 doubles, on the context's stream without
 * synchronizing.  It allocates nothing: the per-block partial sums go to a
 * fixed work array of the library on each GPU (at most 16384 blocks, 1 MiB,
 * held until the process ends) instead of the context's own.  All calls on
 * one GPU share that array, so calls that overlap in time on one GPU (on
 * different streams or host threads) race; calls ordered on one stream do
 * not.  Errors: LBM_EINVAL (NULL argument, or a context whose step runs more
 * than 16384 blocks), LBM_EDEVICE. */
int lbm_reduce_noalloc(lbm_ctx *c, double *out_dev);

/* Checkpoint: copies the current populations f_i(x, t) (2*19*N doubles, the
 * ABI layout above) out; solid sites give 0. */
int lbm_get_populations(lbm_ctx *c, double *f, int on_device);

/* Resume / test hook: replaces the state by the populations f (2*19*N
 * doubles, the ABI layout; solid sites ignored), rounded to the storage
 * precision.  get after set returns f exactly at FP64.  The component masses
 * of the periodic check are re-recorded from the new state, and at 16 bits a
 * default shift reference (rho_ref 0) is recomputed as the new state's mean
 * density, so a checkpoint resumes correctly into a context created from
 * placeholder fields. */
int lbm_set_populations(lbm_ctx *c, const double *f, int on_device);

/* Warm start: replaces the state by f_eq(rho1, rho2, u) as lbm_init does.
 * u may be NULL (rest).  Component masses for the check are re-recorded. */
int lbm_set_fields(lbm_ctx *c, const double *rho1, const double *rho2, const double *u, int on_device);

/* Restart from macroscopic fields, as lbm_moments reports them: rho1, rho2
 * and the force-shifted velocity u_F of Eq. (8) (3N, required).  Component
 * a's populations are f_eq(rho_a, u_F - F_a / (2 rho_a)) (Eq. 3, with F_a
 * the force of Eqs. 7 and 11 plus rho_a g evaluated on the given densities,
 * so that Eq. 8 gives back u_F) plus the non-equilibrium part that the
 * strain of u_F implies to first order in the Chapman-Enskog expansion:
 * Pi = -rho T0 tau_mix (grad u_F + grad u_F^T) (tau_mix of Eqs. 5-6),
 * shared by the components in proportion to their densities and projected
 * as in Eq. (10).  grad u_F takes central differences, a solid neighbour
 * standing for a wall half a site away where u_F = 0.  Component masses for
 * the check are re-recorded.  Allocates and frees a 12N-double work buffer.
 * Errors: LBM_EINVAL (NULL argument or invalid fields), LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_set_fields_strain(lbm_ctx *c, const double *rho1, const double *rho2, const double *u, int on_device);

/* Convergence residual of a steady solve, in FP64 on the device:
 * out[0] = ||u_F - u_F'|| / ||u_F||, out[1] = ||rho1 - rho1'|| / ||rho1||
 * (2-norms over the lattice; u_F of Eq. 8), where the primed fields are
 * those of the previous lbm_residual call on this context, or zero after
 * lbm_init, lbm_set_fields(_strain) and lbm_set_populations (the first
 * call then gives 1).  Keeps the current fields as the next call's primed
 * ones (4N doubles held by the context from the first call).  A zero norm
 * with a zero difference gives 0.  Synchronizes the context's stream.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE. */
int lbm_residual(lbm_ctx *c, double out[2]);

/* Distance of the current state from given fields, in FP64 on the device:
 * out[0] = ||u_F - u|| / ||u||, out[1] = ||rho1 - r1|| / ||r1|| (2-norms over
 * the lattice; u_F of Eq. 8, as lbm_moments reports it), for judging a solve
 * against a reference state.  r1 (N) and u (3N) are host arrays or, with
 * on_device, device arrays; host arrays are staged through a temporary 4N-
 * double device buffer.  Does not touch the residual's fields.  A zero norm
 * with a zero difference gives 0.  Synchronizes the context's stream.
 * Errors: LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE. */
int lbm_distance(lbm_ctx *c, const double *r1, const double *u, int on_device, double out[2]);

/* Facts about a context, for reports: number of fluid sites, steps done,
 * bytes of population storage per site update (read + write), and the
 * step kernel's launch configuration (zchunk 0: balanced work items). */
typedef struct {
    int64_t n_sites, n_fluid, steps_done;
    int32_t bytes_per_lu;        /* 2 * 2 * 19 * sizeof(storage) */
    int32_t tile_x, tile_y, zchunk, blocks;
    double mass0[2];             /* component masses recorded at init / set_fields */
} lbm_info_t;
int lbm_info(const lbm_ctx *c, lbm_info_t *out);

/* ------------------------------------------------------------------------
 * Batches: many independent domains (different sizes, viscosities, G,
 * geometries) advanced together, one kernel launch per step over a work list
 * of every domain's tiles; runs of plain steps replay a captured HIP graph.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Groups n contexts (borrowed; they must outlive the batch) that share one
 * precision, tile shape and device.  Each keeps its own state, parameters
 * and check period, and stays usable with the calls above between batch
 * steps.  Errors: LBM_EINVAL (mismatch, duplicate, NULL), LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_batch_create(lbm_ctx *const *ctxs, int32_t n, lbm_batch **out);

/* Advances every domain of the batch by n steps (Eqs. 1-11 per domain),
 * with each domain's periodic FP64 check; returns when the work is done.
 * A failed check stops the batch and names the domain in the error text. */
int lbm_batch_step(lbm_batch *b, int64_t n);

/* Text of the last failure of b (or of the last failed lbm_batch_create
 * when b is NULL); never NULL. */
const char *lbm_batch_last_error(const lbm_batch *b);

/* Releases the batch (not its contexts).  NULL is accepted. */
void lbm_batch_free(lbm_batch *b);

/* Text of the last failure of c (or of the last failed lbm_init when c is
 * NULL); never NULL. */
const char *lbm_last_error(const lbm_ctx *c);

/* Releases the context and its device memory (synchronizes its stream).
 * NULL is accepted. */
void lbm_free(lbm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
