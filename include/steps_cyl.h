/*
 * steps_cyl.h -- C ABI of the MI355X (gfx950) library for direct-sum gravity
 * in a domain periodic along z (period L) and open in x and y: the S1 x R2
 * topology of cylindrical StePS (Sect. 2.1, eq. ForceCylindrical).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - G = 1 and scale factor a = 1 inside force calls: the returned
 *    acceleration of particle i is
 *        a_i = sum_{j != i} sum_{n=-n_img}^{n_img} -m_j F(|s|, h_i + h_j) s/|s|,
 *    s = (x_i - x_j, y_i - y_j, w(z_i - z_j) - n L), with F the cubic-spline
 *    softened force law (Sect. 2.1, eq. Force_spline_kernel, the pair
 *    softening h_i + h_j of eq. ComovingEquationsOfMotion) and
 *    w(t) = t - L floor(t/L + 1/2) the minimum-image separation.  The image
 *    window |n| <= n_img about the minimum image is the cylinder of
 *    half-height (n_img + 1/2) L centred on each target (the paper's N_cut
 *    cut-off read with a half-integer value, identical for i->j and j->i).
 *    The potential is phi_i = sum m_j P(|s|, h_i + h_j) with dP/dr = F and
 *    P(inf) = 0, so P = -1/r outside the softening length.
 *  - Self pairs j == i are excluded, images included.  Coincident distinct
 *    particles feel no force and contribute P(0) = -2.8 / (h_i + h_j).
 *  - Particle data are caller-owned DEVICE arrays in structure-of-arrays
 *    layout: pos = [x_0..x_{N-1} | y_0..y_{N-1} | z_0..z_{N-1}] (FP64, 3N
 *    doubles), mass[N] >= 0 and eps[N] > 0 (FP64; eps_i is the softening
 *    length h_i).  z may lie anywhere; it is wrapped into [0, L) in FP64 as
 *    z - L floor(z/L) before use.  Outputs are caller-owned device arrays.
 *    The library never frees caller memory.
 *  - Workspace: the force entry points that need device scratch (spatial
 *    order, staged records, partial sums) come in two forms.  The *_ws form
 *    takes a caller-owned device workspace (workspace, workspace_bytes) and
 *    allocates nothing; steps_cyl_forces_workspace() returns the bytes it
 *    needs on the current device (STEPS_EINVAL if the workspace is smaller).
 *    Its contents are undefined after the call; calls that share one
 *    workspace must be ordered on one stream.  The plain form takes the same
 *    amount as stream-ordered memory (hipMallocAsync on `stream`, released
 *    with hipFreeAsync on it after the call's launches; STEPS_ENOMEM if it
 *    cannot be had).  Network, table and tree handles own their memory.
 *  - Target order: with 4096 or more targets, the per-target entry points
 *    (steps_cyl_forces_ex in its per-target modes,
 *    steps_cyl_forces_learned_ex, steps_cyl_forces_table with a list) first
 *    sort the targets by a 30-bit Morton key of (x, y, z) so that each
 *    workgroup holds neighbours; every output stays at its target's position
 *    and every target's result is bitwise that of the unsorted walk.  The
 *    keys (about 16 bytes per target plus the radix sort's storage) live in
 *    the workspace.
 *  - Short target lists: when a per-target call's target blocks alone would
 *    not fill the device, the sources are split into C chunks of at least
 *    4096 (C = min(ceil(2048 / target blocks), ceil(N / 4096)), target blocks
 *    of 256 targets, 128 with a network); each chunk's compensated totals go
 *    to the workspace in FP64 (32 C bytes per target) and are added in chunk
 *    order.  Results are deterministic, and two calls on the same particles
 *    give a target bit for bit the same result whenever they take the same
 *    C (always for N <= 4096); otherwise they agree to FP32 rounding.
 *  - Every call is asynchronous on `stream` (0 = the null stream); results
 *    are valid after the stream is synchronised.  Argument errors are found
 *    on the host before any device work and return a negative status; the
 *    device data themselves are not validated (NaN/negative masses or
 *    softenings <= 0 give unspecified, but finite-time, results).
 *  - No C++ exception crosses this interface.  steps_cyl_last_error() returns
 *    a message for the last non-OK status of the calling thread.
 */
#ifndef STEPS_CYL_H
#define STEPS_CYL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STEPS_OK = 0,
    STEPS_EINVAL = -1,   /* invalid argument (null pointer, size, range)      */
    STEPS_EDOMAIN = -2,  /* argument outside the supported domain             */
    STEPS_ENODEV = -3,   /* no usable gfx950 device                           */
    STEPS_EHIP = -4,     /* a HIP runtime call or kernel launch failed        */
    STEPS_ENOMEM = -5,   /* allocation failed (network handles only)          */
    STEPS_EIO = -6       /* file missing, truncated or of the wrong format    */
} steps_status;

/* Largest image count accepted by the force entry points. */
#define STEPS_MAX_NIMG 4096

/* Largest particle count (and target-list length) accepted by every entry
 * point: 2^29, so that the kernels' 32-bit offsets into the SoA arrays
 * (component c of particle i at c*N + i, c <= 3) never overflow. */
#define STEPS_MAX_N (1LL << 29)

typedef struct steps_cyl_table steps_cyl_table;   /* opaque; owns device memory (see below) */

/* Force paths, for steps_cyl_forces_workspace. */
#define STEPS_PATH_EXACT   0   /* steps_cyl_forces[_ws], steps_cyl_forces_ex[_ws]          */
#define STEPS_PATH_LEARNED 1   /* steps_cyl_forces_learned[_ws], _learned_ex[_ws]          */
#define STEPS_PATH_TABLE   2   /* steps_cyl_forces_table[_ws]                              */
#define STEPS_PATH_F64     3   /* steps_cyl_forces_f64[_ws]                                */

/* Summation modes of steps_cyl_forces_ex. */
#define STEPS_SUM_COMPENSATED 0   /* FP32 pairs, Kahan-compensated per-target sums */
#define STEPS_SUM_PLAIN       1   /* FP32 pairs, plain FP32 per-target sums        */
#define STEPS_SUM_PAIRWISE    2   /* every unordered pair once, all targets only   */

/*
 * steps_cyl_forces -- exact image-sum accelerations (and potentials) of all N
 * particles.  Paper: Sect. 2.1, eqs. ComovingEquationsOfMotion (pair sum),
 * Force_spline_kernel, NewtonianForce and ForceCylindrical.
 *
 *   pos      device, 3N doubles, SoA (x | y | z)
 *   mass     device, N doubles, >= 0
 *   eps      device, N doubles, > 0 (softening length h_i)
 *   N        number of particles, 1 <= N <= STEPS_MAX_N
 *   L        period along z, finite and > 0
 *   n_img    images n = -n_img..n_img per pair, 0 <= n_img <= STEPS_MAX_NIMG
 *   out_acc  device, 3N floats, SoA (a_x | a_y | a_z), written
 *   out_pot  device, N floats, written; or NULL to skip the potential
 *   stream   HIP stream
 *
 * Every unordered pair is evaluated once and applied to both particles: the
 * pair term is odd in the separation (the image set of (j, i) is the negated
 * set of (i, j)), so the reaction is the action with dx, dy and F_z negated
 * (F_z keeps its sign where both particles take the minimum image -L/2).
 * Arithmetic: pair separations and the z wrap in FP64, FP32 pair terms,
 * FP64 sums.  Groups of 64 S particles in spatial order (S parts of 64,
 * one particle per lane of a one-wave workgroup) meet in a fixed
 * round-robin tournament (one launch per round, no atomics), so repeated
 * calls are bitwise equal.  Total momentum is conserved to the rounding of
 * the sums.  Workspace (stream-ordered here; see steps_cyl_forces_ws): 32
 * bytes per particle for the records, 64 S for 2S slots of FP64 sums (S = 16
 * parts per group up to N = 2^21, else 8), 1 for boxes, plus the spatial
 * order's 16 bytes per particle and radix-sort storage (about 1.05 GiB at
 * N = 2^20).  Returns STEPS_OK, or STEPS_EINVAL / STEPS_ENOMEM / STEPS_EHIP.
 */
int steps_cyl_forces(const double *pos, const double *mass, const double *eps,
                     int64_t N, double L, int n_img,
                     float *out_acc, float *out_pot, hipStream_t stream);

/*
 * steps_cyl_forces_workspace -- device workspace, in bytes, that the *_ws
 * form of a force call needs on the current device (no device work).
 *
 *   path       STEPS_PATH_EXACT, _LEARNED, _TABLE or _F64 (see above)
 *   N          particles, 1 <= N <= STEPS_MAX_N
 *   n_img      image count of an exact or FP64 call (otherwise ignored)
 *   n_targets  0 for a call with targets NULL (every particle), else the
 *              length of its target list
 *   mode       summation mode of an exact or learned call: STEPS_SUM_PAIRWISE
 *              for steps_cyl_forces_ws and steps_cyl_forces_learned_ws
 *   table, order  the table and order of a table call (else NULL, 0)
 *   potential  nonzero if the call passes out_pot
 *   bytes      receives the size (0 if the call needs none)
 *
 * Returns STEPS_OK, STEPS_EINVAL or STEPS_ENODEV.
 */
int steps_cyl_forces_workspace(int path, int64_t N, int n_img, int64_t n_targets, int mode,
                               const steps_cyl_table *table, int order, int potential,
                               size_t *bytes);

/* steps_cyl_forces with a caller-owned device workspace of workspace_bytes
 * (at least what steps_cyl_forces_workspace returns for STEPS_PATH_EXACT,
 * n_targets 0, STEPS_SUM_PAIRWISE); allocates nothing.  Same results, bit
 * for bit, as steps_cyl_forces on the same device. */
int steps_cyl_forces_ws(const double *pos, const double *mass, const double *eps,
                        int64_t N, double L, int n_img, float *out_acc, float *out_pot,
                        void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * steps_cyl_forces_noalloc -- steps_cyl_forces for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same pairwise path and arguments,
 * with its workspace in a fixed 128 MiB array of the library's device image
 * instead of per-call memory.  Each device the library runs on holds its own
 * copy of the array until the process ends.  Calls no allocator.
 *
 *   N   1 <= N <= STEPS_NOALLOC_MAX_N (2^20); larger N return STEPS_EINVAL
 *       with a message naming the limit, before any device work
 *
 * Groups hold 16 parts as in steps_cyl_forces, or fewer (fewer sum slots)
 * where the workspace would not fit the array (above N = 125,000); with
 * fewer the sums run in another (fixed) order than in steps_cyl_forces and
 * the results agree with it to FP32 rounding, otherwise bit for bit.  Every call on a device shares that
 * device's array and finds it as the last call left it (nothing in it needs
 * to start at zero): calls that overlap on one device, on different streams
 * or from different threads, race and give undefined results.
 */
#define STEPS_NOALLOC_MAX_N (1LL << 20)
int steps_cyl_forces_noalloc(const double *pos, const double *mass, const double *eps,
                             int64_t N, double L, int n_img,
                             float *out_acc, float *out_pot, hipStream_t stream);

/*
 * steps_cyl_forces_ex -- as steps_cyl_forces, for a subset of targets and a
 * chosen summation mode.  Sources are always all N particles.
 *
 *   targets    device, n_targets int64 indices in [0, N) (repeats allowed),
 *              or NULL for every particle (then n_targets must equal N)
 *   n_targets  number of targets, 1 <= n_targets <= STEPS_MAX_N
 *   mode       STEPS_SUM_COMPENSATED (one thread per target, FP32 pair
 *              terms, Kahan-compensated FP32 sums, bitwise deterministic),
 *              STEPS_SUM_PLAIN (the same with plain FP32 sums), or
 *              STEPS_SUM_PAIRWISE (the path of steps_cyl_forces; targets
 *              must be NULL, else STEPS_EINVAL)
 *   out_acc    device, 3 * n_targets floats, SoA by target position k
 *   out_pot    device, n_targets floats or NULL
 *
 * Indices outside [0, N) are not checked on the device: the caller owns that
 * precondition.
 */
int steps_cyl_forces_ex(const double *pos, const double *mass, const double *eps,
                        int64_t N, double L, int n_img,
                        const int64_t *targets, int64_t n_targets, int mode,
                        float *out_acc, float *out_pot, hipStream_t stream);

/* steps_cyl_forces_ex with a caller-owned workspace (STEPS_PATH_EXACT). */
int steps_cyl_forces_ex_ws(const double *pos, const double *mass, const double *eps,
                           int64_t N, double L, int n_img,
                           const int64_t *targets, int64_t n_targets, int mode,
                           float *out_acc, float *out_pot, void *workspace,
                           size_t workspace_bytes, hipStream_t stream);

/*
 * steps_cyl_forces_f64 -- the same sum with every operation in FP64 on the
 * GPU (a slow reference for precision studies; same definitions, same
 * arguments as steps_cyl_forces_ex, FP64 outputs).  Sources are split into
 * chunks so that small target sets fill the GPU; the chunk partials (32
 * bytes per target and chunk) live in the workspace.
 */
int steps_cyl_forces_f64(const double *pos, const double *mass, const double *eps,
                         int64_t N, double L, int n_img,
                         const int64_t *targets, int64_t n_targets,
                         double *out_acc, double *out_pot, hipStream_t stream);

/* steps_cyl_forces_f64 with a caller-owned workspace (STEPS_PATH_F64). */
int steps_cyl_forces_f64_ws(const double *pos, const double *mass, const double *eps,
                            int64_t N, double L, int n_img,
                            const int64_t *targets, int64_t n_targets,
                            double *out_acc, double *out_pot, void *workspace,
                            size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned far-image correction.
 *
 * For a pair at minimum-image axial offset d and cylindrical separation rho,
 * the images 2 <= |n| <= 1024 of eq. ForceCylindrical are replaced by
 *     R_z   = sign(d) [ b_z(|d|, rho)   + s(rho) o_z ]
 *     R_rho =           b_rho(|d|, rho) + s(rho) o_rho       (per G m_j / L^2)
 * where (o_z, o_rho) is a network 2 -> 64 -> 64 -> 64 -> 64 -> 2 (activation
 * s(u) = u/(1 + 2^-u) = SiLU(u ln 2)/ln 2 after every hidden layer, i.e. SiLU
 * with ln 2 absorbed into the weights) of the features f1 = 4|d|/L - 1 and
 * f2 = 2 ln(rho / (0.05 L)) / ln 400 - 1, s(rho) = 0.02 / (1 + (rho/L)^2),
 * and b is a fixed analytic baseline: the images on each side replaced by a
 * uniform rod from 1.5 L to 1024.5 L, plus the first midpoint-rule
 * correction at 1.5 L.  The network domain is 0.05 <= rho/L <= 20; pairs
 * outside it use the exact image band (for rho/L < 0.05 evaluated from a
 * convergent series in rho^2 whose image sums are held as polynomials in
 * (d/L)^2, equal to the direct sum to FP32 rounding; beyond rho/L = 20 summed
 * image by image).  Sign folding makes R_z odd and R_rho
 * even in d, so learned pair forces stay antisymmetric (momentum is
 * conserved).  This stands in for the paper's interpolated correction table
 * D(rho, z) (Sect. 2.2, eq. S1R2EwaldCorrectionTable) as the way to add the
 * far images to nearest-image forces.
 *
 * Parameters: 12802 FP32 values in the order W1 (64x2), b1 (64), W2 (64x64),
 * b2, W3, b3, W4, b4, W5 (2x64), b5 (2); weights (fan_out, fan_in)
 * row-major.  Evaluation rounds every weight to BF16 and the inputs of layers
 * 2-4 to BF16 (round-to-nearest-even); layers 2-4 run on BF16 MFMA with FP32
 * accumulation, layers 1 and 5 and the activations in FP32.
 * ---------------------------------------------------------------------- */
#define STEPS_MLP_PARAMS 12802

typedef struct steps_cyl_mlp steps_cyl_mlp;   /* opaque; owns device memory */

typedef struct {
    const double *train_in;   /* device [2][n_train]: |d|/L then rho/L (FP64)       */
    int64_t n_train;          /* a power of two >= 32                               */
    const double *val_in;     /* device [2][n_val] or NULL                          */
    int64_t n_val;
    int64_t steps;            /* optimiser steps                                    */
    int64_t batch;            /* samples per step, 32 <= batch <= n_train           */
    float lr, lr_min;         /* cosine schedule from lr (first step) to lr_min     */
    float beta1, beta2, adam_eps;  /* Adam (Kingma & Ba) hyper-parameters          */
    uint64_t seed;            /* order of the samples (one permutation per pass)    */
    int64_t eval_every;       /* record the losses every this many steps (0: never) */
    float *history;           /* host [3 * history_len]: step, batch loss, val loss */
    int64_t history_len;
} steps_cyl_train_cfg;

/* Creates a network from 12802 host FP32 parameters (copied).  Allocates
 * device memory owned by the handle.  STEPS_EINVAL for null pointers or
 * non-finite values, STEPS_ENODEV, STEPS_ENOMEM. */
int steps_cyl_mlp_create(const float *init_params, steps_cyl_mlp **out);

/* Releases the handle and its device memory (NULL is ignored). */
void steps_cyl_mlp_destroy(steps_cyl_mlp *net);

/* Copies the FP32 master parameters to host_out[12802] (synchronous). */
int steps_cyl_mlp_get_params(const steps_cyl_mlp *net, float *host_out);

/* Replaces the parameters with host_params[12802] and resets Adam's state
 * (synchronous). */
int steps_cyl_mlp_set_params(steps_cyl_mlp *net, const float *host_params);

/* Network outputs for B feature pairs: in = device [2][B] FP32 (f1 | f2),
 * out = device [2][B] FP32 (o_z | o_rho). */
int steps_cyl_mlp_forward(const steps_cyl_mlp *net, const float *in, float *out, int64_t B,
                          hipStream_t stream);

/* Loss mean((o - target)^2) over both outputs of B samples and its gradient
 * with respect to the FP32 master parameters: in, target = device [2][B]
 * FP32, grad_out = device [12802] FP32, loss_out = device float or NULL.
 * Allocates per-call scratch ((B/32) x 12802 floats) and synchronises the
 * stream before returning.  1 <= B <= 2^24. */
int steps_cyl_mlp_grad(const steps_cyl_mlp *net, const float *in, const float *target, int64_t B,
                       float *grad_out, float *loss_out, hipStream_t stream);

/* Training samples: for in = device [2][n] FP64 (|d|/L, rho/L), writes the
 * features (device [2][n] FP32) and the fit targets (exact band - baseline)/s
 * (device [2][n] FP32), the band summed in FP64. */
int steps_cyl_mlp_samples(const double *in, int64_t n, float *features, float *targets,
                          hipStream_t stream);

/* Trains the network with Adam on minibatches of the samples generated from
 * cfg->train_in.  Allocates its scratch for the call and synchronises the
 * stream before returning.  Not thread-safe on one handle. */
int steps_cyl_mlp_train(steps_cyl_mlp *net, const steps_cyl_train_cfg *cfg, hipStream_t stream);

/* Saves the FP32 master parameters: 8-byte magic "SCYLMLP1", uint32 format
 * version 1, uint32 parameter count, the parameters, a 64-bit FNV-1a
 * checksum of them.  STEPS_EIO on write errors. */
int steps_cyl_mlp_save(const steps_cyl_mlp *net, const char *path);

/* Loads a file written by steps_cyl_mlp_save into a new handle.  STEPS_EIO
 * for a missing, truncated, oversized or corrupt file (magic, version, count
 * or checksum), before any device allocation. */
int steps_cyl_mlp_load(const char *path, steps_cyl_mlp **out);

/*
 * steps_cyl_forces_learned -- accelerations of all N particles with the
 * exact images |n| <= 1 (spline-softened, as steps_cyl_forces with n_img = 1)
 * plus the learned correction for the images 2 <= |n| <= 1024 (see above),
 * i.e. an approximation of steps_cyl_forces with n_img = 1024.  Pairs with
 * rho/L < 0.05 or rho/L > 20 (and no others) use the exact band instead of
 * the network.  out_pot, when non-NULL, receives the potential of the images
 * |n| <= 1 only (the network has no potential output).  Arguments as
 * steps_cyl_forces; `net` is a handle from steps_cyl_mlp_create/_load.
 * Softening of the replaced images is not modelled (they lie at least 1.5 L
 * away; h_i + h_j below that is assumed).  The learned pair term is odd in
 * the separation (R_z odd in d, R_rho even), so, as in steps_cyl_forces,
 * every unordered pair is evaluated once and applied to both particles, with
 * FP64 sums: groups of 1024 particles (8 sub-groups of 128) meet in the
 * round-robin tournament of steps_cyl_forces (no atomics; repeated calls
 * are bitwise equal).
 * Workspace about 80 bytes per particle (records, sums, spatial order).
 */
int steps_cyl_forces_learned(const double *pos, const double *mass, const double *eps,
                             int64_t N, double L, const steps_cyl_mlp *net,
                             float *out_acc, float *out_pot, hipStream_t stream);

/* steps_cyl_forces_learned with a caller-owned workspace (STEPS_PATH_LEARNED,
 * n_targets 0, STEPS_SUM_PAIRWISE). */
int steps_cyl_forces_learned_ws(const double *pos, const double *mass, const double *eps,
                                int64_t N, double L, const steps_cyl_mlp *net,
                                float *out_acc, float *out_pot, void *workspace,
                                size_t workspace_bytes, hipStream_t stream);

/* As steps_cyl_forces_learned for a target subset and summation mode
 * (arguments as steps_cyl_forces_ex): per target (STEPS_SUM_COMPENSATED,
 * STEPS_SUM_PLAIN; bitwise deterministic) or, with targets NULL,
 * STEPS_SUM_PAIRWISE (the path of steps_cyl_forces_learned). */
int steps_cyl_forces_learned_ex(const double *pos, const double *mass, const double *eps,
                                int64_t N, double L, const steps_cyl_mlp *net,
                                const int64_t *targets, int64_t n_targets, int mode,
                                float *out_acc, float *out_pot, hipStream_t stream);

/* steps_cyl_forces_learned_ex with a caller-owned workspace
 * (STEPS_PATH_LEARNED). */
int steps_cyl_forces_learned_ex_ws(const double *pos, const double *mass, const double *eps,
                                   int64_t N, double L, const steps_cyl_mlp *net,
                                   const int64_t *targets, int64_t n_targets, int mode,
                                   float *out_acc, float *out_pot, void *workspace,
                                   size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Tabulated far-image correction (Sect. 2.2, eq. S1R2EwaldCorrectionTable:
 * a correction tabulated on an equally spaced grid in the cylindrical
 * coordinates, interpolated with CIC or TSC and added to the nearest-image
 * forces).  A table holds an image band of one unit mass,
 * T = (T_z, T_rho) per G m / L^2, at delta = |d|/L = i/(2 n_delta)
 * (i = -1..n_delta+1) and r = rho/L = j rho_max/n_rho (j = -1..n_rho+1),
 * computed in FP64 and stored in FP32; R_z = sign(d) T_z, R_rho = T_rho.
 * The table is in units of L, so one table serves every period.
 *   band table:     the images 2 <= |n| <= n_far, summed directly; pairs
 *                   with rho/L > rho_max use the exact band.
 *   complete table: every image |n| >= 2 (N_cut -> infinity), from the
 *                   Ewald split (Sect. 2.2, eqs. cylindricalEwaldSplit,
 *                   EwaldRealSum, EwaldRecSum); pairs with rho/L > rho_max
 *                   use the line-mass limit F_rho = -2 G m/(L rho) of the
 *                   complete sum (its modes decay as exp(-2 pi rho/L)).
 * ---------------------------------------------------------------------- */

#define STEPS_TABLE_MAX_FAR (1 << 24)

/* Builds a band table (device memory owned by the handle; synchronises
 * stream).  2 <= n_delta, n_rho <= 4096; 0 < rho_max <= 1e4;
 * 2 <= n_far <= STEPS_TABLE_MAX_FAR (n_far = 10^7 is the direct reference of
 * Fig. 2). */
int steps_cyl_table_create(int n_delta, int n_rho, double rho_max, int n_far,
                           hipStream_t stream, steps_cyl_table **out);

/* Fourier kernels of the Ewald split. */
#define STEPS_EWALD_BESSEL  0   /* B(k,rho) = int_{1/(4 alpha^2)}^inf exp(-k^2 t - rho^2/(4t)) dt/(2t),
                                   force (4/L) grad[cos(k d) B]: the Poisson sum of the smooth
                                   part for one periodic direction (exact for any alpha)     */
#define STEPS_EWALD_PRINTED 1   /* the kernel of eq. Bkernel with its printed prefactor
                                   -(2/L); matches the complete sum only where its modes
                                   are negligible (alpha scans of Fig. 2)                    */

/* Builds a complete table from the Ewald split with splitting parameter
 * alpha (per 1/L) in (0, 64], real-space images n = -n_max..n_max
 * (1 <= n_max <= 1024) and modes m = 1..m_max (0 <= m_max <= 1024);
 * rho_max >= 4; other arguments as steps_cyl_table_create. */
int steps_cyl_table_create_ewald(int n_delta, int n_rho, double rho_max, double alpha,
                                 int n_max, int m_max, int kernel, hipStream_t stream,
                                 steps_cyl_table **out);

/* Releases a table (NULL is ignored). */
void steps_cyl_table_destroy(steps_cyl_table *table);

/* Copies the nodes to host_out[(n_rho+3) * (n_delta+3) * 2] FP32, node
 * (i, j) at ((j+1) * (n_delta+3) + i+1) * 2 as (T_z, T_rho) (synchronous). */
int steps_cyl_table_values(const steps_cyl_table *table, float *host_out);

/* The same nodes in FP64, as built (synchronous). */
int steps_cyl_table_values_f64(const steps_cyl_table *table, double *host_out);

/* Grid of a table; *n_far = -1 for a complete table.  Any output may be NULL. */
int steps_cyl_table_info(const steps_cyl_table *table, int *n_delta, int *n_rho,
                         double *rho_max, int *n_far);

/* Accelerations with the exact images |n| <= 1 (spline-softened) plus the
 * interpolated band (order 1 = CIC, 2 = TSC); out_pot, when non-NULL, gets
 * the |n| <= 1 potential.  The table's far-image term is odd in d along z
 * and even in d across, so the tabulated pair is antisymmetric like the
 * exact one.  targets NULL (every particle a target): each unordered pair is
 * evaluated once and applied to both particles, with the arithmetic, the
 * fixed schedule (bitwise reproducible) and the workspace of steps_cyl_forces
 * (groups of 512).  An explicit target list: one thread per target with
 * Kahan-compensated FP32 sums, bitwise deterministic.  Other arguments as
 * steps_cyl_forces_ex. */
int steps_cyl_forces_table(const double *pos, const double *mass, const double *eps,
                           int64_t N, double L, const steps_cyl_table *table, int order,
                           const int64_t *targets, int64_t n_targets,
                           float *out_acc, float *out_pot, hipStream_t stream);

/* steps_cyl_forces_table with a caller-owned workspace (STEPS_PATH_TABLE). */
int steps_cyl_forces_table_ws(const double *pos, const double *mass, const double *eps,
                              int64_t N, double L, const steps_cyl_table *table, int order,
                              const int64_t *targets, int64_t n_targets,
                              float *out_acc, float *out_pot, void *workspace,
                              size_t workspace_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Barnes-Hut octree (Sect. 2.4, "Octree": cubic cells, root cell twice the
 * largest linear size of the volume, random shifts along the axis and
 * rotations about it at every step, radial correction table measured on the
 * initial load).
 *
 * The root cube has side S0 = 2 max(L, 2 R_dom) and centre (0, 0, L/2) in
 * the frame rotated by `angle` about the axis and shifted by `shift` along
 * it (z wrapped into [0, L)); R_dom must bound the particles' radius.  Cells
 * are split while they hold more than leaf_size particles (down to level
 * 21); each acts through its mass at its centre of mass (and optionally
 * its quadrupole).  Particles are
 * grouped for the walk into runs of at most 64 made of whole sibling cells
 * (children of a cell holding more than 64, packed in order); a group walks
 * the tree together and accepts a cell when (S0/2^level)^2 < theta^2 d^2 and
 * d^2 > (h_group + h_cell)^2, with d the distance (periodic in z) from the
 * cell's centre of mass to the group's bounding box and h the largest
 * softening lengths; otherwise the cell is opened, and an opened leaf
 * contributes its particles.  Cells and particles interact through the pair
 * of the tabulated scheme (exact images |n| <= 1, softened, plus the
 * table's band), so theta = 0 gives steps_cyl_forces_table's forces.
 *
 * The tree object owns its device buffers (sized on first use, grown when
 * N or the cell count outgrows them; nothing else is allocated) and the
 * radial correction.  Calls on one tree must not overlap.
 * ---------------------------------------------------------------------- */
typedef struct steps_cyl_tree steps_cyl_tree;   /* opaque */

/* 1 <= leaf_size <= 64.  quadrupole 1: cells also carry their traceless
 * quadrupole about the centre of mass, Q_ab = sum m (3 y_a y_b - |y|^2 d_ab),
 * which adds Q s/r^5 - (5/2)(s.Q.s) s/r^7 for each image |n| <= 4 of an
 * accepted cell (the table's band beyond stays a monopole); 0: monopoles
 * only.  No device work. */
int steps_cyl_tree_create(int leaf_size, int quadrupole, steps_cyl_tree **out);

/* Releases the tree and its buffers (NULL is ignored). */
void steps_cyl_tree_destroy(steps_cyl_tree *tree);

/* Builds the tree for pos (device [3][N] FP64), mass, eps (device [N]) in
 * the frame given by shift and angle, walks it and writes out_acc (device
 * [3][N] FP32, caller's order and frame, G = 1).  table and order (1 CIC,
 * 2 TSC) as steps_cyl_forces_table; theta >= 0 the opening angle.  correct:
 * subtract the radial correction set by steps_cyl_tree_set_correction or
 * steps_cyl_tree_calibrate (STEPS_EINVAL if none is set).  1 <= N <= 2^30.
 * Synchronises the stream once per tree level during the build. */
int steps_cyl_tree_forces(steps_cyl_tree *tree, const double *pos, const double *mass,
                          const double *eps, int64_t N, double L, double R_dom,
                          const steps_cyl_table *table, int order, double theta,
                          double shift, double angle, int correct, float *out_acc,
                          hipStream_t stream);

/* Radial correction: mean radial error (tree minus direct tabulated force)
 * per bin of rho, bins of width R_dom/n_bins, over n_real realisations
 * (host arrays shifts[n_real], angles[n_real], the caller's random draws);
 * stored in the tree and copied to out_corr (host [n_bins], may be NULL).
 * Applied by linear interpolation between bin centres, constant beyond the
 * first and the last.  1 <= n_real <= 1024, 1 <= n_bins <= 256.  Costs one
 * direct tabulated evaluation (O(N^2)) plus n_real tree evaluations; its
 * scratch (two [3][N] FP32 force arrays, the bins) is kept by the tree.
 * Synchronous. */
int steps_cyl_tree_calibrate(steps_cyl_tree *tree, const double *pos, const double *mass,
                             const double *eps, int64_t N, double L, double R_dom,
                             const steps_cyl_table *table, int order, double theta,
                             const double *shifts, const double *angles, int n_real,
                             int n_bins, double *out_corr, hipStream_t stream);

/* Sets (host corr[n_bins], bins of width R_dom/n_bins) or, with n_bins = 0,
 * clears the radial correction.  Synchronous. */
int steps_cyl_tree_set_correction(steps_cyl_tree *tree, const double *corr, int n_bins,
                                  double R_dom);

/* Statistics of the last walk: cells, and cell and particle interactions
 * summed over targets.  Any output may be NULL.  Synchronous. */
int steps_cyl_tree_info(const steps_cyl_tree *tree, int64_t *n_cells,
                        int64_t *cell_interactions, int64_t *particle_interactions);

/* The cells of the last build in depth-first order (host arrays of n_cells
 * entries; com is [3][n_cells]) and the caller's index of each particle in
 * key order (host_order[N]).  Any output may be NULL.  Synchronous. */
int steps_cyl_tree_cells(const steps_cyl_tree *tree, int *host_level, int *host_start,
                         int *host_count, int *host_skip, int *host_leaf, double *host_mass,
                         double *host_com, int *host_order);

/* ------------------------------------------------------------------------
 * Time integration (Sect. 2.1, eq. ComovingEquationsOfMotionCylindrical and
 * its kick-drift-kick integrator in cosmic time; Sect. 2.3 background).
 *
 * State: comoving positions x (pos, FP64 SoA) and momenta p = a^2 dx/dt
 * (mom, FP64 SoA, [3][N]); with them the equations of motion read
 *     dp/dt = (g(x) - F_h(x)) / a,   dx/dt = p / a^2,
 * g the pair-sum acceleration of the force entry points (G = 1, a = 1) and
 * F_h the radial field of the homogeneous cylinder (radius R_cyl, comoving
 * density rho0, half-height Z = (n_img + 1/2) L; 1024.5 L with a network;
 * (n_far + 1/2) L with a band table; infinite with a complete table, where
 * F_h = -2 pi G rho0 rho inside R_cyl, eq. F_horiz_infty) that the image
 * sum adds to every particle.  F_h is
 * evaluated from the line-element integral over disk chords (the form that
 * tends to -2 pi G rho0 rho as Z -> infinity; the paper's printed
 * finite-height formula has the opposite sign and half of the logarithmic
 * term).  Background: H(a)^2 = H0^2 (Or a^-4 + Om a^-3 + Ok a^-2 +
 * OL a^{-3(1+w0+wa)} e^{3 wa (a-1)}) (CPL dark energy).
 * ---------------------------------------------------------------------- */
typedef struct {
    double a_begin, a_end;   /* scale factor at the start and the end of the step (> 0)   */
    double H0;               /* Hubble constant in code units (G = 1), > 0                */
    double Omega_m, Omega_L, Omega_r, Omega_k, w0, wa;  /* density parameters, CPL w(a)   */
    double R_cyl, rho0;      /* compensated cylinder: radius and comoving density; R_cyl
                                also bounds the particles' radius for a tree (R_dom)       */
    int compensate;          /* 1: subtract F_h; 0: pair forces only                        */
    int n_img;               /* exact images when net == NULL                               */
    const steps_cyl_mlp *net;  /* learned correction, or NULL for the exact sum            */
    const double *factors;   /* host [3]: (K1, D, K2) to use instead of the Friedmann
                                solution (e.g. from steps_cyl_history_factors), or NULL;
                                the background fields are then not used             */
    const steps_cyl_table *table;  /* tabulated correction (net must be NULL), or NULL   */
    int table_order;         /* 1 = CIC, 2 = TSC, with a table                              */
    steps_cyl_tree *tree;    /* octree forces over `table` (which must be given), or NULL   */
    double theta;            /* opening angle, with a tree                                  */
    double tree_shift, tree_angle;  /* the step's random frame (caller's draws)            */
    int tree_correct;        /* 1: subtract the tree's radial correction                    */
} steps_cyl_kdk_params;

/* Kick and drift factors of one step (host only, no device work):
 * out[0] = int dt/a over the first half, out[1] = int dt/a^2 over the
 * whole step, out[2] = int dt/a over the second half, in cosmic time, with
 * dt = t(a_end) - t(a_begin) (Gauss-Legendre in ln a) and the Friedmann
 * equation advanced by fourth-order Runge-Kutta.  STEPS_EDOMAIN if H^2 is
 * not positive over the step. */
int steps_cyl_kdk_factors(const steps_cyl_kdk_params *params, double *out);

/* Kick and drift factors on a tabulated expansion history (Sect. 2.3:
 * histories given as a table, interpolated linearly, quadratically or
 * cubically).  t[n], a[n] host arrays, both strictly increasing, a > 0;
 * order 1, 2 or 3: on [t_k, t_k+1] the Lagrange polynomial through nodes
 * k..k+1, k..k+2 or k-1..k+2 (shifted inwards at the table ends).  t(a) is
 * found by bisection on the interpolant, the integrals by Gauss-Legendre on
 * each piece.  out[3] as steps_cyl_kdk_factors.  STEPS_EDOMAIN if the step
 * leaves the table.  Host only. */
int steps_cyl_history_factors(const double *t, const double *a, int64_t n, int order,
                              double a_begin, double a_end, double *out);

/* F_h as a vector field at the particle positions: pos device [3][N] FP64,
 * out device [3][N] FP64 (radial in x, y; zero along z), G = 1.  Z > 0 is
 * the half-height; Z = +infinity gives the infinite cylinder,
 * -2 pi G rho0 rho inside R_cyl (eq. F_horiz_infty) and -2 pi G rho0 R^2/rho
 * outside. */
int steps_cyl_compensation(const double *pos, int64_t N, double R_cyl, double Z, double rho0,
                           double *out, hipStream_t stream);

/* One kick-drift-kick step from a_begin to a_end.  On entry acc_inout
 * (device [3][N] FP32) must hold g at pos (from a force call or the previous
 * step); on return pos, mom and acc_inout hold the new state.  z is wrapped
 * into [0, L) in FP64.  One force evaluation per step. */
int steps_cyl_kdk_step(double *pos, double *mom, const double *mass, const double *eps,
                       int64_t N, double L, const steps_cyl_kdk_params *params,
                       float *acc_inout, hipStream_t stream);

/* Message for the last non-OK status returned to the calling thread
 * ("" if none).  The pointer stays valid until the thread's next call. */
const char *steps_cyl_last_error(void);

/* Library version string. */
const char *steps_cyl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STEPS_CYL_H */
