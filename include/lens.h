/*
 * lens.h -- C ABI of the MI355X (gfx950) image-plane chi^2 library.
 *
 * The library evaluates the strong-lensing goodness of fit of Rexroth,
 * Schaefer, Fourestey & Kneib (2019), "High Performance Computing for
 * gravitational lens modeling: single vs double precision on GPUs and CPUs":
 *   - the deflection gradient grad Psi of a sum of pseudo-elliptical
 *     potentials at every node of a regular image-plane grid (Algorithm 1;
 *     the singular isothermal radial profile generalised to the cored/cut
 *     isothermal profile named in Sec. 5),
 *   - the lens equation in the form of Sec. 2.2.2,
 *     beta = theta - (D_LS/D_OS) grad Psi(theta),
 *   - the re-lensing chi^2 of Sec. 2.2.1-2.2.2 and Fig. 1: observed images to
 *     the source plane, barycentre per system, two triangles per grid cell
 *     mapped to the source plane, containment of the barycentre, predicted
 *     images, chi^2 = sum_i sum_j |x_obs,ij - x_ij|^2 / sigma_ij^2.
 *
 * Conventions shared by every entry point
 *   Units: angles in arcsec, position angle phi in radians counter-clockwise
 *   from the theta_1 axis, velocity dispersion in km/s.
 *   Memory: every array argument is a DEVICE pointer (memory of the device
 *   the context was created on) unless stated otherwise; the caller owns all
 *   of them.  The context owns only its internal scratch.
 *   Streams: all work is enqueued on the given stream and is asynchronous;
 *   outputs are valid once the stream has been synchronised.  The context
 *   keeps per-call scratch, so calls that share one context must be issued on
 *   one stream (or be otherwise serialised); one context per host thread.
 *   Errors: every function returns LENS_OK or a LENS_ERR_* code for problems
 *   visible on the host (null pointers, sizes, grid shape, device errors).
 *   Problems in device-resident values (parameter domains, capacity) are
 *   reported in the device status word (stats[LENS_STAT_STATUS] or the
 *   status argument), and the numeric outputs are then NaN.  No C++
 *   exception crosses this interface.
 */
#ifndef LENS_H
#define LENS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LENS_OK 0
#define LENS_ERR_INVALID 1   /* bad argument or parameter domain             */
#define LENS_ERR_DEVICE 2    /* a HIP call failed                             */
#define LENS_ERR_CAPACITY 3  /* more predicted images than the output holds  */
#define LENS_ERR_SCRATCH 4   /* input too large for lens_image_chi2_noalloc's fixed scratch */

/* Slots of the int64 statistics array written by lens_image_chi2. */
#define LENS_STAT_HITS 0        /* predicted images (triangle hits) found          */
#define LENS_STAT_FLAGGED 1     /* FP32 tests sent to the FP64 fallback            */
#define LENS_STAT_TILE_PASS 2   /* (tile, system) pairs surviving the tile cull    */
#define LENS_STAT_BBOX_PASS 3   /* triangle tests surviving the bounding-box test  */
#define LENS_STAT_STATUS 4      /* LENS_OK or LENS_ERR_INVALID / _CAPACITY         */
#define LENS_STAT_FB_HITS 5     /* hits decided by the FP64 fallback               */
#define LENS_STAT_TESTS 6       /* triangle x system tests in the full problem     */
#define LENS_STAT_N 8

typedef struct lens_ctx lens_ctx;

typedef enum {
    LENS_FP64 = 0,  /* every step in FP64                                        */
    LENS_FP32 = 1,  /* deflection only: FP32 field (lens_deflect)                 */
    LENS_MIXED = 2  /* FP32 field and containment tests, FP64 where the FP32 test
                       cannot decide, FP64 source positions, images and chi^2     */
} lens_precision;

/* Potentials as a structure of arrays (Sec. 2.3), n entries each, device
 * memory, float64.  Domain: 0 <= eps < 1; r_core >= 0; r_cut > r_core
 * (r_cut = +INFINITY: no cut); sigma_v >= 0; all values finite except r_cut.
 * r_core = 0 and r_cut = +INFINITY is the singular isothermal ellipsoid of
 * Algorithm 1.  n may be 0 (no deflection). */
typedef struct {
    int32_t n;
    const double *x, *y;          /* centre, arcsec                              */
    const double *eps;            /* pseudo-ellipticity of the potential         */
    const double *phi;            /* position angle, radians                     */
    const double *r_core, *r_cut; /* core and cut radius, arcsec                 */
    const double *sigma_v;        /* velocity dispersion, km/s                   */
} lens_potentials;

/* Regular grid of nodes: node (i, j) = (x0 + i h, y0 + j h), 0 <= i < nx,
 * 0 <= j < ny; node arrays are row-major [ny][nx].  nx, ny >= 2, h > 0.
 * Cell (i, j) is split along its anti-diagonal into triangle 0 with vertices
 * (i,j), (i+1,j), (i,j+1) and triangle 1 with vertices (i+1,j+1), (i,j+1),
 * (i+1,j); triangle id = 2 (j (nx-1) + i) + k (Fig. 1 of the paper). */
typedef struct {
    double x0, y0, h;
    int32_t nx, ny;
} lens_grid;

/* Observed multiple-image systems (Sec. 2.2.1) in CSR form.  Host-side
 * counts; device arrays. */
typedef struct {
    int32_t n_sys;               /* number of systems (sources), >= 1            */
    int32_t n_img;               /* number of observed images, == sys_off[n_sys] */
    const int32_t *sys_off;      /* [n_sys + 1], non-decreasing, sys_off[0] = 0  */
    const double *x, *y;         /* [n_img] observed positions, arcsec           */
    const double *sigma;         /* [n_img] positional error sigma_ij, arcsec    */
    const double *dls_dos;       /* [n_sys] D_LS/D_OS of each source (Sec. 2.2.2,
                                    computed once per source, e.g. lens_dls_dos) */
} lens_obs;

typedef struct {
    lens_precision prec;  /* LENS_FP64 or LENS_MIXED                                 */
    int32_t fb_mode;      /* MIXED only.  0: a test is sent to FP64 when its FP32 sign
                             is not certified by the FP32 error bound (hit sets equal
                             to the FP64 path).  1: literal threshold, a test is sent
                             to FP64 when min_k |c_k| < fb_tau * h^2                 */
    double fb_tau;        /* literal-mode factor (e.g. 1e-6); ignored in mode 0    */
    int32_t hit_capacity; /* rows of out->hits / out->img_xy, 1 .. 8192            */
    int32_t field_npl;    /* grid nodes per thread of the FP32 field kernel: 1, 2, 4 or
                             8 (batched: 1, 2, 4); 0 = the autotuned choice, else
                             chosen from the grid size (batched: 2)               */
    int32_t tile;         /* cells per triangle-stage tile: 1 = 32x8, 2 = 64x16,
                             3 = 64x8, 4 = 32x16; 0 = the autotuned choice, else
                             32x8                                                 */
} lens_chi2_opts;

typedef struct {
    double *chi2;        /* [1]       total chi^2 (+inf if any system has no image) */
    double *chi2_sys;    /* [n_sys]   per-system chi^2                              */
    int32_t *n_pred;     /* [n_sys]   predicted images per system                   */
    int32_t *hits;       /* [2 * hit_capacity] (system, triangle id) pairs, sorted    */
    double *img_xy;      /* [2 * hit_capacity] predicted image positions (x, y)       */
    int32_t *match;      /* [n_img]   index into hits of each observed image's match,
                                      -1 if its system has no predicted image; may
                                      be NULL                                        */
    int64_t *stats;      /* [LENS_STAT_N] statistics and device status               */
} lens_chi2_out;

/* Create a context on HIP device `device`.  Returns LENS_ERR_INVALID for a
 * null ctx pointer or a bad device, LENS_ERR_DEVICE if HIP fails. */
int lens_create(lens_ctx **ctx, int device);

/* Release the context and its scratch.  Synchronises the device first.
 * NULL is ignored. */
void lens_destroy(lens_ctx *ctx);

/* D_LS/D_OS for n source redshifts zs[n] behind a lens at zl in a flat
 * universe (Omega_m + Omega_Lambda = 1; the paper uses 0.3, 0.7), by
 * composite Simpson quadrature of the comoving distance on the device.
 * zs, out: device float64 [n].  A source at zs <= zl gets 0. */
int lens_dls_dos(lens_ctx *ctx, double zl, const double *zs, int32_t n, double omega_m,
                 double omega_l, double *out, hipStream_t stream);

/* Deflection gradient grad Psi at every node of the grid (Algorithm 1 summed
 * over all potentials; Sec. 2.2.2 superposition).  prec = LENS_FP64: ax, ay
 * are double [ny*nx]; LENS_FP32 or LENS_MIXED: float [ny*nx].  Output layout
 * row-major, node (i,j) at index j*nx + i.  status: device int32 [1] or NULL,
 * receives LENS_OK or LENS_ERR_INVALID (parameter domain; outputs NaN). */
int lens_deflect(lens_ctx *ctx, const lens_potentials *pot, const lens_grid *grid,
                 lens_precision prec, void *ax, void *ay, int32_t *status, hipStream_t stream);

/* Pseudo-elliptical NFW halos (structure of arrays, DEVICE pointers, double,
 * length n): the second profile family the paper names (Sec. 5), in the frame
 * construction of Algorithm 1 (Sec. 2.2.2). */
typedef struct {
    int32_t n;
    const double *x, *y;     /* centre [arcsec]                                        */
    const double *eps;       /* pseudo-ellipticity of the potential, 0 <= eps < 1      */
    const double *phi;       /* position angle [rad]                                   */
    const double *r_s;       /* scale radius [arcsec], > 0                             */
    const double *kappa_s;   /* characteristic convergence rho_s r_s / Sigma_cr, >= 0  */
} lens_nfw;

/* Deflection gradient of NFW halos at every node: with m = M (theta - centre),
 * R^2 = (theta - centre) . m as in Algorithm 1 and x = R / r_s,
 *     alpha = sum over halos of 4 kappa_s g(x)/x^2 m,  g(x) = ln(x/2) + F(x),
 *     F = arccosh(1/x)/sqrt(1 - x^2) (x < 1), 1 (x = 1), arccos(1/x)/sqrt(x^2 - 1) (x > 1)
 * (Bartelmann 1996); a node at a centre gets 0 from that halo.  prec =
 * LENS_FP64: ax, ay double [ny*nx]; LENS_FP32: float [ny*nx] (node offsets from
 * an exact split of each centre, as the FP32 isothermal field).  status: device
 * int32 [1] or NULL: LENS_OK, or LENS_ERR_INVALID for a halo outside the domain
 * (outputs NaN). */
int lens_deflect_nfw(lens_ctx *ctx, const lens_nfw *halos, const lens_grid *grid, lens_precision prec, void *ax,
                     void *ay, int32_t *status, hipStream_t stream);

/* Options of the paper's mixed-precision gradient (Sec. 3.2, 3.3, Appendix A.3). */
typedef struct {
    int32_t n_cluster;      /* the first n_cluster potentials are the cluster-scale halos      */
    int32_t patch_cluster;  /* side of their double-precision pixel blocks (the paper: 400)    */
    int32_t patch_galaxy;   /* side of the blocks of the other (galaxy-scale) halos (paper: 20) */
    double t12;             /* criteria thresholds, arcsec: |dx - d1|, |dx - d2| < t12 ...      */
    double t34;             /* ... or |d3|, |d4| > t34 (paper: 0.0092, 0.0104 for dx = 0.03")  */
} lens_mixed_opts;

/* The paper's mixed-precision gradient of an SIE lens (every potential with
 * r_core = 0 and r_cut = +inf, the model its precision study covers; Sec. 3.2):
 *  1. grad Psi in FP32 at every node (node offsets from an exact split of the
 *     centre, alpha = K M d / R), except
 *  2. FP64 inside a block of patch_cluster^2 nodes centred on each
 *     cluster-scale halo and patch_galaxy^2 nodes on every other halo (node
 *     indices [k - p/2, k - p/2 + p) per axis, k the node nearest the centre,
 *     rounded half away from zero; clipped to the grid);
 *  3. on that field, with dx = grid->dx, d1 = ax(i,j) - ax(i-1,j),
 *     d2 = ay(i,j) - ay(i,j-1), d3 = ax(i,j) - ax(i,j-1), d4 = ay(i,j) - ay(i-1,j)
 *     (differences whose neighbour lies outside the grid are not evaluated),
 *     every other node with |dx - d1| < t12, |dx - d2| < t12, |d3| > t34 or
 *     |d4| > t34 is recomputed in FP64 (Sec. 3.3).
 * ax, ay: device double [ny*nx] (row-major, node (i,j) at j*nx + i).  mask:
 * device uint8 [ny*nx] or NULL; receives 0 (FP32), 1 (FP64 block) or 2 (FP64
 * by the criteria).  stats: device int64 [4]: block nodes, criteria nodes, all
 * FP64 nodes, status (LENS_OK, or LENS_ERR_INVALID for a potential outside the
 * SIE domain: outputs NaN, counts 0).  ny*nx < 2^32.  Host-side argument errors
 * return LENS_ERR_INVALID. */
int lens_deflect_mixed(lens_ctx *ctx, const lens_potentials *pot, const lens_grid *grid,
                       const lens_mixed_opts *opts, double *ax, double *ay, uint8_t *mask, int64_t *stats,
                       hipStream_t stream);

/* Source positions of the observed images and barycentres of the systems
 * (Sec. 2.2.2): beta_ij = theta_ij - (D_LS/D_OS)_i grad Psi(theta_ij) in FP64,
 * barycentre = unweighted mean of the system's beta_ij.  beta_x, beta_y:
 * double [n_img]; bar_x, bar_y: double [n_sys]. */
int lens_source_positions(lens_ctx *ctx, const lens_potentials *pot, const lens_obs *obs,
                          double *beta_x, double *beta_y, double *bar_x, double *bar_y,
                          int32_t *status, hipStream_t stream);

/* Full image-plane chi^2 (Sec. 2.2.1, 2.2.2, Fig. 1).  Each observed image is
 * paired with the nearest predicted image of its system (ties to the lower
 * triangle id); a system without predicted images has chi2_sys = +inf.  If
 * more hits exist than opts->hit_capacity, stats[LENS_STAT_STATUS] =
 * LENS_ERR_CAPACITY, stats[LENS_STAT_HITS] holds the required capacity and
 * chi2 outputs are NaN. */
int lens_image_chi2(lens_ctx *ctx, const lens_potentials *pot, const lens_grid *grid,
                    const lens_obs *obs, const lens_chi2_opts *opts, lens_chi2_out *out,
                    hipStream_t stream);

/* Bytes of the fixed device scratch of lens_image_chi2_noalloc (per device). */
#define LENS_NOALLOC_SCRATCH_BYTES (512ull << 20)

/* lens_image_chi2 for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments (no context), results, status and stream semantics as
 * lens_image_chi2; it runs on the calling thread's current HIP device with the
 * library's default tile shape and field layout for the grid size (or those
 * set in opts), and calls no hipMalloc, hipFree or allocating routine.  Its
 * scratch is one fixed array of LENS_NOALLOC_SCRATCH_BYTES in device memory
 * that the library holds on every device it runs on until the process ends
 * (512 MiB holds a 4096^2 grid with 100 systems in either precision).
 * An input that needs more returns LENS_ERR_SCRATCH before anything is
 * enqueued.  The array's address on a device is looked up once, on the first
 * call on that device or by lens_create for it; that lookup is not a stream
 * operation, so make the first call outside graph capture or create a context
 * on the device first.  Every call on one device shares that array and
 * leaves its contents behind: calls whose work overlaps on one device
 * (different streams, or threads without ordering) race and give wrong
 * results. */
int lens_image_chi2_noalloc(const lens_potentials *pot, const lens_grid *grid, const lens_obs *obs,
                            const lens_chi2_opts *opts, lens_chi2_out *out, hipStream_t stream);

/* Outputs of the batched chi^2 (device arrays). */
typedef struct {
    double *chi2;       /* [n_samples]          total chi^2 of each sample                 */
    double *chi2_sys;   /* [n_samples * n_sys]  per-system chi^2                           */
    int32_t *n_pred;    /* [n_samples * n_sys]  predicted images per system                */
    int32_t *status;    /* [n_samples]          LENS_OK / LENS_ERR_INVALID / _CAPACITY      */
    int64_t *stats;     /* [LENS_STAT_N] totals over the batch; stats[4] is 1 if any sample
                           is not OK, stats[7] the number of such samples                 */
    /* Optional triangle hits of every sample (all three NULL, or all three set):   */
    int32_t *n_hits;    /* [n_samples]          hits of each sample (0 if not OK)         */
    int32_t *hits;      /* [n_samples * 2 * hit_capacity] sample s: (system, triangle id)
                           pairs in rows [s * hit_capacity, s * hit_capacity + n_hits[s]),
                           sorted as lens_image_chi2's                                   */
    double *img_xy;     /* [n_samples * 2 * hit_capacity] predicted image positions (x, y)
                           of those hits                                                  */
} lens_batch_out;

/* Batched image-plane chi^2: n_samples lens models -- the proposals of a
 * sampler over the parameter space (Sec. 2.2.1) -- with their own potentials
 * and grids, sharing the observed systems.  Sample s owns parameter columns
 * [pot_off[s], pot_off[s+1]) of the concatenated structure of arrays `all`
 * and the grid grids[s].  pot_off (n_samples + 1 entries, pot_off[0] = 0,
 * non-decreasing, pot_off[n] = all->n) and grids are HOST arrays: they fix
 * the work plan (heaviest samples first, memory-bounded chunks), which the
 * context caches per distinct (pot_off, grids, opts) and uploads once; a
 * captured HIP graph replays the plan of the captured call.  Each sample is
 * evaluated exactly as lens_image_chi2 would; opts->hit_capacity (<= 1024) is
 * per sample, and a batch needs n_img <= 1024, n_sys <= 1024. */
int lens_image_chi2_batched(lens_ctx *ctx, const lens_potentials *all, int32_t n_samples,
                            const int32_t *pot_off, const lens_grid *grids, const lens_obs *obs,
                            const lens_chi2_opts *opts, lens_batch_out *out, hipStream_t stream);

/* ---------------------------------------------------------------- sampler steps
 *
 * The paper evaluates chi^2 inside a sampler over the lens parameters
 * (Sec. 2.2.1).  Two steps of such samplers run on the device.  A parameter
 * table is a device double array [7][n] (rows x, y, eps, phi, r_core, r_cut,
 * sigma_v, the layout of lens_potentials' arrays placed one after another);
 * step: device double [7][n], a parameter with step 0 is held fixed.  The
 * random numbers are inputs, so a step is a deterministic function of them.
 * Both are stream-ordered and capturable (no host synchronisation). */

/* One Hamiltonian Monte Carlo step on the source-plane chi^2 (lens_src_chi2):
 * potential energy U = chi^2/2, coordinates z = q/step with unit masses,
 * n_leapfrog (1..1000) leapfrog steps of size 1 in z (half momentum kicks at
 * both ends), then acceptance when u < exp(H0 - H1), H = U + |p|^2/2 over the
 * free parameters, and both chi^2 valid.  state: [7][n], replaced by the
 * trajectory's end on acceptance.  momentum: device [7][n] N(0,1) draws; u:
 * device [1] U(0,1) draw; chi2: device [1], receives the chi^2 of the
 * resulting state; accepted: device int32 [1]. */
int lens_hmc_step(lens_ctx *ctx, double *state, int32_t n, const lens_obs *obs, const double *step,
                  int32_t n_leapfrog, const double *momentum, const double *u, double *chi2, int32_t *accepted,
                  hipStream_t stream);

/* One random-walk Metropolis step of n_chains independent chains on the
 * image-plane chi^2 (log-likelihood -chi^2/2), n potentials each, every chain
 * on `grid`: proposals = state + step * noise (multiply and add rounded
 * separately; step [7][n] shared by the chains), evaluated by one
 * lens_image_chi2_batched call with `opts`; chain b accepts when its proposal's
 * status is OK, its chi^2 finite and log u_b < -(chi2_new - chi2_b)/2 (any
 * valid proposal when chi2_b is not finite).  states: device [7][n_chains*n]
 * (chain b owns columns [b*n, b*n + n)), updated; noise: device
 * [7][n_chains*n] N(0,1); u: device [n_chains] U(0,1); chi2: device
 * [n_chains], the current chains' chi^2 on input (e.g. from
 * lens_image_chi2_batched), updated; accepted: device int32 [n_chains]. */
int lens_mh_step_batched(lens_ctx *ctx, double *states, int32_t n_chains, int32_t n, const lens_grid *grid,
                         const lens_obs *obs, const lens_chi2_opts *opts, const double *step, const double *noise,
                         const double *u, double *chi2, int32_t *accepted, hipStream_t stream);

/* ---------------------------------------------------------------- autotuning
 *
 * A context keeps a table of the fastest triangle-stage tile shape
 * (lens_chi2_opts.tile) and FP32 field nodes per thread (.field_npl) per
 * bucket (precision, single or batched call, ceil(log2 of the grid side
 * max(nx, ny)), ceil(log2 of the potential count P)); for a batch the side is
 * the largest over the samples and P the rounded-up mean.  A call whose
 * opts->tile or opts->field_npl is 0 takes the table's choice for its bucket
 * when there is one, else the fixed default.  lens_create merges the JSON file
 * named by the environment variable LENS_AUTOTUNE_CACHE, if it exists and
 * parses (otherwise the table starts empty).  Entries carry the GPU
 * architecture (e.g. gfx950); a file written on another one adds nothing. */

/* Times the candidates on the caller's problem -- the default configuration
 * first, then the other nodes per thread 1, 2, 4, 8 (MIXED only) with tile
 * shape 1, then the other tile shapes with the best of those -- each by one
 * warm-up and `reps` (1..100) timed calls (median, HIP events on `stream`).  A
 * candidate replaces the best so far only when it is more than 2 % faster
 * (timing noise keeps the default).  Records the choice in the table and
 * leaves `out` holding the result of one more call with it.  opts->tile and
 * opts->field_npl are ignored; a candidate whose scratch bound is exceeded
 * (LENS_ERR_CAPACITY) is skipped.  Synchronises `stream` (not capturable).
 * tile, field_npl: host, may be NULL; receive the choice (field_npl 0 for
 * FP64, where it has no effect). */
int lens_autotune_chi2(lens_ctx *ctx, const lens_potentials *pot, const lens_grid *grid, const lens_obs *obs,
                       const lens_chi2_opts *opts, lens_chi2_out *out, int32_t reps, int32_t *tile,
                       int32_t *field_npl, hipStream_t stream);

/* The same for lens_image_chi2_batched (nodes per thread 1, 2, 4). */
int lens_autotune_chi2_batched(lens_ctx *ctx, const lens_potentials *all, int32_t n_samples,
                               const int32_t *pot_off, const lens_grid *grids, const lens_obs *obs,
                               const lens_chi2_opts *opts, lens_batch_out *out, int32_t reps, int32_t *tile,
                               int32_t *field_npl, hipStream_t stream);

/* The table's choice for the bucket of (prec, batched 0/1, grid side n_side,
 * n_pot potentials): *tile, *field_npl (host), both 0 if the table has none. */
int lens_autotune_lookup(lens_ctx *ctx, lens_precision prec, int32_t batched, int32_t n_side, int32_t n_pot,
                         int32_t *tile, int32_t *field_npl);

/* Writes the table as JSON (through a temporary file renamed into place);
 * LENS_ERR_INVALID if it cannot be written. */
int lens_autotune_save(lens_ctx *ctx, const char *path);

/* Merges a JSON table written by lens_autotune_save (an entry replaces the
 * one of its bucket).  LENS_ERR_INVALID for a missing or malformed file, which
 * leaves the table unchanged. */
int lens_autotune_load(lens_ctx *ctx, const char *path);

/* ---------------------------------------------------------------- backward form
 *
 * The paper has no derivatives.  These are the analytic derivatives of the
 * deflection of Algorithm 1, generalised to the cored/cut profile
 * (Sec. 2.2.2), with respect to the seven parameters of every potential, in
 * the order of lens_potentials: x, y, eps, phi, r_core, r_cut, sigma_v.  A
 * parameter gradient `grad` is a device double array [7 * n], row-major
 * [parameter][potential], the layout of a [7, n] parameter table.  Derivatives
 * with respect to an infinite r_cut are 0; the centre of a singular profile
 * contributes nothing (as in the forward deflection).  Potentials outside the
 * model's domain give NaN gradients and status LENS_ERR_INVALID. */

/* Vector-Jacobian product of the deflection field:
 *     grad[k*n + p] = sum over nodes of g_ax * d ax/d q + g_ay * d ay/d q,
 * q = parameter k of potential p.  g_ax, g_ay: device double [ny*nx], the
 * layout of lens_deflect's output.  prec = LENS_FP64: every product in FP64;
 * LENS_FP32: per-node products in FP32 (node offsets from the same exact
 * centre split as the FP32 field), summed per thread over 16 nodes in FP32
 * and reduced in FP64.  Deterministic (fixed reduction order).  status:
 * device int32 [1] or NULL. */
int lens_deflect_backward(lens_ctx *ctx, const lens_potentials *pot, const lens_grid *grid,
                          lens_precision prec, const double *g_ax, const double *g_ay, double *grad,
                          int32_t *status, hipStream_t stream);

/* Source-plane chi^2 of the observed systems (FP64): beta_ij = theta_ij -
 * (D_LS/D_OS)_i grad Psi(theta_ij) (Sec. 2.2.2), bar_i the unweighted mean of
 * system i's beta_ij, chi2 = sum_i sum_j |beta_ij - bar_i|^2 / sigma_ij^2,
 * summed in a fixed order.  chi2: device double [1].  The paper's chi^2 is the
 * image-plane one; this source-plane form is the differentiable companion of
 * the backward form. */
int lens_src_chi2(lens_ctx *ctx, const lens_potentials *pot, const lens_obs *obs, double *chi2,
                  int32_t *status, hipStream_t stream);

/* Gradient of the source-plane chi^2: grad = g_chi2 * d chi2/d q (FP64), with
 * d beta_ij/d q = -(D_LS/D_OS)_i d grad Psi(theta_ij)/d q.  g_chi2: device
 * double [1] (the upstream derivative) or NULL for 1.  Recomputes the
 * forward pass. */
int lens_src_chi2_backward(lens_ctx *ctx, const lens_potentials *pot, const lens_obs *obs,
                           const double *g_chi2, double *grad, int32_t *status, hipStream_t stream);

/* Kernel timing (instrumentation, for roofline measurement).  While enabled,
 * every launch of the deflection-field kernel (the dominant kernel of
 * lens_deflect and lens_image_chi2) and of the two kernels of
 * lens_deflect_backward is bracketed by HIP events recorded on
 * the call's stream.  lens_field_timing waits for the recorded events and
 * returns the summed kernel time in milliseconds and the number of launches
 * since the last reset (reset != 0 clears the totals).  Do not enable while a
 * stream is being captured into a graph. */
int lens_set_timing(lens_ctx *ctx, int enable);
int lens_field_timing(lens_ctx *ctx, double *total_ms, int64_t *launches, int reset);

/* Human-readable name of a return code (static string). */
const char *lens_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LENS_H */
