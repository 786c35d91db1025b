/*
 * p3msr.h - C ABI of the MI355X short-range P3M pair-force library.
 *
 * The library computes the short-range ("particle-particle") half of the
 * P3M gravity of the CONCEPT 1.0 paper (arXiv:2112.01508), section 2.1.3,
 * lower half of eq. p3m_gravity, for point particles by default:
 *
 *   a_i = - sum_{j != i, |r_ij| < r_cut} mu_j g(|r_ij| / (2 x_s)) r_ij / |r_ij|^3,
 *   g(u) = erfc(u) + (2 / sqrt(pi)) u exp(-u^2),
 *
 * and with the B-spline softening bracket of the same equation when a
 * softening length is set (p3m_sr_set_softening): mu_j (|r|_B^-3 - |r|^-3) r_ij
 * is then added for |r_ij| < eps_B.  Here mu_j = G m_j and r_ij is the
 * separation to the nearest periodic image of
 * j (the single image n' of eq. p3m_gravity).  The sum is strict
 * (|r| < r_cut); a pair at zero separation contributes nothing.  Receivers
 * are the active particles only; every particle is a supplier (section
 * 2.2.2, individual time steps: particles receive kicks only on their own
 * rung but supply force on every rung).
 *
 * Conventions shared by every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller.  The
 *     library never frees them and only reads inputs / writes outputs.
 *   - pos is n x 3 row-major FP64 (x0 y0 z0 x1 ...); positions outside
 *     [0, box) are wrapped into the box.  Positions must be finite.
 *   - mass is n FP64 values holding G*m_j; NULL means all ones.
 *   - Every call is asynchronous on `stream` (a hipStream_t passed as
 *     void*, NULL = the null stream); pointers must stay valid until the
 *     stream's work has completed.  Parts of a call's build phase run on
 *     streams of the handle (default priority) that wait for `stream` and
 *     that `stream` waits for before the pair kernel, so a call's work is
 *     done when `stream`'s is.  The force calls do not wait for the
 *     GPU: the work-item array is sized by a bound on the item count, and
 *     the pair kernels read the count on the device.  Two cases wait for
 *     the count instead (one small device-to-host read): the deterministic
 *     mode, and layouts whose item bound passes 1 GiB (large rung-batched
 *     calls with several subtiles per tile).  A call that grows the
 *     workspace waits for the stream before freeing the old buffer.
 *   - Outputs are fully overwritten (rows of non-receivers become 0).
 *   - Errors return a negative code, leave outputs untouched when detected
 *     before any launch, and set a per-thread message (p3m_sr_last_error).
 *   - A handle is not thread-safe: use one handle per host thread.
 *
 * Geometry requirements (EINVAL otherwise): box > 0, x_s > 0, r_cut > 0,
 * r_cut < box / 2 (a single nearest image, as eq. p3m_gravity assumes), and
 * floor(box / r_cut) >= 3 tiles per dimension (section 2.1.3: at least three
 * tiles across the box so that no tile pair is visited twice).  r_cut may
 * not exceed 4.5 x_s, the paper's default (EUNSUPPORTED): the kernel-shape
 * fits cover u = r / (2 x_s) <= 2.25.
 */
#ifndef P3MSR_H
#define P3MSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p3m_sr_context *p3m_sr_handle;

typedef enum {
    P3M_FP64 = 0, /* all pair arithmetic in FP64 */
    P3M_FP32 = 1  /* FP32 kernel shape, FP64 accumulation.  The separation, r^2 and the
                     cut-off test are FP64, except with layout screen = 2 on all-active
                     forward calls and on backward calls (p3m_sr_set_config): FP32
                     on cluster-relative
                     coordinates, redone in FP64 where FP32 could decide a pair
                     differently or lose accuracy, so the accepted pairs are the FP64
                     ones */
} p3m_precision;

/* FP32 forward kernel shape (p3m_sr_set_shape) */
typedef enum {
    P3M_SHAPE_POLY = 0,       /* hardware rsqrt + degree-9 polynomial, error 1.9e-7 in g */
    P3M_SHAPE_TAB_NGP = 1,    /* the paper's table on r^2, nearest grid point */
    P3M_SHAPE_TAB_LINEAR = 2  /* the same table, linear interpolation */
} p3m_shape;

enum {
    P3M_OK = 0,
    P3M_EINVAL = -1,      /* invalid argument (no work launched) */
    P3M_ENOMEM = -2,      /* device workspace could not be grown */
    P3M_EHIP = -3,        /* a HIP runtime call failed */
    P3M_EUNSUPPORTED = -4 /* valid request outside what this build supports */
};

/* Per-call counters of the most recent force / backward / batched call. */
typedef struct {
    int64_t n;               /* particles */
    int64_t receivers;       /* receiver rows summed over subsets */
    int64_t interactions;    /* accepted ordered pairs (i receiver, j != i, r < r_cut) */
    int64_t candidates;      /* (receiver, supplier) pairs handed to the pair loop */
    int64_t clusters;        /* receiver groups of <= cluster_size */
    int64_t items;           /* work items of the persistent launch */
    int64_t steps;           /* wavefront steps over suppliers (64 lane-slots each) */
    int32_t tiles_per_dim;   /* tiles per dimension (>= 3) */
    int32_t subtiles_per_dim;/* subtiles per tile per dimension */
    int32_t item_target;     /* work-item size target (supplier candidates) */
    int32_t precision;       /* p3m_precision of the call */
    float ms_build;          /* sort + compaction + planning, when timing is on, else -1 */
    float ms_pairs;          /* the persistent pair-kernel launch, when timing is on, else -1 */
    float ms_total;          /* whole call (GPU side), when timing is on, else -1 */
    int32_t cluster_size;    /* receivers per cluster: 8, 16, 32 or 64 */
    int32_t screen;          /* 1: suppliers screened against each cluster's box */
    int32_t shape;           /* p3m_shape of the FP32 forward kernel shape used */
    int64_t screened;        /* supplier records tested by the screen (0 without it) */
    double eps_b;            /* B-spline softening length of the call (0: none) */
    int64_t fp64_steps;      /* screen 2: wavefront steps that redid a pair in the plain
                                FP64 form (x_i - x_j) - n' box */
    float ms_sort;           /* the counting sort into tile -> subtile -> fine order (keys,
                                scan, scatter, fine order), when timing is on, else -1 */
    int32_t deterministic;   /* 1: the call ran in the deterministic mode (p3m_sr_set_deterministic) */
} p3m_sr_stats;

/* Timings of the most recent p3m_lr_force call (when timing is on, else -1). */
typedef struct {
    int64_t n;               /* particles */
    int32_t n_grid;          /* PM grid points per dimension */
    int32_t pad;
    float ms_sort;           /* counting sort of the particles by CIC node, kernel tables */
    float ms_deposit;        /* CIC deposit (sparse nodes per brick, dense nodes by atomics) */
    float ms_fft_x_fwd;      /* real-to-half-spectrum pass along x */
    float ms_fft_y_fwd;      /* forward pass along y */
    float ms_fft_z_conv;     /* forward z, kernel multiply, inverse z (one pass) */
    float ms_fft_y_inv;      /* inverse pass along y */
    float ms_fft_x_inv;      /* half-spectrum-to-real pass along x */
    float ms_readout;        /* 4-point difference + CIC readout */
    float ms_total;          /* whole call (GPU side) */
} p3m_lr_stats;

/* Counters of the most recent p3m_kdk_step call. */
typedef struct {
    int64_t n;               /* particles */
    int32_t highest_rung;    /* L: highest rung of the period (drift sub-step dt / 2^L) */
    int32_t substeps;        /* drift sub-steps: n_steps 2^L */
    int32_t sr_calls;        /* short-range force evaluations (the start + sub-steps with kicks) */
    int32_t lr_calls;        /* long-range force evaluations (rung-0 kicks) */
    float ms_total;          /* whole call (GPU side), when timing is on, else -1 */
    int32_t pad;
    int64_t interactions;    /* accepted pairs summed over the period's short-range calls */
} p3m_kdk_stats;

/* p3m_kdk_step flags */
enum { P3M_KDK_FIXED_RUNGS = 1 };

/* Create a context on HIP device `device`.  *h receives the handle. */
int p3m_sr_create(p3m_sr_handle *h, int device);

/* Destroy a context and free its workspace (synchronises the device). */
int p3m_sr_destroy(p3m_sr_handle h);

/* Message of the last error on this host thread; never NULL. */
const char *p3m_sr_last_error(void);

/* Library version string; never NULL. */
const char *p3m_sr_version(void);

/*
 * Short-range acceleration (section 2.1.3, lower half of eq. p3m_gravity;
 * with softening when p3m_sr_set_softening set eps > 0).
 *   active  n uint8 (nonzero = receiver) or NULL (all receive).
 *   acc_out n x 3 FP64; rows of non-receivers are set to 0.
 * Ownership: caller owns every array.  Errors: EINVAL for bad geometry,
 * n < 0, NULL pos/acc_out or pointers not 8-byte aligned; ENOMEM when the
 * workspace cannot grow; EHIP on runtime failure.
 */
int p3m_sr_force(p3m_sr_handle h, const double *pos, const double *mass,
                 const uint8_t *active, int64_t n, double box, double x_s, double r_cut,
                 int precision, double *acc_out, void *stream);

/*
 * p3m_sr_force for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, arguments, layout choice and errors, with every
 * workspace buffer carved from one fixed 64 MiB device array that the
 * library holds on each GPU it runs on until the process ends; the call
 * makes no hipMalloc, hipFree or other allocating call.
 * Limits (EUNSUPPORTED, before any launch): n <= 2^18 particles, and the
 * decomposition's buffers (about 150 bytes per particle plus 4 bytes per
 * fine cell and 68 bytes per tile) must fit; if the work items the device
 * plans for the call do not fit in the rest of the array, the call returns
 * EUNSUPPORTED after its first kernels have run and acc_out is undefined.
 * All calls on one GPU share the array: calls that overlap on one GPU (other
 * streams, other threads, other handles) race and must be serialised by the
 * caller.  Every part of the array a call reads is written or cleared by
 * that call.
 */
int p3m_sr_force_noalloc(p3m_sr_handle h, const double *pos, const double *mass,
                         const uint8_t *active, int64_t n, double box, double x_s,
                         double r_cut, int precision, double *acc_out, void *stream);

/*
 * Vector-Jacobian product of p3m_sr_force with respect to positions, for a
 * fixed pair set (the pairs with |r| < r_cut at these positions):
 *   grad_pos_k = sum_i (d acc_i / d x_k)^T grad_acc_i
 *             = - sum_{j: |r_kj| < r_cut} J(r_kj) (mu_j w_k [k act] - mu_k w_j [j act]),
 *   J(r) = (g/r^3) I - (3 g / r^5 + exp(-u^2) / (2 sqrt(pi) x_s^3 r^2)) r r^T,
 * with w = grad_acc.  Rows of grad_acc for non-receivers are ignored.
 * grad_pos is n x 3 FP64, fully overwritten.  Same errors as p3m_sr_force
 * plus EINVAL for NULL grad_acc / grad_pos.
 */
int p3m_sr_force_backward(p3m_sr_handle h, const double *pos, const double *mass,
                          const uint8_t *active, int64_t n, double box, double x_s,
                          double r_cut, int precision, const double *grad_acc,
                          double *grad_pos, void *stream);

/*
 * Rung-batched short-range acceleration: n_sub receiver subsets evaluated at
 * the same positions in ONE persistent launch.  Subset k holds the particles
 * with rung[i] >= min_rung[k] (the kick at hierarchy depth k of the
 * rung-based leapfrog of section 2.2.2 touches every rung >= k); every
 * particle supplies.  Each subset's pairs are evaluated in full.
 *   rung      n uint8 on the device.
 *   min_rung  n_sub uint8 thresholds in HOST memory, 1 <= n_sub <= 64.
 *   acc_out   n_sub x n x 3 FP64 on the device, subset-major.
 */
int p3m_sr_force_batched(p3m_sr_handle h, const double *pos, const double *mass,
                         const uint8_t *rung, int64_t n, int n_sub, const uint8_t *min_rung,
                         double box, double x_s, double r_cut, int precision,
                         double *acc_out, void *stream);

/*
 * Measure-and-keep autotuning (the paper's automatic subtile refinement,
 * section 2.1.3 "Subtiles": try a finer subdivision, time it, keep it if
 * faster).  Times p3m_sr_force on these inputs for candidate subtile counts
 * per dimension crossed with cluster layouts (cluster size, screening, and
 * for all-active forward calls and unsoftened adjoints the mutual layout
 * screen = 2) and,
 * at level >= 2, work-item sizes around the winner; stores the fastest in the
 * handle (a candidate replaces an earlier one only when more than 3 % faster,
 * so near-ties do not flip with timing noise); later calls on the same
 * particle count and geometry use it.
 * acc_scratch is an n x 3 FP64 device buffer the trials write into.
 * level: 1 = subtiles only, 2 = subtiles and item size.  Synchronises.
 * Results persist: each is filed (with its time) in a JSON cache under
 * the device, n, the tile count, the precision, the call kind and the
 * occupancy signature of the particle set (a 32-bin histogram of particles
 * per tile), in the file named by the environment variable P3MSR_TUNE_CACHE
 * (empty: no file) or else $HOME/.cache/p3msr/autotune.json, or the file set
 * with p3m_sr_set_tune_cache.  A handle loads the file when it is created
 * (its device's entries become the layouts later calls use), and an
 * autotune call whose key and signature match a cached entry (normalised
 * histograms within 0.05 in L1) installs it without timing anything, unless
 * level has P3M_TUNE_FORCE.  p3m_sr_tune_status reports which happened.
 * Without P3M_TUNE_ADJOINT the forward is tuned, and the adjoint
 * (p3m_sr_force_backward) takes the same decomposition; with level |
 * P3M_TUNE_ADJOINT the adjoint is timed instead (unit weights on every
 * receiver, workspace of n x 3 doubles for them) and keeps its own winner.
 * When the winner evaluates each pair once for both partners (screen 2),
 * the three fastest of the other candidates are timed again and the
 * fastest of them is kept (and cached, as kind 3 for the forward, 4 for
 * the adjoint) beside it: calls with this key that cannot take screen 2
 * (with an active mask, with a tabulated shape, in the deterministic mode,
 * or softened adjoints) run in that layout.
 */
#define P3M_TUNE_ADJOINT 4
#define P3M_TUNE_FORCE 8
int p3m_sr_autotune(p3m_sr_handle h, const double *pos, const double *mass,
                    const uint8_t *active, int64_t n, double box, double x_s, double r_cut,
                    int precision, int level, double *acc_scratch, void *stream);

/*
 * The same measure-and-keep for the rung-batched call: times
 * p3m_sr_force_batched on these rungs and thresholds (its own subsets, in
 * one launch) for 1 and 2 subtiles per dimension crossed with the screened
 * layouts of 16, 32 and 64 receivers (items of 4096; at level 2 also 1024
 * and 16384 around the winner), each timed once after a warm-up call, and
 * keeps the fastest for
 * later batched calls with this n, geometry, precision and subset count
 * (which otherwise take the forward's layout).  Cached like p3m_sr_autotune.
 * acc_scratch: n_sub x n x 3 FP64 on the device.  level: 1 or 2, optionally
 * | P3M_TUNE_FORCE.  Errors: those of p3m_sr_force_batched.  Synchronises.
 */
int p3m_sr_autotune_batched(p3m_sr_handle h, const double *pos, const double *mass,
                            const uint8_t *rung, int64_t n, int n_sub, const uint8_t *min_rung,
                            double box, double x_s, double r_cut, int precision, int level,
                            double *acc_scratch, void *stream);

/*
 * Use `path` as the autotuner's cache file (NULL: the default of
 * p3m_sr_autotune; "": none) and load it now (its entries for this device
 * become the layouts later calls use).  A missing or unreadable file is an
 * empty cache.
 */
int p3m_sr_set_tune_cache(p3m_sr_handle h, const char *path);

/* What the last autotune call did: trials timed, and 1 if it installed a
 * cached layout instead of timing. */
int p3m_sr_tune_status(p3m_sr_handle h, int *trials_timed, int *from_cache);

/*
 * Read an autotuner cache file with the parser the handles use, without a
 * handle or a GPU: *entries = the entries a handle would load (lines that
 * do not parse, or hold an invalid layout, are skipped), *lines = the lines
 * read (either pointer may be NULL).  EINVAL for a NULL path or a file that
 * cannot be opened.
 */
int p3m_sr_tune_cache_check(const char *path, int *entries, int *lines);

/*
 * Fix the decomposition instead of autotuning (0 / -1 = automatic):
 *   subtiles_per_dim  subtiles per tile per dimension, 1..16 (section 2.1.3
 *                     "Subtiles");
 *   item_target       work-item target size in supplier candidates, 64..1<<20;
 *   cluster_size      receivers per cluster, 8, 16, 32 or 64.  Particles are
 *                     kept in tile -> subtile order (section 2.1.3) and, inside
 *                     each dense subtile, in the Morton order of an 8^3 grid of
 *                     sub-cells, so a cluster of consecutive receivers is
 *                     spatially compact; a wavefront carries 64 / cluster_size
 *                     copies of a cluster that walk different suppliers;
 *   screen            1: each supplier of the surviving subtiles is tested
 *                     against the cluster's bounding box before the pair
 *                     loop (the subtile-pair culling of section 2.1.3
 *                     carried down to single suppliers); 0: no screening;
 *                     2: screened, and for all-active P3M_FP32 forward calls
 *                     (polynomial shape, softened or not), all-active
 *                     P3M_FP64 forward calls (softened or not) and backward
 *                     calls without softening (n <= 2^27 for all) each pair
 *                     is evaluated once for
 *                     both partners (Newton's third law, as the paper's tile
 *                     pairing in section 2.1.3, "Tiles"; the adjoint's pair
 *                     term is antisymmetric too): clusters visit the upper
 *                     half of their tile stencil, the pair arithmetic is on
 *                     coordinates relative to the cluster's centre (FP32, or
 *                     FP64 for P3M_FP64 calls, where pairs within a relative
 *                     2^-40 of r_cut^2 or much closer than the receiver's
 *                     offset are redone in the plain form) and the
 *                     reactions are added to the partners' FP64 sums;
 *                     cluster_size must be 16, 32 or 64 (0 keeps the
 *                     automatic choice); other calls take screen 1 (or,
 *                     with an autotuned screen 2, the layout the autotuner
 *                     kept beside it); -1: automatic.
 * EINVAL outside those ranges.  Results do not depend on these settings
 * beyond FP64 summation order and, with screen 2, the rounding of the
 * separation (within the path's accuracy).
 */
int p3m_sr_set_config(p3m_sr_handle h, int subtiles_per_dim, int item_target,
                      int cluster_size, int screen);

/*
 * Kernel-shape knob for FP32 forward calls without softening (force and
 * batched; FP64, adjoint and softened calls always evaluate the polynomial):
 * g(u)/r^3 = r^-3 + H(u^2) / (2 x_s)^3, with r^-3 from a hardware rsqrt and
 * the smooth H either from the degree-9 polynomial (P3M_SHAPE_POLY, the
 * default) or looked up in a table over r^2 in [0, r_cut^2) as section 2.1.3
 * ("Other optimisations") does for its whole bracket: P3M_SHAPE_TAB_NGP takes
 * the value at the centre of the r^2 bin (the paper's choice, 2^12 entries by
 * default), P3M_SHAPE_TAB_LINEAR interpolates linearly between the bin's
 * ends (the paper's smaller-table alternative).  The table is filled from an
 * FP64 evaluation of H at each call and held in LDS by every pair-kernel
 * block.  table_size: a power of two in [64, 4096] (NGP) or [64, 2048]
 * (linear), 0 for the largest.  Accuracy: see the measured errors with each
 * choice; the NGP table's error grows like 1 / table_size, the linear one's
 * like 1 / table_size^2.  EINVAL for an unknown kind or table size.
 */
int p3m_sr_set_shape(p3m_sr_handle h, int kind, int table_size);

/*
 * Softening (section 2.1.1 and the softening bracket of eq. p3m_gravity):
 * every following force, backward and batched call on this handle adds
 * mu_j (|r|_B^-3 - |r|^-3) r_ij to the pair force for |r_ij| < eps_B, with
 * the B-spline |r|_B^-3 of eq. bspline_force and eps_B = 2.8 eps (eps is the
 * Plummer-equivalent softening length; the paper's choice of eps_B).  The
 * adjoint differentiates the softened force.  eps = 0 (the default) gives
 * point particles.  EINVAL for a negative or non-finite eps.
 */
int p3m_sr_set_softening(p3m_sr_handle h, double eps);

/*
 * Deterministic mode (enable = 1; 0, the default, turns it off): every
 * following force, backward and batched call on this handle returns the
 * same bits for the same inputs, call after call.  The sums are then taken
 * in a fixed order:
 *   - particles of a cell are ordered by (fine sub-cell, input index) with a
 *     stable radix sort, instead of the order that the atomic counting gives;
 *   - a cluster whose stencil is split into several work items gets each
 *     item's sums in a slot of its own, added in item order after the pair
 *     launch, instead of FP64 atomics;
 *   - layout screen 2 runs as screen 1, or as the layout the autotuner kept
 *     beside an autotuned screen 2 (the kernel that evaluates each pair for
 *     both partners adds its reactions with atomics).
 * The accepted pairs are the same in both modes and the forces differ only
 * by the rounding of the summation order.  The sort and the partial slots
 * cost time and workspace (24 B per particle, 24 B per item and receiver
 * slot).  Long-range (PM) and KDK calls are not covered.  EINVAL unless
 * enable is 0 or 1.
 */
int p3m_sr_set_deterministic(p3m_sr_handle h, int enable);

/*
 * Debug limits for testing out-of-memory handling.  max_workspace_bytes > 0
 * caps the device workspace this handle may hold (the short-range, PM and
 * KDK buffers grown with hipMalloc); a growth that would pass it fails with
 * P3M_ENOMEM before anything of the call is launched past that point, as a
 * failed hipMalloc does.  fail_after >= 0 lets that many more growths
 * succeed and makes the next one fail (-1: no such limit).  0 / -1 turn
 * the limits off.  After a P3M_ENOMEM the handle stays usable: lifting the
 * limit and calling again gives the normal result.  The no-alloc entry
 * point, whose workspace is fixed, ignores both.  EINVAL for
 * max_workspace_bytes < 0 or fail_after < -1.
 */
int p3m_sr_set_debug_limits(p3m_sr_handle h, int64_t max_workspace_bytes, int fail_after);

/*
 * Record HIP events on the call's stream around the build phase and the
 * pair-kernel launch of every following call (enable != 0), reported in
 * p3m_sr_stats.  Off by default.
 */
int p3m_sr_set_timing(p3m_sr_handle h, int enable);

/* Counters of the most recent call on this handle (synchronises its stream). */
int p3m_sr_get_stats(p3m_sr_handle h, p3m_sr_stats *out);

/*
 * Long-range (PM) acceleration: the upper half of eq. p3m_gravity (section
 * 2.1.3), i.e. the PM method of eq. pm_method with the Poisson kernel
 * replaced by the long-range kernel exp(-x_s^2 k^2) / k^2 of
 * eq. ewald_potential:
 *   rho_m   = sum_j mu_j W(x_m - x_j)            CIC (eq. W_CIC), nodes at
 *                                                 x_m = h (m + 1/2), h = box/n_grid
 *   phi     = F^-1 [ exp(-x_s^2 k^2) / k^2 * prod_d sinc(h k_d / 2)^-4 * F rho ],
 *             the k = 0 mode zeroed, F^-1 normalised (eq. weight_fourier:
 *             two CIC deconvolutions)
 *   a_i     = 4 pi / h^4 * sum_m W(x_i - x_m) D4 phi_m
 *             (eq. symmetric_diff_4 along each axis, per grid unit).
 * Every particle deposits; rows of non-receivers (active[i] == 0) are set
 * to 0.  a_i + the short-range acceleration of p3m_sr_force with the same
 * x_s is the P3M acceleration of eq. p3m_gravity (without softening).
 *   n_grid  grid points per dimension: a power of two, 16..1024 (the paper
 *           uses n_grid = 2 cbrt(N) with x_s = 1.25 box / n_grid).
 * All arithmetic is FP64.  The workspace holds 12 n_grid^3 + 16 (n_grid/2+1)
 * n_grid^2 + 56 n bytes (grids, node histogram, particles sorted by node).
 * The deposit adds with FP64 atomics (in LDS for nodes holding at most 8
 * particles, in HBM for denser ones), so results can differ between runs in
 * the last bits.  Errors: EINVAL for n < 0, box or x_s not positive and
 * finite, n_grid outside the supported set, NULL pos/acc_out with n > 0, or
 * pointers not 8-byte aligned; EUNSUPPORTED for n > 2^31 - 16; ENOMEM; EHIP.
 */
int p3m_lr_force(p3m_sr_handle h, const double *pos, const double *mass,
                 const uint8_t *active, int64_t n, double box, int n_grid, double x_s,
                 double *acc_out, void *stream);

/* Timings of the most recent p3m_lr_force call (synchronises its stream). */
int p3m_lr_get_stats(p3m_sr_handle h, p3m_lr_stats *out);

/*
 * The whole P3M acceleration of eq. p3m_gravity (section 2.1.3): the
 * short-range sum of p3m_sr_force plus the long-range PM term of
 * p3m_lr_force, with the same x_s, written to acc_out (n x 3 FP64).  The
 * two halves are independent until the final sum, so the long range runs on
 * an auxiliary stream of the handle (default priority, created on the first
 * call) that waits for the work queued on `stream` before the call, while
 * the short range runs on `stream`; `stream` then waits for the long range
 * and adds it.  On return every piece of the call is ordered before later
 * work on `stream`, as for the other entry points.  Arguments, layouts,
 * softening, shape and precision of the short range are those of
 * p3m_sr_force; n_grid, the long range's workspace and its FP64 arithmetic
 * those of p3m_lr_force; the workspace adds n x 3 doubles for the long-range
 * half.  Rows of non-receivers (active[i] == 0) are 0.  p3m_sr_get_stats
 * and p3m_lr_get_stats report the two halves.  Calls on one handle must not
 * overlap (the auxiliary stream and the workspace are per handle).
 * Errors: those of p3m_sr_force and p3m_lr_force; on an error of the short
 * range, `stream` still waits for the queued long range.
 */
int p3m_force(p3m_sr_handle h, const double *pos, const double *mass, const uint8_t *active,
              int64_t n, double box, double x_s, double r_cut, int n_grid, int precision,
              double *acc_out, void *stream);

/*
 * Rung-hierarchical kick-drift-kick step (section 2.2.2, "Individual time
 * steps", the time-stepping figure and eq. rung) in a static periodic box:
 * drift x += v tau, kick v += a t_kick, with a from p3m_sr_force (B-spline
 * softening eps) and, when n_grid > 0, from p3m_lr_force.
 *   pos, vel  n x 3 FP64, in/out: a synchronised state, advanced by
 *             n_steps steps of dt and synchronised again (the paper's period
 *             of steps between synchronisations).  Positions stay in [0, box).
 *   rung      n uint8, out: eq. rung from the final short-range
 *             accelerations, rung = max(0, ceil(log2(dt sqrt(|a| /
 *             (2 eta eps))))) capped at max_rung (the next period's rungs).
 *             With flags & P3M_KDK_FIXED_RUNGS it is an input instead and
 *             stays unchanged: every particle keeps its rung.
 * The period starts from eq. rung on the short-range accelerations at the
 * start (or the fixed rungs); L is the highest rung and positions drift in
 * dt / 2^L sub-steps.  Rung l kicks every dt / 2^l with the short-range
 * force, its particles as receivers and all particles as suppliers; a kick
 * brings the particle's momentum half a step of its rung ahead (the first
 * is the half kick from the start, the last ends at the period's end).
 * After each kick the rung follows eq. rung by at most one step, downwards
 * only where the lower rung kicks next (the next kick after a jump is then
 * half or three quarters of the usual one).  The long-range force kicks
 * every particle whenever rung 0 kicks.
 *   n_grid    0 (short range only) or the PM grid of p3m_lr_force.
 *   eta, eps  eq. rung's accuracy parameter (the paper: 0.025) and the
 *             Plummer-equivalent softening length (also the softening of the
 *             short-range force; eps > 0 unless rungs are fixed).
 *   max_rung  0..7 (the paper's default maximum of 8 rungs).
 * Synchronises with the host once per sub-step.  Errors: those of
 * p3m_sr_force, plus EINVAL for dt <= 0, n_steps outside [1, 64], max_rung
 * outside [0, 7], unknown flags, eps < 0, eps or eta not positive without
 * fixed rungs, fixed rungs above max_rung, NULL vel or rung.
 */
int p3m_kdk_step(p3m_sr_handle h, double *pos, double *vel, const double *mass, uint8_t *rung,
                 int64_t n, double box, double x_s, double r_cut, int n_grid, double dt,
                 int n_steps, double eta, double eps, int max_rung, int flags, int precision,
                 void *stream);

/* Counters of the most recent p3m_kdk_step call. */
int p3m_kdk_get_stats(p3m_sr_handle h, p3m_kdk_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* P3MSR_H */
