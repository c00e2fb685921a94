/*
 * rms.h -- C ABI of an MI355X (gfx950) Monte Carlo diffusion walker in 3d
 * voxelized label volumes, after Lee, Fieremans & Novikov, "Realistic
 * Microstructure Simulator (RMS)", arXiv 2012.06478.
 *
 * Units throughout: micrometres (um), milliseconds (ms), um^2/ms for
 * diffusivities, um/ms for permeabilities, ms/um^2 for b values.
 *
 * Conventions for every entry point:
 *   - returns RMS_OK (0) or a negative RMS_E_* code; rms_last_error() then
 *     describes the failure (per calling thread);
 *   - pointers are host pointers unless stated otherwise; the library copies
 *     what it needs and never keeps or frees caller memory;
 *   - no exception crosses the ABI;
 *   - results are deterministic given the substrate, parameters, seed,
 *     walker count, step count, protocol and precision: they do not depend on
 *     the stream, on concurrent calls or on the server's mix of requests.
 */
#ifndef RMS_H
#define RMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RMS_ABI_VERSION 3

/* Error codes. */
#define RMS_OK 0
#define RMS_E_INVALID_ARG (-1)         /* malformed argument (message says which) */
#define RMS_E_LABEL_RANGE (-2)         /* a voxel label >= n_labels */
#define RMS_E_STEP_TOO_LARGE (-3)      /* max step length >= voxel size (section 2.1.1) */
#define RMS_E_PROB_TOO_LARGE (-4)      /* a permeation probability > RMS_MAX_PERM_PROB */
#define RMS_E_UNBALANCED_WAVEFORM (-5) /* |sum_i G_i| > 1e-9 sum_i |G_i| for a shape */
#define RMS_E_OOM (-6)                 /* device or host allocation failed */
#define RMS_E_DEVICE (-7)              /* a HIP runtime call failed (no result) */
#define RMS_E_BUSY (-8)                /* server: request cannot be admitted now */
#define RMS_E_TIMEOUT (-9)             /* server: wait timed out */
#define RMS_E_WAIT_GAVE_UP (-10)       /* a wave of the persistent walk gave up its
                                          bounded wait for the previous segment of
                                          its walkers; every wave then stopped and
                                          the run has no result (the substrate and
                                          later runs are unaffected) */

/* Permeation rules (rms_params.perm_model). */
#define RMS_PERM_KAPPA 0  /* Eq. (perm-prob-general); with concentrations Eq. (gen-perm-prob) */
#define RMS_PERM_BAXTER 1 /* Eq. (alt-perm-prob1-2) on the membranes with kappa > 0 */

/* Precision forms of rms_run. */
#define RMS_FP64 0  /* double-precision walk and reductions */
#define RMS_MIXED 1 /* int32 voxel + fp32 offset walk, fp64 reductions */

/* Walk kernels (rms_result.walk_kernel, RMS_OPT_WALK_KERNEL). */
#define RMS_WALK_AUTO (-1)       /* option value: the library chooses (default) */
#define RMS_WALK_ONE_LAUNCH 0    /* one thread per walker, every step in one launch */
#define RMS_WALK_PERSISTENT 1    /* resident waves take (64 walkers, segment of steps)
                                    items from per-XCD queues */
#define RMS_WALK_PACKED 2        /* launches over step ranges with the walker states in
                                    device memory (rms_run_record, the server) */

/* Size limits. */
#define RMS_MAX_SHAPES 4     /* gradient waveform shapes per run */
#define RMS_MAX_SIGNALS 960  /* n_shapes * n_b * n_dirs per run */
#define RMS_MAX_LABELS 4096  /* compartment labels per substrate */
/* Largest permeation probability per membrane hit a run accepts (Table 1:
 * P << 1; rms_result.max_perm_prob reports the largest one a run uses). */
#define RMS_MAX_PERM_PROB 0.1

/* Per-walker dump record (doubles), in this order:
 *   0-2  displacement x, y, z (um, unwrapped)
 *   3    R = sum_c t_c / T2_c (so alpha = exp(-R))
 *   4    label at the end
 *   5-7  voxel index x, y, z at the end
 *   8-10 offset inside that voxel at the end (voxel lengths, in [0, 1])
 *   11   label at the start
 *   12   face events (face reached: pass, permeation or reflection)
 *   13   membrane hits (faces between different labels)
 *   14   permeations
 *   15.. phase vector Phi_s = dt sum_i G_s[i] (x_i - x_0) (3 per shape, um ms)
 */
#define RMS_DUMP_FIXED 15
#define RMS_DUMP_WIDTH(n_shapes) (RMS_DUMP_FIXED + 3 * (n_shapes))

/* Opaque, immutable, device-resident substrate: the label volume (section
 * 2.1.1: the voxelized geometry is its own lookup table of compartment
 * labels) plus default tissue parameters.  Safe to share between concurrent
 * runs and the server once created. */
typedef struct rms_substrate rms_substrate;

/* Tissue parameters of one run (overrides the substrate defaults).
 *   D      [n_labels] intrinsic diffusivity D0 per label (um^2/ms), > 0 for
 *          every label that is not dead (section 2.1.3, Eq. step-size);
 *   kappa  [n_labels * n_labels] permeability per label pair (um/ms),
 *          row-major, symmetric, >= 0; the diagonal is ignored; NULL means
 *          every membrane is impermeable (section 2.1.3, Eq.
 *          perm-prob-general);
 *   T2     [n_labels] transverse relaxation time per label (ms), > 0,
 *          INFINITY for none; NULL means no relaxation (section 2.1.4, Eq.
 *          wt-relax);
 *   rho    [n_labels * n_labels] surface relaxivity (um/ms), >= 0, row-major:
 *          rho[a * n_labels + b] makes the faces from label a to label b
 *          absorbing for walkers in a (magnetization transfer, end of section
 *          2.1.3): such a walker is saturated with probability
 *          P_MT = rho ds_a C_3 / D_a (at most RMS_MAX_PERM_PROB, else
 *          RMS_E_PROB_TOO_LARGE), decided at the membrane before and
 *          independently of the permeation decision, and keeps walking with
 *          weight 0 (Eq. wt-mt; its R becomes INFINITY in walker_dump).  NULL
 *          or all zero: no membrane absorbs.  If every walker is saturated,
 *          sum_alpha is 0 and the normalized results are NaN;
 *   conc   [n_labels] spin concentration per label, > 0 for every label that is
 *          not dead, or NULL: all equal (App. C, general case).  Walkers start
 *          with density proportional to conc (a uniform draw accepted with
 *          probability c / max c; the mean acceptance over the allowed voxels
 *          must be at least 1e-3), and with RMS_PERM_KAPPA a membrane between
 *          labels a < b permeates by Eq. (gen-perm-prob) with side 1 = a and
 *          the input kappa corrected by Eq. (gen-kappa-correction);
 *   lambda exponent of Eq. (gen-perm-prob) in [0, 1], or < 0 for the closed
 *          form 1 / (1 + c_b sqrt(D_b) / (c_a sqrt(D_a))) printed as the
 *          minimising choice; ignored without conc;
 *   perm_model  RMS_PERM_KAPPA (kappa's value sets the permeability) or
 *          RMS_PERM_BAXTER (the membranes with kappa > 0 permeate by Eq.
 *          (alt-perm-prob1-2): probability c_lo sqrt(D_lo) / (c_hi sqrt(D_hi))
 *          from the side of larger c sqrt(D), 1 from the other; the limit
 *          RMS_MAX_PERM_PROB does not apply).
 * A zero-initialised rms_params apart from n_labels and D gives the plain
 * model. */
typedef struct {
    int n_labels;
    const double* D;
    const double* kappa;
    const double* T2;
    const double* rho;
    const double* conc;
    double lambda;
    int perm_model;
} rms_params;

/* Results of one run.  The caller allocates every array it wants filled and
 * sets the pointer (NULL = not wanted); the library fills them.
 *   signal      [n_shapes][n_b][n_dirs][2] (re, im) of
 *               S = <alpha exp(-i phi)> / <alpha> (section 2.3, Eq. signal)
 *   m2          alpha-weighted <dx_i dx_j> / <alpha>, order xx xy xz yy yz zz
 *   m4          alpha-weighted <dx_i dx_j dx_k dx_l> / <alpha>, i<=j<=k<=l in
 *               lexicographic order (xxxx xxxy xxxz xxyy xxyz xxzz xyyy xyyz
 *               xyzz xzzz yyyy yyyz yyzz yzzz zzzz)
 *   D_dir       [n_dirs] (g.M2.g) / (2 t), t = n_steps dt (section 2.3)
 *   K_dir       [n_dirs] (M4:g^4) / (g.M2.g)^2 - 3 (section 2.3, with both
 *               moments divided by <alpha>)
 *   b_disc      [n_shapes] b value of each shape at unit scale; each shape is
 *               scaled by sqrt(b / b_disc) so that its discrete b equals b
 *   walker_dump [n_walkers][RMS_DUMP_WIDTH(n_shapes)] per-walker records */
typedef struct {
    double* signal;
    double m2[6];
    double m4[15];
    double* D_dir;
    double* K_dir;
    double sum_alpha;
    double* b_disc;
    int64_t n_face_events;
    int64_t n_membrane_hits;
    int64_t n_permeations;
    double max_perm_prob;       /* largest permeation probability in the run */
    double max_step_over_voxel; /* largest ds / voxel size in the run */
    double wall_s;              /* rms_run: host wall time of the call; server: latency
                                   from rms_server_submit to completion */
    double kernel_ms;           /* rms_run: walk kernel time, HIP events on the run's
                                   stream; server: 0 (launches are shared) */
    double queue_s;             /* server: submit to admission; rms_run: 0 */
    double* walker_dump;
    int walk_kernel;            /* RMS_WALK_ONE_LAUNCH or RMS_WALK_PERSISTENT (rms_run),
                                   RMS_WALK_PACKED (rms_run_record, the server): the walk
                                   kernel that ran */
} rms_result;

/* ABI version (RMS_ABI_VERSION of the built library). */
int rms_abi_version(void);

/* Description of the last failure on the calling thread ("" if none). */
const char* rms_last_error(void);

/* Process-wide options of the walk launch and the server, for measurements
 * and tests of the launch paths (every run or server afterwards uses them; not
 * thread-safe against runs in flight).  No option changes a result: a
 * walker's trajectory depends only on (seed, walker, step).
 *   RMS_OPT_WALK_KERNEL     RMS_WALK_AUTO (default: the persistent walk when
 *                           the walkers fill between 1.5 and 4.5 rounds of
 *                           resident waves, else one launch),
 *                           RMS_WALK_ONE_LAUNCH or RMS_WALK_PERSISTENT (taken
 *                           by runs of at most 4.5 rounds of six resident waves
 *                           per SIMD, which hold its state buffer; others run
 *                           one launch);
 *   RMS_OPT_SEG_POLL_LIMIT  polls (each a sleep of about a microsecond) a wave
 *                           of the persistent walk makes for the previous
 *                           segment of its walkers before it gives up and the
 *                           run fails with RMS_E_WAIT_GAVE_UP; >= 0, default
 *                           2^20 (about a second);
 *   RMS_OPT_SERVER_WALKERS  walker slots of the servers created afterwards:
 *                           the admitted requests of a server hold at most
 *                           this many walkers together (a larger request is
 *                           admitted alone); >= 0, default 0 = sixteen
 *                           rounds of the device's resident waves of the
 *                           mixed walker (compute units x 4 SIMDs x 6 waves
 *                           x 64 x 16, 6.3e6 on MI355X).
 * RMS_E_INVALID_ARG for an unknown option or value. */
#define RMS_OPT_WALK_KERNEL 1
#define RMS_OPT_SEG_POLL_LIMIT 2
#define RMS_OPT_SERVER_WALKERS 3
int rms_set_option(int option, int64_t value);

/* Build a device-resident substrate (sections 2.1.1 and 2.2 item 1).
 *   labels      host array of nx*ny*nz labels, x fastest then y then z,
 *               uint8 (label_bytes = 1) or uint16 (label_bytes = 2); copied;
 *   dims        {nx, ny, nz}, each >= 1, (nx+2)(ny+2)(nz+2) < 2^31; the
 *               volume is periodic in all three axes;
 *   voxel_um    isotropic voxel size l_p (um), > 0;
 *   n_labels    number of labels, 1..RMS_MAX_LABELS; every voxel < n_labels;
 *   D, kappa, T2  default tissue parameters (see rms_params);
 *   dead        [n_labels] or NULL: nonzero marks a label no walker starts in
 *               or enters (section 2.2, item 1);
 *   out         receives the handle.
 * The substrate lives on the HIP device current at the call, as the volume
 * inside a one-voxel periodic halo: (nx+2)(ny+2)(nz+2) entries of 1 byte
 * (uint8 labels with n_labels <= 32) or 2 bytes (otherwise).  Volumes of
 * more than 2^22 voxels are checked and padded on up to 16 host threads
 * (joined before the call returns).  A label >= n_labels gives
 * RMS_E_LABEL_RANGE naming the first such voxel; RMS_E_OOM if host staging
 * or device memory runs out. */
int rms_create_substrate(const void* labels, int label_bytes, const int64_t dims[3],
                         double voxel_um, int n_labels, const double* D, const double* kappa,
                         const double* T2, const uint8_t* dead, rms_substrate** out);

/* Free a substrate (NULL is a no-op).  No run may be using it. */
void rms_destroy_substrate(rms_substrate* sub);

/* Simulate n_walkers independent walkers for n_steps steps of dt_ms each
 * (section 2.2, items 1-5) and reduce their signals and moments (section
 * 2.3).
 *   sub          substrate; params overrides its tissue parameters (NULL =
 *                substrate defaults; n_labels must match);
 *   seed         64-bit key of the counter-based random streams: walker w's
 *                trajectory depends only on (seed, w, substrate, params, dt);
 *   n_walkers    in [1, 2^32 - 2]; n_steps in [0, 2^32 - 2]; dt_ms > 0;
 *   n_shapes     0..RMS_MAX_SHAPES gradient shapes; waveform is
 *                [n_shapes][n_steps], sample i applies during step i+1, each
 *                shape balanced (sum of samples ~ 0);
 *   dirs         [n_dirs][3] gradient directions (normalized here);
 *   bvals        [n_b] b values >= 0 (b > 0 needs a nonzero shape);
 *   precision    RMS_FP64 or RMS_MIXED;
 *   hip_stream   hipStream_t to run on (NULL = the null stream);
 *   out          results (see rms_result).
 * Blocks until the results are in host memory.  A run's device memory comes
 * from a stream-ordered pool the library creates on each device at its first
 * run there and keeps until the process ends; the pool holds up to 4 GiB of
 * freed memory for the next run instead of returning it to the driver at
 * each synchronization (the device's default pool is not touched). */
int rms_run(const rms_substrate* sub, const rms_params* params, uint64_t seed, int64_t n_walkers,
            int64_t n_steps, double dt_ms, int n_shapes, const double* waveform, int n_dirs,
            const double* dirs, int n_b, const double* bvals, int precision, void* hip_stream,
            rms_result* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rms_run
 * with every device buffer of the run in a scratch array of the library,
 * RMS_NOALLOC_MAX_BYTES on each GPU it runs on, held until the process ends.
 * Arguments, results and errors are those of rms_run, and so are the
 * kernels: the results equal rms_run's bit for bit.  It calls no device
 * allocation routine (the array's address and two timing events are set up
 * at the first call on a device).  A run whose buffers need more than
 * RMS_NOALLOC_MAX_BYTES (the double-precision form with one gradient shape
 * and 180 signals fits about 900 000 walkers; the dump buffer of a run is
 * per-walker records, 8 (15 + 3 n_shapes) bytes a walker) is refused with
 * RMS_E_INVALID_ARG before any device work.  Every call on one GPU uses the
 * same array: calls that overlap in time on one GPU (from several threads, or
 * on several streams) race and give wrong results; calls one after another
 * are safe, as each run clears whatever it needs cleared. */
#define RMS_NOALLOC_MAX_BYTES (256ull * 1024ull * 1024ull)
int rms_run_noalloc(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                    int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                    const double* waveform, int n_dirs, const double* dirs, int n_b,
                    const double* bvals, int precision, void* hip_stream, rms_result* out);

/* Displacement moments recorded during a walk: the time dependence of D and
 * K (section 2.3 defines both from the moments of the displacement over the
 * diffusion time t).  After step steps[r] (t = steps[r] dt) each walker is
 * weighted by alpha(t) = exp(-R(t)), R(t) its T2 integral up to that step
 * (section 2.1.4, Eq. wt-relax), and
 *   sum_alpha  [n_rec]           sum over walkers of alpha(t)
 *   m2         [n_rec][6]        alpha(t)-weighted <dx_i dx_j> / sum_alpha
 *   m4         [n_rec][15]       alpha(t)-weighted <dx_i dx_j dx_k dx_l> / sum_alpha
 *   D_dir      [n_rec][n_dirs]   (g.M2.g) / (2 t), or NULL
 *   K_dir      [n_rec][n_dirs]   (M4:g^4) / (g.M2.g)^2 - 3, or NULL
 * with the component orders of rms_result.  n_rec is 1..RMS_MAX_RECORDS and
 * steps ascend strictly within 1..n_steps.  The caller allocates every array;
 * sum_alpha, m2 and m4 are required. */
#define RMS_MAX_RECORDS 4096
typedef struct {
    int n_rec;
    const int64_t* steps;
    double* sum_alpha;
    double* m2;
    double* m4;
    double* D_dir;
    double* K_dir;
} rms_record;

/* rms_run with the displacement moments recorded at rec->steps.  Every other
 * argument and every field of `out` is as for rms_run, and the end results
 * equal rms_run's bit for bit (a walker's trajectory depends only on seed,
 * walker and step).  The walk runs interval by interval between record
 * steps, keeping the walker states in device memory (120 extra bytes per
 * walker in FP64, 100 in the mixed form, with one waveform shape) and a
 * second buffer of walker records (8 (15 + 3 n_shapes) bytes per walker); half
 * of the walkers walk on hip_stream and half on a non-blocking stream the call
 * creates, waits for and destroys before it returns.  out->kernel_ms covers
 * the walk launches and the record reductions between them.  Errors as
 * rms_run, and RMS_E_INVALID_ARG for a malformed record list. */
int rms_run_record(const rms_substrate* sub, const rms_params* params, uint64_t seed,
                   int64_t n_walkers, int64_t n_steps, double dt_ms, int n_shapes,
                   const double* waveform, int n_dirs, const double* dirs, int n_b,
                   const double* bvals, int precision, void* hip_stream, const rms_record* rec,
                   rms_result* out);

/* ---------------------------------------------------------------------------
 * Post-processing of a run's signals (host only; no device work).
 * ------------------------------------------------------------------------- */

/* Direction average of the signal for each b value (the spherical mean; the
 * directions are taken as a uniform sampling of the sphere or, with the
 * antipodal symmetry of the signal, of a hemisphere).
 *   signal  [n_b][n_dirs][2] (re, im): one shape of rms_result.signal;
 *   out     [n_b][2] caller-allocated.
 * RMS_E_INVALID_ARG for n_b < 1, n_dirs < 1 or a NULL pointer. */
int rms_spherical_mean(int n_b, int n_dirs, const double* signal, double* out);

/* Cumulant fit of the signal per direction (section 2.3: D and K from the
 * signal's b dependence, here for any pulse width): least squares of
 * ln Re S(b) = -b D + b^2 D^2 K / 6 over the b values in (0, b_max] (ln S(0) =
 * 0 is held exactly).
 *   bvals  [n_b] ms/um^2; signal [n_b][n_dirs][2] as above;
 *   D_out, K_out  [n_dirs] caller-allocated (um^2/ms; dimensionless).
 * RMS_E_INVALID_ARG if fewer than two b values lie in (0, b_max], or a
 * signal there is not positive. */
int rms_cumulant_fit(int n_b, const double* bvals, int n_dirs, const double* signal,
                     double b_max, double* D_out, double* K_out);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of simulation requests on one GPU.
 *
 * A server keeps the substrates its requests name resident (the caller keeps
 * them alive until every request on them has completed), admits requests in
 * arrival order while their device memory fits in the budget, and advances
 * every admitted request by a slice of steps in one packed launch per slice
 * (requests of different sizes share a launch, grouped by precision, label
 * width and shape count).  The next slice is queued on the device before the
 * server waits for the current one, so the device does not idle between
 * slices.  A request that arrives while others run joins at the next slice
 * built; a finished request's results are reduced and copied in the slice
 * that finishes it, and its memory is freed for the next admission.  Walker trajectories depend only
 * on (seed, walker, step) and each request is reduced on its own in a fixed
 * order, so a request's results are bit-identical alone, in any mix and to
 * rms_run with the same arguments.
 * ------------------------------------------------------------------------- */
typedef struct rms_server rms_server;
typedef int64_t rms_ticket;

/* One request: the arguments of rms_run.  Every array is copied at submit. */
typedef struct {
    const rms_substrate* substrate;
    const rms_params* params; /* NULL = substrate defaults */
    uint64_t seed;
    int64_t n_walkers;
    int64_t n_steps;
    double dt_ms;
    int n_shapes;
    const double* waveform; /* [n_shapes][n_steps] */
    int n_dirs;
    const double* dirs;     /* [n_dirs][3] */
    int n_b;
    const double* bvals;    /* [n_b] */
    int precision;          /* RMS_FP64 or RMS_MIXED */
} rms_request;

typedef struct {
    int64_t submitted, completed, failed, pending, active;
    int64_t launches;       /* packed walk launches so far */
    int64_t walker_steps;   /* walker-steps of completed requests */
    double busy_s;          /* device time of the packed launches (HIP events) */
    size_t bytes_in_use, bytes_budget;
} rms_server_stats;

/* Create a server on the HIP device current at the call.
 *   mem_budget_bytes  device memory the server may hold for admitted requests
 *                     (0 = 3/4 of the device's free memory);
 *   slice_steps       steps per slice (>= 2, rounded up to a multiple of 4), or 0
 *                     to size each slice to about 4e9 walker-steps of the
 *                     admitted requests. */
int rms_server_create(size_t mem_budget_bytes, int slice_steps, rms_server** out);

/* Queue a request; returns at once with its ticket.  Argument errors are
 * reported here (as by rms_run); a request that cannot fit in the budget even
 * alone returns RMS_E_BUSY. */
int rms_server_submit(rms_server* srv, const rms_request* req, rms_ticket* ticket);

/* *done = 1 once the request has completed or failed. */
int rms_server_poll(rms_server* srv, rms_ticket ticket, int* done);

/* Wait up to timeout_s seconds (< 0: forever) for a request, fill `out` as
 * rms_run would (walker_dump is not available and must be NULL) and release
 * the ticket.  RMS_E_TIMEOUT leaves the ticket valid; a failed request
 * returns its error code and is released. */
int rms_server_wait(rms_server* srv, rms_ticket ticket, double timeout_s, rms_result* out);

int rms_server_stats_get(rms_server* srv, rms_server_stats* out);

/* Stop the server: requests not yet complete fail, resources are freed. */
void rms_server_destroy(rms_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* RMS_H */
