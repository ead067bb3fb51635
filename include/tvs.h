/*
 * tvs.h -- C ABI of the MI355X (gfx950) hot path of total-variation-
 * superiorized (TVS) proton-CT reconstruction, after Schultze, Censor,
 * Karbasi, Schubert and Schulte, "An Improved Method of Total Variation
 * Superiorization Applied to Reconstruction in Proton Computed Tomography"
 * (arXiv 1803.01112).
 *
 * The problem (Section I): every proton history gives one linear equation
 * whose left side is the sum, over the voxels its most likely path (MLP)
 * crosses, of the chord length in the voxel times the voxel's unknown
 * relative stopping power (RSP), and whose right side is its measured
 * water-equivalent path length (WEPL).  Each cycle k of NTVS (Appendix C)
 * applies N perturbation steps x += beta * v, v = -grad TV / ||grad TV||,
 * beta = alpha^ell, optionally checking that TV does not increase, and then
 * one feasibility-seeking sweep P_T: block-iterative DROP with relaxation
 * lambda over blocks of B histories (Section III-D).
 *
 * Conventions shared by every entry point:
 *   - Every call returns a status (TVS_OK or a negative TVS_E* code); no
 *     exception or signal crosses the ABI.  tvs_last_error(ctx) gives a
 *     human-readable reason for the last failure on that context.
 *   - Pointers marked "host or device" are read as device pointers when the
 *     accompanying on_device flag is 1 (e.g. torch.Tensor.data_ptr() of a
 *     CUDA tensor), else as host pointers.  Input arrays are borrowed for the
 *     duration of the call only: the library copies what it keeps.
 *   - `stream` is a hipStream_t (NULL: the context's own stream).  Work is
 *     enqueued on it; a call that returns data in host memory waits for it.
 *     Calls on one context that name different streams are ordered by the
 *     caller (as for any two streams), except that the library orders its
 *     own second stream, on which rows are formed on the fly, after the
 *     load's work and before every later use of the rows.
 *   - Lengths are in mm; images are float32 RSP, nx*ny*nz values, x fastest
 *     (index ix + nx*(iy + ny*iz)).
 *   - One context must not be used by two threads at once; distinct
 *     contexts are independent (each owns all of its device memory).
 */
#ifndef TVS_H
#define TVS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tvs_ctx tvs_ctx;

enum tvs_status {
    TVS_OK = 0,
    TVS_EINVAL = -1,   /* invalid argument (NaN/inf input, bad grid or parameter) */
    TVS_ENOMEM = -2,   /* footprint exceeds the HBM budget or free device memory */
    TVS_EDEVICE = -3,  /* HIP runtime error */
    TVS_ESTATE = -4,   /* call out of order (e.g. iterate before load) */
    TVS_ERANGE = -5    /* an index or size outside what the context holds */
};

/* Voxel grid: nx*ny*nz voxels of vx*vy*vz mm; (ox,oy,oz) is the corner of
 * voxel (0,0,0) (Section III-D uses 200x200 voxels of 1.0x1.0x2.5 mm per
 * 20 slices). */
typedef struct {
    int32_t nx, ny, nz;
    double vx, vy, vz;
    double ox, oy, oz;
} tvs_grid;

/* How the rows of the system are formed during a sweep. */
enum tvs_path_mode {
    TVS_PATH_ON_THE_FLY = 0, /* MLP walked for every history on every sweep */
    TVS_PATH_STORE_F32 = 1,  /* rows formed once: 32-bit entry tag + float32 chord */
    TVS_PATH_STORE_F16 = 2,  /* rows formed once: 32-bit entry tag + float16 chord */
    TVS_PATH_STORE_Q16 = 3   /* rows formed once, 6 bytes per entry like float16: a 32-bit
                                entry tag + a 16-bit word; the chord is a fixed-point code
                                (a multiple of the longest chord of the loaded rows / the
                                largest code) of 16 + 24 - ceil(log2 B) bits (at most 30):
                                its low 16 bits in the word, the rest in the tag bits that
                                the row index of a block of B histories leaves free (28 bits
                                at B = 3200: 1e-8 mm steps for 1 x 1 x 2.5 mm voxels);
                                B <= 2^20 */
};

typedef struct {
    int32_t block_size;      /* B, histories per DROP block (Section III-D: 3200); >= 1 */
    int32_t path_mode;       /* enum tvs_path_mode */
    double mlp_step_mm;      /* depth spacing of MLP vertices; <= 0: min(vx, vy) */
    int32_t mlp_log_term;    /* 1: Highland logarithmic correction in the MLP moments */
    int32_t mlp_const_power; /* 1: constant scattering power (test mode) */
    int64_t chunk_histories; /* on-the-fly: histories whose rows are formed together; 0: auto */
    uint64_t hbm_budget_bytes; /* 0: 80 % of the device memory free at tvs_create */
    int32_t device;          /* HIP device ordinal */
    int32_t max_tries;       /* bound on the retries of one checked TV step; 0: 100000 */
    int32_t sweep_kernel;    /* 0 or 1: one launch per DROP block (finish the previous block
                                and form this block's dot products, tile by tile);
                                2: the same work in two launches per block */
    int32_t tile_threads;    /* threads per image-tile workgroup of the DROP kernels
                                (64, 128, 256); 0: 128 on the fly and for grids of
                                more than 16 image tiles per CU, else 256 */
    int32_t time_sample;     /* k > 0: kernel-stamped HIP events on the launches of every
                                k-th DROP block (per-launch durations in tvs_stats); 0: off */
    int32_t fill_wgs_per_cu; /* on-the-fly rows: cap on the workgroups per compute unit of
                                the row formation that runs beside the DROP chain; 0 or < 0:
                                no cap */
    int32_t fill_wide_pct;   /* on-the-fly rows: percentage of the chunks formed at the row
                                kernel's full occupancy (three waves per SIMD, which leaves a
                                SIMD no room for DROP waves); the others are held at two
                                waves per SIMD, with room for four DROP waves beside them;
                                spread evenly over the sweep; < 0: the library's choice (0) */
} tvs_config;

/* Fills *cfg with the defaults above (B = 3200, on-the-fly rows, log term on). */
void tvs_config_default(tvs_config *cfg);

/* Proton histories as structure-of-arrays float32 streams of equal length
 * (Section I: entry/exit positions and directions, and WEPL):
 *   ex,ey,ez / qx,qy,qz : entry / exit position on the object hull, mm;
 *   eth,eps / qth,qps   : entry / exit slopes dt/du and dv/du, where u is
 *                         the beam (depth) axis, t = (-uy, ux, 0) the
 *                         in-plane lateral axis and v = z;
 *   ux,uy               : beam axis in the x-y plane (normalised internally);
 *   wepl                : measured WEPL, mm. */
typedef struct {
    const float *ex, *ey, *ez, *qx, *qy, *qz;
    const float *eth, *eps, *qth, *qps;
    const float *ux, *uy;
    const float *wepl;
} tvs_histories;

enum tvs_variant {
    TVS_NTVS = 0,      /* Appendix C: ell_k = rand(k, ell_{k-1}); N steps of beta = alpha^ell */
    TVS_OTVS = 1,      /* Appendix B: one checked step per cycle, beta = (1/2)^ell */
    TVS_DECOUPLED = 2  /* Section VI proposal: beta_{k,n} = alpha^n gamma^k, n = 1..N */
};

/* Reconstruction parameters (Section III-E). */
typedef struct {
    double lambda;     /* DROP relaxation, > 0 */
    int32_t N;         /* TV perturbation steps per cycle, >= 0 */
    double alpha;      /* perturbation kernel, 0 < alpha < 1 */
    int32_t tv_check;  /* NTVS: 1 = keep the TV-reduction check, 0 = exclude it */
    int32_t variant;   /* enum tvs_variant */
    double tv_eps;     /* TV smoothing: m = sqrt(dx^2 + dy^2 + eps^2), phi = sum (m - eps); >= 0 */
    uint64_t seed;     /* seed of the SplitMix64 stream that draws ell_k */
    double gamma;      /* TVS_DECOUPLED only, 0 < gamma < 1 */
} tvs_params;

typedef struct {
    int64_t k;           /* cycles completed since the image was set */
    int64_t ell;         /* current exponent ell */
    int64_t n_hist;      /* histories loaded */
    int64_t n_skipped;   /* histories forming no row (exit not beyond entry, or empty row) */
    int64_t nnz;         /* row entries over all histories (0 until rows were formed) */
    int64_t steps;       /* perturbation steps taken (records in the step log) */
    int64_t tries;       /* TV-check tries in total */
    int64_t max_row_nnz; /* longest row */
    /* Device times from HIP events recorded on the launch stream during the
     * last tvs_iterate call (reading them waits for that work). */
    double last_sweep_ms;  /* last cycle's sweep P_T */
    double last_tv_ms;     /* last cycle's perturbation steps */
    double last_rows_ms;   /* row formation inside the last sweep (on-the-fly rows) */
    uint64_t device_bytes; /* device memory held by the context */
    double tv_ms_total;    /* all perturbation steps of the call */
    double sweep_ms_total; /* all sweeps of the call */
    double rows_ms_total;  /* all row-formation launches of the call */
    double drop_ms_total;  /* all DROP launches of the call */
    int64_t cycles_timed;  /* cycles of the call */
    int64_t rows_launches; /* row-formation launches of the call */
    int64_t drop_launches; /* DROP chains timed (one per sweep) */
    double k1_ms_total;    /* sampled blocks: the block's launch (with sweep_kernel 2 its
                              first launch, the finish of the previous block) */
    double k2_ms_total;    /* sampled blocks, sweep_kernel 2 only: the second launch */
    int64_t k_samples;     /* sampled blocks of the last tvs_iterate call */
    double batch_ms_total; /* cycles of the last tvs_iterate_batch call */
    int64_t batch_cycles;  /* cycles of that call */
    int32_t batch_size;    /* S of the current batch (0: none) */
    int32_t pad;
} tvs_stats;

/* One record per perturbation step (Appendix C; checked steps record TV). */
typedef struct {
    int32_t k, n;
    int32_t tries;       /* tries until accepted (1 for unchecked steps) */
    int32_t accepted;    /* 0: the step gave up after max_tries, image unchanged */
    int64_t ell_start;   /* ell at the first try */
    double phi_x;        /* TV before the step (checked steps) */
    double phi_z;        /* TV of the accepted image (checked steps) */
    double gnorm;        /* ||grad TV|| */
} tvs_step_log;

/* Creates a context on cfg->device for the given grid.  Validates the grid
 * (positive sizes and spacings, finite origin, nx*ny*nz < 2^31) and the
 * configuration.  *out receives the context (NULL on failure). */
int tvs_create(const tvs_grid *grid, const tvs_config *cfg, tvs_ctx **out);

/* Frees every device buffer of ctx; NULL is accepted. */
void tvs_destroy(tvs_ctx *ctx);

/* Loads n proton histories (host or device arrays, see tvs_histories),
 * replacing any loaded before.  Rejects NaN/inf values and zero beam axes
 * with TVS_EINVAL, a footprint beyond the HBM budget with TVS_ENOMEM; on
 * failure nothing stays loaded.  A history whose exit is not deeper than
 * its entry along the beam axis, or whose path misses the grid, forms no
 * row: it is counted in n_skipped, not rejected.  With a path store the
 * rows (MLP + voxel walk, Section I) are formed here, once.  Resets the
 * image to zero and the cycle state to k = 0, ell = 0. */
int tvs_load_histories(tvs_ctx *ctx, int64_t n, const tvs_histories *h, int on_device,
                       void *stream);

/* Sets the initial iterate x-bar (Appendix A) from nx*ny*nz floats (host or
 * device) and resets the cycle state (k = 0, ell = 0, RNG unseeded). */
int tvs_set_image(tvs_ctx *ctx, const float *x0, int on_device, void *stream);

/* Runs K more cycles (Appendix C / B, or the Section VI schedule) from the
 * current state.  The first cycle after tvs_set_image / tvs_load_histories
 * seeds the RNG from p->seed; later calls continue the same stream, so K
 * cycles in one call equal the same K cycles split over several calls.
 * The work is queued on the stream and the call returns without waiting,
 * with or without the TV-reduction check: a checked step is decided on the
 * device (its tries, ell and the RNG state stay there), and its records
 * reach the step log when tvs_get_step_log or tvs_get_stats is called, an
 * unchecked call follows, or more than 4096 records are pending (then the
 * call waits once for the work queued so far).
 * TVS_EINVAL for lambda <= 0, alpha outside (0,1), N < 0, tv_eps < 0;
 * TVS_ESTATE before tvs_load_histories. */
int tvs_iterate(tvs_ctx *ctx, const tvs_params *p, int32_t K, void *stream);

/* Copies the current image (nx*ny*nz floats) to out (host or device).  The
 * DROP sums are exact 64-bit integers in units of 2^-36 (row dot products)
 * and 2^-40 (corrections); a product |a_ij x_j| beyond 2^26 / (longest row)
 * cannot be summed so and is reported here, by tvs_get_stats and by
 * tvs_get_batch_image as TVS_ERANGE (until the next tvs_set_image). */
int tvs_get_image(tvs_ctx *ctx, float *out, int on_device, void *stream);

/* Batched reconstructions: S settings of the loaded histories (a parameter
 * study over lambda, N, alpha as in Section III-E), each with its own
 * tvs_params and all starting from the image set by tvs_set_image, advanced
 * K cycles together.  Every cycle reads each row once and applies it to all
 * S images; the launches of one cycle are captured in a hipGraph and
 * replayed for every cycle (on-the-fly rows are formed in that graph on a
 * second stream, beside the TV steps and the DROP chain).  Unchecked schedules only (TVS_NTVS with
 * tv_check = 0, or TVS_DECOUPLED); 1 <= S <= 32; p points to S parameter
 * sets.  A call with the same S and parameters as the previous one
 * continues those reconstructions; otherwise they restart from the initial
 * image.  The main image (tvs_iterate / tvs_get_image) is not touched.
 * Waits for the work before returning.  TVS_EINVAL for an invalid setting,
 * TVS_ESTATE before tvs_load_histories, TVS_ENOMEM when the S images do not
 * fit the budget. */
int tvs_iterate_batch(tvs_ctx *ctx, const tvs_params *p, int32_t S, int32_t K, void *stream);

/* Copies image s (0 <= s < S) of the current batch to out (host or device);
 * TVS_ERANGE for s outside the batch, TVS_ESTATE without a batch. */
int tvs_get_batch_image(tvs_ctx *ctx, int32_t s, float *out, int on_device, void *stream);

/* Initial iterate by filtered backprojection (FBP) of the loaded histories,
 * then an in-slice median filter.  The paper starts each reconstruction from
 * a median-filtered initial iterate, radius 2 (arXiv 1803.01112, Section
 * V-A, citing earlier work for how it is formed); the form here is the
 * textbook parallel-beam one: every history's straight line from entry to
 * exit is binned where it crosses the rotation axis (depth u = 0) by beam
 * angle (A bins over 360 degrees), lateral position (bins of width t_bin_mm
 * centred on the axis, enough to cover the grid) and slice; a bin holds the
 * mean WEPL of its histories; rows are filtered with the discrete Ram-Lak
 * kernel and backprojected with linear interpolation.  The result becomes
 * the context image, as by tvs_set_image (schedule and batch reset), and is
 * also copied to out (nx * ny * nz float32, x fastest, host or device) when
 * out is not NULL.  Waits for the work.  TVS_EINVAL for n_angles < 1,
 * t_bin_mm < 0 or median_radius outside 0..2; TVS_ESTATE before
 * tvs_load_histories; TVS_ENOMEM when the bins do not fit the budget. */
typedef struct {
    int32_t n_angles;       /* A, beam angles evenly spaced over 360 degrees */
    int32_t median_radius;  /* 0 (none) .. 2; the paper's initial iterate uses 2 */
    double t_bin_mm;        /* lateral bin width; 0: the grid's vx */
    int32_t clip_negative;  /* 1: negative values set to 0 before the median */
    int32_t pad;
} tvs_fbp_params;

int tvs_initial_fbp(tvs_ctx *ctx, const tvs_fbp_params *p, float *out, int on_device, void *stream);

/* tvs_initial_fbp for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same initial iterate, with every intermediate (bin sums
 * and counts, mean and filtered projections, angle table, backprojected
 * image) in one fixed workspace of 64 MiB that the library holds on every
 * device it runs on, from the first tvs_create there until the process
 * ends.  It calls no hipMalloc, hipFree or other allocating routine.  The
 * workspace needs 28 B per bin (n_angles x nz x lateral bins) + 16 B per
 * angle + 8 B per voxel, each part rounded up to 256 B; a larger problem
 * is refused with TVS_ERANGE before any device work (200x200x20 voxels of
 * 1x1x2.5 mm at 180 angles and 1 mm bins need 35 MB).  Every call on one device
 * shares that device's workspace and overwrites it, clearing what must
 * start at zero itself: calls that overlap on one device (two streams, two
 * threads) race and must be serialised by the caller.  Waits for the work
 * only when out is host memory; otherwise the work is queued on the stream.
 * Other arguments, the result and the errors are those of tvs_initial_fbp. */
int tvs_initial_fbp_noalloc(tvs_ctx *ctx, const tvs_fbp_params *p, float *out, int on_device,
                            void *stream);

/* Hull detection of the object from the loaded histories, before the MLP is
 * relied on (the paper's preprocessing, Section III-D, bounds the object and
 * cites earlier work for how).  The textbook straight-line detectors on each
 * history's line from its entry to its exit point, voxels taken by the same
 * midpoint walk as the rows:
 *   space modelling: a line whose WEPL is at least wepl_in_mm counts every
 *     voxel it crosses (protons that lost energy crossed the object);
 *   space carving: a line whose WEPL is below wepl_out_mm carves every voxel
 *     it crosses (a proton that lost no energy crossed no object);
 *   a voxel is inside when at least min_in lines count it and at most
 *   max_out lines carve it.
 * hull receives nx*ny*nz bytes (x fastest, 1 inside, 0 outside; host or
 * device, may be NULL).  With mask_image set, the context image is set to
 * itself times the hull (as by tvs_set_image: schedule and batch reset), so
 * that an initial iterate from tvs_initial_fbp or tvs_set_image is bounded
 * by the hull.  Waits for the work.  TVS_EINVAL for min_in < 0, max_out < 0
 * or a NaN threshold; TVS_ESTATE before tvs_load_histories; TVS_ENOMEM when
 * the two counters (4 bytes per voxel each) do not fit the budget. */
typedef struct {
    double wepl_in_mm;      /* space modelling threshold */
    double wepl_out_mm;     /* space carving threshold (0: no carving) */
    int32_t min_in;         /* counting lines needed inside (0: space modelling off) */
    int32_t max_out;        /* carving lines tolerated inside */
    int32_t mask_image;     /* 1: the context image is multiplied by the hull */
    int32_t pad;
} tvs_hull_params;

int tvs_hull_detect(tvs_ctx *ctx, const tvs_hull_params *p, uint8_t *hull, int on_device,
                    void *stream);

/* Counters and timings of the context. */
int tvs_get_stats(tvs_ctx *ctx, tvs_stats *out);

/* Copies up to cap step records (oldest first) to out; *n receives the number
 * of records held.  The log is cleared by tvs_set_image / tvs_load_histories. */
int tvs_get_step_log(tvs_ctx *ctx, tvs_step_log *out, int64_t cap, int64_t *n);

/* Exports the rows of histories [first, first+count) for inspection: row
 * lengths (row_nnz[count]), voxel indices and chords concatenated in history
 * order (at most cap entries), and ||a||^2 (norm2[count]); all host arrays.
 * Rows are formed by the same kernels the sweep uses.  TVS_ERANGE when
 * [first, first+count) is outside the loaded histories or cap is too small
 * (row_nnz is still filled then). */
int tvs_debug_rows(tvs_ctx *ctx, int64_t first, int64_t count, int64_t *row_nnz, int32_t *idx,
                   float *chord, float *norm2, int64_t cap);

/* ------------------------------------------------------------------------
 * Serving: a continuous-batching server of reconstruction requests.
 * Requests queue in arrival order and are admitted first-in first-out when
 * a slot is free and their device-memory footprint fits under the server's
 * HBM budget together with the running requests.  Each admitted request
 * runs on its own context and stream (one worker thread per slot), so
 * requests overlap on the device; a request that arrives while others run
 * starts as soon as a slot and memory free up.  A failing request fails
 * alone.  With `simulate` set no device work is done: a request sleeps
 * sim_ns_per_history_cycle * n * K nanoseconds (for testing the policy).
 * ------------------------------------------------------------------------ */
typedef struct tvs_server tvs_server;

typedef struct {
    int32_t device;
    int32_t max_active;         /* requests running at once, 1..16 (default 3) */
    uint64_t hbm_budget_bytes;  /* bound on the sum of admitted footprints; 0: 80 % of free */
    int64_t chunk_histories;    /* on-the-fly row chunk of each request (default 262144) */
    int32_t simulate;           /* 1: no device work (policy testing); needs a budget */
    int32_t pad;
    double sim_ns_per_history_cycle;
} tvs_server_config;

/* One reconstruction request.  The history arrays are host memory borrowed
 * until the request completes (tvs_server_wait returned or the server was
 * destroyed); x0 (nx*ny*nz floats, or NULL for zeros) is copied at submit. */
typedef struct {
    tvs_grid grid;
    int32_t block_size;         /* <= 0: 3200 */
    int32_t path_mode;          /* enum tvs_path_mode */
    tvs_params params;
    int32_t K;                  /* cycles */
    int32_t pad;
    int64_t n;
    tvs_histories h;
    const float *x0;
} tvs_request;

typedef struct {
    int32_t state;              /* 0 queued, 1 running, 2 done, 3 failed */
    int32_t status;             /* TVS_* status of a finished request */
    double submit_ms, admit_ms, done_ms;  /* steady-clock ms since the server started */
    uint64_t bytes;             /* footprint reserved while running */
    int64_t admit_order;        /* 1-based admission rank */
} tvs_request_info;

typedef struct {
    uint64_t budget_bytes, in_use_bytes, peak_bytes;
    int32_t active, peak_active, queued, pad;
    int64_t completed, failed;
} tvs_server_counters;

/* Fills *cfg with defaults (device 0, 3 slots, budget 80 % of free memory). */
void tvs_server_config_default(tvs_server_config *cfg);
/* Starts the worker threads.  TVS_EINVAL for max_active outside 1..16 or a
 * simulated server without a budget; TVS_EDEVICE if the device is unusable. */
int tvs_server_create(const tvs_server_config *cfg, tvs_server **out);
/* Device bytes reserved for a request (history streams, row lengths, row
 * buffers of one chunk or the whole store, image buffers).  The row entries
 * of a store are estimated from the histories' straight entry-exit lines,
 * the most likely path taken within 10 mm plus half the line's length times
 * the entry and exit slopes of them (a host pass over the arrays); the
 * estimate also bounds the request's own context, so a request whose rows
 * exceed it fails alone with TVS_ENOMEM. */
uint64_t tvs_server_footprint(const tvs_server *sv, const tvs_request *r);
/* Queues a request; *id receives its handle.  TVS_EINVAL for a bad grid or
 * sizes, TVS_ENOMEM when its footprint alone exceeds the budget. */
int tvs_server_submit(tvs_server *sv, const tvs_request *r, int64_t *id);
/* State of a request without waiting. */
int tvs_server_query(tvs_server *sv, int64_t id, tvs_request_info *info);
/* Waits for the request; copies its image (image_len >= nx*ny*nz floats, or
 * image = NULL) and info.  Returns the request's status. */
int tvs_server_wait(tvs_server *sv, int64_t id, float *image, int64_t image_len,
                    tvs_request_info *info);
int tvs_server_get_counters(tvs_server *sv, tvs_server_counters *out);
/* Lets running requests finish, fails queued ones (TVS_ESTATE), joins the
 * workers and frees the server. */
void tvs_server_destroy(tvs_server *sv);

/* ------------------------------------------------------------------------
 * Autotuning of the launch shape.  Times every candidate shape (threads per
 * image-tile workgroup 64 / 128 / 256, one or two launches per DROP block)
 * on the first 1,024 blocks of the loaded histories, from the current image,
 * which is restored afterwards, and keeps the fastest for the context.  On
 * the fly a second stage then times whole sweeps (row formation beside the
 * chain) for the share of chunks formed at the row kernel's full occupancy
 * (tvs_config.fill_wide_pct: 0, 20, 40, 60, 80, 100) and keeps the fastest.
 * The block size B is a parameter of the method and is never changed (a
 * larger B is always faster per sweep, and changes the reconstruction).
 * With cache_path (a text file, created if missing) a shape measured before
 * for the same device, grid, history count, B and path mode is reused
 * without timing, and new measurements are appended.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t tile_threads;    /* chosen shape */
    int32_t sweep_kernel;    /* 1: one launch per block, 2: two */
    double ms_per_block;     /* its measured time per DROP block */
    int32_t from_cache;      /* 1: taken from the cache file */
    int32_t n_candidates;
    int32_t cand_threads[8];
    int32_t cand_sweep[8];
    double cand_ms[8];       /* per block, per candidate */
    int32_t fill_wide_pct;   /* on the fly: chosen share of full-occupancy chunks, % */
    int32_t n_fill;          /* on the fly: shares timed (0 otherwise) */
    int32_t cand_pct[8];
    double cand_sweep_ms[8]; /* per sweep, per share */
} tvs_tune_result;

/* TVS_ESTATE before tvs_load_histories; TVS_EINVAL for lambda <= 0. */
int tvs_autotune(tvs_ctx *ctx, double lambda, const char *cache_path, tvs_tune_result *out,
                 void *stream);

/* Autotuning of the batched sweep's step (tvs_iterate_batch) for S settings
 * p[0..S-1]: threads per workgroup (128, 256) x settings applied per pass
 * through LDS (2, 4, 8, 16; untuned: 256 x 4), each timed on the first DROP blocks (on the fly,
 * of the first chunk, formed for the purpose) with S images started from
 * the initial image; keeps the fastest for the context and appends it to
 * cache_path (reused for the same device, grid, history count, B, path mode
 * and S).  The next tvs_iterate_batch starts its settings afresh from the
 * initial image.  Errors as tvs_iterate_batch (settings validated the same
 * way) and tvs_autotune. */
typedef struct {
    int32_t threads;         /* chosen threads per workgroup */
    int32_t group;           /* chosen settings per LDS pass */
    double ms_per_block;     /* its measured time per DROP block */
    int32_t from_cache;
    int32_t n_candidates;
    int32_t cand_threads[8];
    int32_t cand_group[8];
    double cand_ms[8];       /* per block, per candidate */
} tvs_batch_tune_result;

int tvs_autotune_batch(tvs_ctx *ctx, const tvs_params *p, int32_t S, const char *cache_path,
                       tvs_batch_tune_result *out, void *stream);

/* Static description of a status code. */
const char *tvs_strerror(int status);

/* Message of the last failure on ctx ("" if none); valid until the next call. */
const char *tvs_last_error(tvs_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TVS_H */
