/*
 * zmc.h -- C ABI of the MI355X (gfx950) direct Monte Carlo parameter-scan
 * library, libzmc.so.
 *
 * The operation (ZMCintegral-v5, arXiv:1910.01965, Sec. 2, Eq. (1)): for every
 * point x of an M-dimensional parameter grid, each parameter x_l running over
 * its own list of values, estimate f(x) = integral of g(y; x) dy over an
 * N-dimensional box by direct (crude) Monte Carlo (Sec. 1 and Sec. 2: no
 * stratification, no adaptive tree search), and return the whole grid of
 * results (Sec. 2, last paragraph; Sec. 3.3).  Each point's estimate is
 *     f     = V * (1/n) sum_s g(y_s; x)
 *     sigma = V * sqrt( sum_s (g_s - mean)^2 / (n (n-1)) )
 * with V the box volume.  The paper names no random generator and reports no
 * error bar; this library fixes both:
 *   - sample s, coordinate k of grid point g uses word w = s*N + k of the
 *     Philox4x32-10 stream (Salmon et al., SC'11) with key = seed and counter
 *     (b mod 2^32, b / 2^32, g mod 2^32, g / 2^32), b = w / 4, lane w mod 4;
 *   - FP64 path: u = (r + 1/2) 2^-32, y_k = fma(hi_k - lo_k, u, lo_k);
 *     FP32 path: u = ((r >> 9) + 1/2) 2^-23 from the top 23 bits.
 * Results therefore do not depend on how the library splits the work.
 *
 * Grid flattening is C order: flat index g = ((i_1 L_2 + i_2) L_3 + ...) L_M
 * + i_M (the last parameter varies fastest); outputs are indexed by g.
 *
 * Conventions for every entry point:
 *   - the return value is a zmc_status; nothing is thrown or aborted across
 *     the ABI; zmc_last_error() gives a message for the calling thread;
 *   - pointers named d_* are device (HBM) pointers on the current HIP device;
 *     other pointers are host memory; all are owned by the caller and read or
 *     written only during the call (for asynchronous calls: until the work on
 *     the given stream has completed);
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - the host side of the scan, batch, range and server entry points is
 *     marked with ROCTx ranges named after them, for rocprofv3 --marker-trace.
 */
#ifndef ZMC_H
#define ZMC_H

#include <stddef.h>
#include <stdint.h>

/* Environment: ZMC_LOG = 1 reports set-up events on stderr (tune-table
 * loads, batch and server creation, run-time compiles), 2 also every plan,
 * every server admission and completion, and every split-partial buffer the
 * device scan's cache allocates or retires; unset or 0, the library prints
 * nothing.  ZMC_TUNE_TABLE names the tile-shape table (see the batch API);
 * ZMC_COPY_THREADS the host threads of chunked scans (zmc_scan_chunked). */

#ifdef __cplusplus
extern "C" {
#endif

typedef enum zmc_status {
  ZMC_OK = 0,
  ZMC_E_INVALID = 1,     /* malformed descriptor or argument              */
  ZMC_E_NOMEM = 2,       /* device or host allocation failed, or a buffer
                            the call would size exceeds 2^56 bytes         */
  ZMC_E_DEVICE = 3,      /* a HIP call failed (no device, launch error)   */
  ZMC_E_UNSUPPORTED = 4, /* valid request the library does not implement  */
  ZMC_E_BUSY = 5,        /* resource limit reached; retry later           */
  ZMC_E_CANCELLED = 6    /* a served request cancelled before admission   */
} zmc_status;

/* Integrand families, compiled in as templates.  SIN_SUM is the paper's test
 * integrand (Eq. (2) on [0,10]^N, Eq. (4) on [0,1]^6). */
typedef enum zmc_family {
  ZMC_SIN_SUM = 0, /* sin(sum_{l=1..M} x_l + sum_{k=1..N} y_k), any M          */
  ZMC_GAUSS = 1,   /* exp(-(sum_{k<=M} x_k y_k^2 + sum_{k>M} y_k^2)), M <= N   */
  ZMC_COSEXP = 2,  /* cos(x1 y1 + x2 y2 + sum_{k>=3} y_k) exp(-x3^2 y1 y2) + x4,
                      M = 4, N >= 2                                             */
  ZMC_CONST = 3,   /* 1 (sampler and estimator check)                          */
  ZMC_LINEAR = 4,  /* sum_k y_k (sampler and estimator check)                  */
  ZMC_USER = 5     /* a user function compiled at run time (zmc_integrand_create),
                      given by desc->integrand; any M, n_params <= 16          */
} zmc_family;

typedef struct zmc_integrand zmc_integrand;

typedef enum zmc_precision {
  ZMC_FP64 = 0,         /* FP64 sampling, integrand and accumulation         */
  ZMC_FP32_MERGE64 = 1  /* FP32 integrand and per-lane Kahan-compensated sums,
                           FP64 merging across lanes, waves, blocks, splits  */
} zmc_precision;

/* One scan.  Limits: 0 <= M <= 16; 1 <= N <= 16; every axis_len >= 1;
 * G = prod axis_len <= 2^62; lo_k < hi_k, both finite; samples >= 2 and
 * samples * N <= 2^62; n_params = 0 for the five compiled-in families,
 * 0 <= n_params <= 16 for ZMC_USER. */
typedef struct zmc_scan_desc {
  int32_t M;                /* number of parameters                          */
  int32_t N;                /* integration dimensions                        */
  const int64_t* axis_len;  /* [M] list lengths L_l                          */
  const double* axis_vals;  /* [sum L_l] host copy of the lists, back to back
                               (finite values; f and sigma are unspecified
                               for points with a non-finite one); read by
                               the device entry points only when their
                               d_axis_vals is NULL                          */
  const double* lo;         /* [N] lower box edges                           */
  const double* hi;         /* [N] upper box edges                           */
  int32_t family;           /* zmc_family                                    */
  int32_t precision;        /* zmc_precision                                 */
  const double* params;     /* [n_params] constants passed to a ZMC_USER
                               integrand as p[0..n_params-1] (p[i] = 0 beyond) */
  int32_t n_params;
  uint64_t samples;         /* n, samples per grid point                     */
  uint64_t seed;            /* Philox key                                    */
  const zmc_integrand* integrand;  /* ZMC_USER only (else ignored)           */
} zmc_scan_desc;

/* Work decomposition.  Zero fields mean "choose automatically".  The results
 * do not depend on these beyond floating-point summation order. */
typedef enum zmc_mode {
  ZMC_MODE_AUTO = 0,
  ZMC_MODE_POINT_MAJOR = 1,  /* each lane owns one point, a wave 64 points;
                                sample range optionally cut into splits       */
  ZMC_MODE_SAMPLE_MAJOR = 2  /* a block owns one point; its lanes share the
                                samples; wave then LDS reduction; optionally
                                several blocks per point (splits)             */
} zmc_mode;

typedef struct zmc_launch_opts {
  int32_t mode;          /* zmc_mode                                          */
  int32_t block;         /* threads per block: 64..1024 (point-major, and any
                            scan with N > 8: ..256),
                            multiple of 64                                    */
  int32_t splits;        /* sample-range pieces per point (>= 1)              */
  int32_t cu_count;      /* planner only: compute units assumed (0 = device)  */
  void* ev_begin;        /* optional hipEvent_t recorded on the stream just
                            before the main scan kernel (for timing)          */
  void* ev_end;          /* optional hipEvent_t recorded just after it, before
                            the split-merge pass                              */
} zmc_launch_opts;

typedef struct zmc_plan_info {
  int32_t mode;              /* chosen zmc_mode                               */
  int32_t block;             /* threads per block                             */
  int32_t splits;            /* sample-range pieces per point                 */
  int32_t reserved;
  uint64_t grid_points;      /* G                                             */
  uint64_t groups;           /* ceil(samples / 4): groups of four samples     */
  uint64_t groups_per_split; /* groups in each piece (the last may be short)  */
  uint64_t blocks;           /* blocks of the main kernel                     */
  uint64_t workspace_bytes;  /* device bytes of split partials (0 if none)    */
} zmc_plan_info;

/* Message describing the last failure on the calling thread ("" if none). */
const char* zmc_last_error(void);

/* Library version string. */
const char* zmc_version(void);

/* Host-only validation of a descriptor (no device use).  Returns ZMC_OK,
 * ZMC_E_INVALID or ZMC_E_UNSUPPORTED; *grid_points (if not NULL) gets G. */
zmc_status zmc_validate(const zmc_scan_desc* desc, uint64_t* grid_points);

/* Host-only work decomposition that zmc_scan_device_ex would use with these
 * options (opts may be NULL).  Without opts->cu_count, queries the current
 * device's compute-unit count (ZMC_E_DEVICE if there is none).  Explicit
 * splits whose partials (16 B per point and piece) would exceed 2^56 bytes
 * give ZMC_E_NOMEM; automatic plans keep them under 8 GiB. */
zmc_status zmc_plan(const zmc_scan_desc* desc, const zmc_launch_opts* opts,
                    zmc_plan_info* out);

/* Synchronous scan with host memory: stages desc->axis_vals to the device,
 * computes, copies f and sigma (G doubles each, C order) back into the
 * caller's host arrays.  On error the outputs are unspecified.  Grids whose
 * f and sigma would exceed 2^56 bytes of staging give ZMC_E_NOMEM (use
 * zmc_scan_chunked). */
zmc_status zmc_scan(const zmc_scan_desc* desc, double* f, double* sigma);

/* Asynchronous scan on `stream` with device-resident data: d_axis_vals holds
 * the concatenated value lists (sum L_l doubles); d_f and d_sigma receive G
 * doubles each.  desc->axis_vals is read only when d_axis_vals is NULL (and
 * M > 0): the call then stages the lists itself into a device copy that it
 * frees on the stream, and has read desc->axis_vals when it returns; under
 * stream capture that gives ZMC_E_INVALID (a replay cannot re-read host
 * memory), and with both pointers NULL too.
 * Split partials, when the plan needs them (16 B per point and sample
 * piece), come from a per-device cache of at most four buffers of
 * power-of-two sizes from 1 MiB to 256 MB, held by the library until the
 * process ends and reused
 * without a host wait (a buffer still in use by another call's kernels is
 * ordered after them on the device); larger partials, and every call made
 * under stream capture, live in stream-ordered device memory released on
 * the same stream.  Returns after enqueueing.
 * The call may be recorded by stream capture into a caller's HIP graph
 * (kernels plus, for split plans, graph memory nodes; no memset nodes); each
 * replay recomputes the same results, provided the device has been used
 * once (the compute-unit count is cached) before the capture begins. */
zmc_status zmc_scan_device(const zmc_scan_desc* desc, const double* d_axis_vals,
                           double* d_f, double* d_sigma, void* stream);

/* Out-of-core scan into host memory, for grids whose f and sigma do not
 * fit on the device (the paper's scale claim, Sec. 1 and Sec. 3.3): the grid
 * runs as consecutive chunks of chunk_points points (0 = 2^24), each with
 * the decomposition of the whole grid, so the results equal those of one
 * scan of the whole grid bit for bit.  While the device computes chunk i,
 * chunk i-1 is copied back over PCIe and, when f and sigma are pageable,
 * from pinned staging into them on host threads ($ZMC_COPY_THREADS, 1..64,
 * default 8); outputs in pinned memory
 * (hipHostMalloc) take the copies directly.  Device memory: the lists plus
 * 2 x 16 B x chunk_points plus the chunk's split partials.  Synchronous.
 * f and sigma must be host memory (ZMC_E_INVALID for device pointers). */
zmc_status zmc_scan_chunked(const zmc_scan_desc* desc, double* f, double* sigma,
                            uint64_t chunk_points);

/* Points [g_begin, g_end) of the grid (flat C-order indices), computed as
 * zmc_scan_chunked computes the whole grid, into host arrays of
 * g_end - g_begin doubles (f[i] is point g_begin + i).  The values equal
 * that slice of a scan of the whole grid bit for bit, so ranges can run in
 * separate processes or on separate devices and be concatenated, and an
 * interrupted scan resumes from its first unfinished range.  ZMC_E_INVALID
 * for an empty range or one outside the grid. */
zmc_status zmc_scan_range(const zmc_scan_desc* desc, uint64_t g_begin, uint64_t g_end,
                          double* f, double* sigma, uint64_t chunk_points);

/* zmc_scan_device with an explicit decomposition (opts may be NULL). */
zmc_status zmc_scan_device_ex(const zmc_scan_desc* desc, const double* d_axis_vals,
                              double* d_f, double* d_sigma,
                              const zmc_launch_opts* opts, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture that must record no memory nodes, tight serving loops, harnesses
 * that forbid hipMalloc): zmc_scan_device with the same arguments, the same
 * plan and the same kernels, so its f and sigma equal zmc_scan_device's bit
 * for bit, but it calls no hipMalloc, hipFree or allocating routine.  The
 * split partials of its plan (16 B per point and sample piece) live in a
 * fixed device array of ZMC_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends; the first call on a device
 * looks up that device's copy (make one call before capturing).  Plans
 * whose partials exceed the array (e.g. 1e6 points x 9 pieces = 144 MB) give
 * ZMC_E_NOMEM and launch nothing; ZMC_USER scans give ZMC_E_UNSUPPORTED
 * (their kernels are built and loaded on first use).  Every call on a device
 * shares its array and leaves its contents behind (nothing in it needs to
 * start at zero): calls that overlap on one device race, so the caller
 * orders them (one stream, or events).  Asynchronous on `stream`. */
#define ZMC_NOALLOC_SCRATCH_BYTES ((uint64_t)128 << 20)
zmc_status zmc_scan_device_noalloc(const zmc_scan_desc* desc, const double* d_axis_vals,
                                   double* d_f, double* d_sigma, void* stream);

/* Debug: words w0 .. w0+count-1 of grid point g's Philox stream, computed by
 * the device generator, into d_out (count uint32).  Asynchronous. */
zmc_status zmc_debug_words(uint64_t seed, uint64_t g, uint64_t w0, int64_t count,
                           uint32_t* d_out, void* stream);

/* Diagnostics: a calibration load for the VALU counters (not part of the
 * method).  `blocks` blocks of 256 threads each run `iters` iterations of
 * eight steps of eight independent FP32 multiply-add chains (64 x iters FMAs
 * per lane) and
 * write one float per thread to d_out (blocks x 256 floats, device memory).
 * A launch that fills the device should read as ~100 % issue-busy in the
 * counters used for the scan kernels.  Asynchronous on `stream`. */
zmc_status zmc_debug_valu_probe(int32_t blocks, int64_t iters, float* d_out, void* stream);

/* Diagnostics: instruction-rate loads (not part of the method), one per
 * instruction form that the scan kernels issue.  `blocks` blocks of 256
 * threads each run `iters` loop trips of 64 instructions of the form (eight
 * dependent chains per lane, each step reading three of them) and write one
 * 64-bit word per thread to d_out (blocks x 256 words, device memory).
 * Timing a launch gives the form's issue rate in lane-instructions per
 * second.  Asynchronous on `stream`; ZMC_E_INVALID for an unknown op. */
typedef enum zmc_rate_op {
  ZMC_RATE_XOR_B32 = 0,      /* v_xor_b32: two-operand integer               */
  ZMC_RATE_ADD_F32 = 1,      /* v_add_f32: two-operand FP32                  */
  ZMC_RATE_FMA_F32 = 2,      /* v_fma_f32: three-operand FP32                */
  ZMC_RATE_MAD_U64_U32 = 3,  /* v_mad_u64_u32: Philox's 32x32->64 product    */
  ZMC_RATE_BITOP3_B32 = 4,   /* v_bitop3_b32: Philox's three-way xor         */
  ZMC_RATE_EXP_F32 = 5,      /* v_exp_f32: the FP32 exp2 unit                */
  ZMC_RATE_SIN_F32 = 6,      /* v_sin_f32: the FP32 sine unit                */
  ZMC_RATE_FMA_F64 = 7       /* v_fma_f64                                     */
} zmc_rate_op;
zmc_status zmc_debug_rate_probe(int32_t op, int32_t blocks, int64_t iters, uint64_t* d_out,
                                void* stream);

/* Debug: integrand values g(y_s; x_g) for samples s = s0 .. s0+count-1 of
 * grid point g, computed by the device sampler and integrand in the
 * descriptor's precision and widened to FP64, into d_out (count doubles). */
zmc_status zmc_debug_values(const zmc_scan_desc* desc, const double* d_axis_vals,
                            uint64_t g, uint64_t s0, int64_t count, double* d_out,
                            void* stream);

/* ------------------------------------------------------------------------
 * User integrands (the paper's user-defined integrand of a parameter scan,
 * Sec. 2 and Sec. 4, compiled with hipRTC instead of Numba).  `source` is
 * HIP C++ that defines, at global scope,
 *
 *   template <typename T> __device__ T integrand(const T* y, const T* x,
 *                                                const T* p);
 *
 * returning g(y; x) for the sample's coordinates y[0..N-1] in the box, the
 * grid point's parameters x[0..M-1] and the scan's constants p[0..15]
 * (desc->params, zero-filled), in the working precision T (double for
 * ZMC_FP64, float for ZMC_FP32_MERGE64); device math functions (sin, exp,
 * ...) are available.  The same sampler, accumulators and merges as the
 * compiled-in families run around it.
 *
 * zmc_integrand_create copies the source and compiles one small variant to
 * report errors (ZMC_E_INVALID with the compiler's log in zmc_last_error);
 * every (precision, N, M) variant a scan needs is then compiled on first use
 * (a few seconds) and kept, and loaded once per device.  It needs no GPU.
 * The handle may be shared by threads.  zmc_integrand_destroy waits for
 * each device it was loaded on to go idle before unloading its kernels.
 * ZMC_USER scans run through every entry point: single scans, chunked
 * scans, batches (one persistent kernel per (handle, precision, N, M), built
 * at batch creation) and the server (built when a request is admitted).  The
 * handle must outlive every batch and request that uses it. */
zmc_status zmc_integrand_create(const char* source, zmc_integrand** out);

/* zmc_integrand_create with option flags (0 = zmc_integrand_create).
 * ZMC_INTEGRAND_FAST_MATH: the handle's FP32 variants are compiled with
 * approximate transcendentals (clang's -fgpu-approx-transcendentals and
 * -fapprox-func): expf, exp2f, logf, log2f, sinf, cosf and the like map to
 * the hardware's approximate instructions (v_exp_f32, v_log_f32, v_sin_f32,
 * v_cos_f32 with a scaling), and FP32 division and square root may use
 * approximations of about an ulp.  Relative error per call is then a few
 * FP32 ulps, except that sinf and cosf lose accuracy linearly in |x|
 * (about 1e-4 absolute at |x| = 1000: no exact argument reduction).  For
 * callers whose FP32 integrands call such functions with moderate
 * arguments and who want the compiled-in families' speed.  FP64 variants
 * are compiled exactly as without the flag, so their results do not change.
 * Unknown flag bits give ZMC_E_INVALID. */
#define ZMC_INTEGRAND_FAST_MATH 1u
zmc_status zmc_integrand_create_ex(const char* source, uint32_t flags, zmc_integrand** out);

/* Compiler log of the handle's last build (empty when it produced none). */
const char* zmc_integrand_log(const zmc_integrand* integrand);

zmc_status zmc_integrand_destroy(zmc_integrand* integrand);

/* ------------------------------------------------------------------------
 * Batched scans.  Many independent scans of uneven grid sizes, sample
 * counts, families and dimensions run as one unit of work: the planner cuts
 * every scan into tiles (256 grid points x one sample piece, or one point x
 * one sample piece for grids below the tuned threshold), with tile shapes
 * from the autotuned table (tune_table.txt next to the library, or
 * $ZMC_TUNE_TABLE); one persistent kernel per (family, precision, N)
 * variant drains its longest-first tile queue; a second pass merges split
 * partials in split order.  The whole sequence is captured once in a
 * hipGraph and replayed by zmc_batch_launch.  A scan's tiles depend only on
 * the scan itself, so its results are bitwise the same alone and in any
 * batch.  This generalises the paper's batches (Sec. 2, Fig. 1), where a
 * grid is cut into pieces that each go to one GPU.
 * ---------------------------------------------------------------------- */
typedef struct zmc_batch zmc_batch;

typedef struct zmc_batch_opts {
  int32_t use_graph;          /* 1: capture and replay a hipGraph; 0: launch the
                                 kernels directly on each zmc_batch_launch      */
  int32_t parallel_variants;  /* 1: one graph branch per kernel variant (they may
                                 overlap on the device); 0: one chain           */
  int64_t pm_groups;          /* > 0: groups of four samples per lane in a
                                 point-major tile (overrides the table)        */
  int64_t sm_groups;          /* > 0: groups per sample-major tile (override)   */
  int64_t pm_min_points;      /* > 0: smallest grid given point-major tiles     */
  int32_t cu_count;           /* planner only: compute units (0 = device)       */
  int32_t one_kernel;         /* 1: a single persistent kernel per precision runs
                                 every family and N (one tile queue; register
                                 use of the largest variant); 0: one kernel per
                                 (family, precision, N) variant               */
} zmc_batch_opts;

typedef struct zmc_batch_info {
  int32_t scans;              /* scans in the batch                            */
  int32_t variants;           /* distinct (family, precision, N) kernels       */
  int64_t tiles;              /* tiles over all scans                          */
  uint64_t samples;           /* sum over scans of G * samples                 */
  uint64_t points;            /* sum over scans of G                           */
  uint64_t workspace_bytes;   /* device bytes of tables, staged lists, partials */
  int32_t merge_scans;        /* scans with more than one sample piece         */
  int32_t graph;              /* 1 when a hipGraph is replayed                 */
} zmc_batch_info;

/* Default options: use_graph = 1, parallel_variants = 1, table-driven tiles.
 * Passing opts = NULL to the calls below means these defaults. */
void zmc_batch_default_opts(zmc_batch_opts* opts);

/* Host-only plan of a batch (validation, tiles, workspace), no device use
 * when opts->cu_count > 0. */
zmc_status zmc_batch_plan(const zmc_scan_desc* scans, int32_t n_scans,
                          const zmc_batch_opts* opts, zmc_batch_info* info);

/* Plans the batch, allocates its device tables and workspace, uploads them,
 * and (use_graph) captures the graph, all on the current device.  d_f[i] and
 * d_sigma[i] receive scan i's G doubles; d_axis_vals[i] holds its lists on
 * the device (entries may be NULL when M = 0); when d_axis_vals itself is
 * NULL the library stages scans[i].axis_vals into memory the batch owns.
 * The descriptors are read only during this call; the device buffers must
 * stay valid until zmc_batch_destroy.  Returns ZMC_E_INVALID (naming the
 * scan) for any invalid descriptor. */
zmc_status zmc_batch_create(const zmc_scan_desc* scans, int32_t n_scans,
                            const double* const* d_axis_vals, double* const* d_f,
                            double* const* d_sigma, const zmc_batch_opts* opts,
                            zmc_batch** out);

/* Enqueues the whole batch on `stream` (graph replay or direct launches).
 * Calls on one batch must not overlap on the device: they share its
 * counters and partials. */
zmc_status zmc_batch_launch(zmc_batch* batch, void* stream);

zmc_status zmc_batch_get_info(const zmc_batch* batch, zmc_batch_info* info);

/* Frees the batch after waiting for its work to finish. */
zmc_status zmc_batch_destroy(zmc_batch* batch);

/* One-shot: create, launch on `stream`, wait for the stream, destroy. */
zmc_status zmc_scan_batch(const zmc_scan_desc* scans, int32_t n_scans,
                          const double* const* d_axis_vals, double* const* d_f,
                          double* const* d_sigma, void* stream);

/* Where the tile table came from: a file path or "built-in defaults". */
const char* zmc_tune_source(void);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.  Scans are submitted
 * one by one at any time; a scheduler thread admits them in arrival order
 * while their device state (staged lists and split partials) fits the HBM
 * budget and a slot is free, cuts each into the same tiles a batch would
 * (so every result is bitwise the same alone, in a batch or in the mix),
 * and runs short slices: each slice takes tiles round-robin from all
 * admitted requests and runs them in one persistent kernel per precision,
 * so requests that arrive while others are on the GPU join the next slice
 * and their work overlaps on the device.  A request completes when its last
 * tile and its split merge have run; its latency is completion minus submit
 * time.  Requests that can never fit the budget fail with ZMC_E_NOMEM.
 * ---------------------------------------------------------------------- */
typedef struct zmc_server zmc_server;

typedef struct zmc_server_opts {
  uint64_t hbm_budget_bytes;   /* device-state budget of admitted requests
                                  (0 = 64 GiB)                               */
  int32_t max_slots;           /* admitted requests at once (0 = 256)        */
  int32_t slice_tiles;         /* at most this many tiles per slice
                                  (0 = 64 per resident block)                */
  int32_t max_inflight;        /* slices enqueued ahead of the device (0 = 2) */
  int32_t cu_count;            /* compute units (0 = device)                 */
  uint64_t slice_samples;      /* samples per slice, shared equally among
                                  the admitted requests, the rest oldest
                                  first (0 = 4e9, a few ms of device time)    */
  int32_t admission;           /* zmc_admission: order of admission from the
                                  queue (0 = arrival order)                  */
  int32_t max_wait_ms;         /* ZMC_ADMIT_SHORTEST only: a request queued
                                  longer than this is admitted before any
                                  shorter one, oldest first (0 = no bound)    */
  int32_t slice_us;            /* > 0: size slices for about this much device
                                  time in microseconds: slices take
                                  slice_samples until the server has measured
                                  the device's throughput on them, then that
                                  throughput times slice_us (a slice never
                                  lasts less than its longest tile); 0 = every
                                  slice takes slice_samples                  */
} zmc_server_opts;

/* Admission order.  Arrival order (FIFO) gives every request the same queueing
 * delay.  Shortest first admits the queued request with the least estimated
 * device work (G * samples * N) whenever a slot and budget are free: under
 * overload most requests are small and finish within milliseconds, while the
 * largest ones wait; max_wait_ms bounds that wait.  Results do not depend on
 * the order (each request's f and sigma are bitwise its alone result). */
typedef enum zmc_admission {
  ZMC_ADMIT_FIFO = 0,
  ZMC_ADMIT_SHORTEST = 1
} zmc_admission;

typedef struct zmc_server_stats {
  uint64_t submitted, admitted, completed, failed;
  uint64_t pending;            /* waiting for admission                      */
  uint64_t active;             /* admitted, not yet complete                 */
  uint64_t samples_completed;  /* sum of G * samples over completed requests */
  uint64_t slices;             /* slices launched                            */
  uint64_t tiles;              /* tiles launched                             */
  uint64_t bytes_in_use;       /* device state held by admitted requests     */
  uint64_t bytes_peak;
  /* Over the most recent 65536 completed requests (0 before the first):
   * latency (completion - submission, seconds) at the 50th and 99th
   * percentiles (linear interpolation between order statistics) and its
   * maximum; and samples_completed / (last completion - first submission). */
  double latency_p50_s, latency_p99_s, latency_max_s;
  double samples_per_s;
  uint64_t tickets;            /* requests still tracked: submitted and not yet
                                  released with zmc_server_release           */
  uint64_t slice_samples_now;  /* the sample budget of the next slice        */
  uint64_t cancelled;          /* requests finished by zmc_server_cancel (also
                                  counted in failed)                          */
} zmc_server_stats;

/* Starts the scheduler thread on the current device (opts may be NULL for
 * all defaults; max_slots > 65536, max_inflight > 16, an unknown admission,
 * a negative max_wait_ms or a negative slice_us give ZMC_E_INVALID).  submit, poll, wait
 * and get_stats may be called from any number of threads at once; destroy
 * must not overlap any other call on the same server, and the handle is
 * invalid once it has returned. */
zmc_status zmc_server_create(const zmc_server_opts* opts, zmc_server** out);

/* Queues one scan; never waits for the GPU.  The descriptor and its host
 * arrays are copied (and dropped once the request finishes).  d_axis_vals
 * may be NULL (the server stages desc->axis_vals); d_f and d_sigma (G
 * doubles each) must stay valid until the request completes, and no work on
 * another stream may still be using them when submit is called (the server
 * writes them from its own streams).  *ticket identifies the request until
 * zmc_server_release. */
zmc_status zmc_server_submit(zmc_server* server, const zmc_scan_desc* desc,
                             const double* d_axis_vals, double* d_f, double* d_sigma,
                             uint64_t* ticket);

/* Non-blocking: *done = 1 when the request has finished, with its status and
 * latency in seconds (submit to completion). */
zmc_status zmc_server_poll(zmc_server* server, uint64_t ticket, int32_t* done,
                           zmc_status* result, double* latency_s);

/* Blocks until the request has finished. */
zmc_status zmc_server_wait(zmc_server* server, uint64_t ticket, zmc_status* result,
                           double* latency_s);

/* Forgets a finished request: its ticket becomes unknown to poll, wait and
 * release (ZMC_E_INVALID), and the server drops what it still held for it
 * (status and latency).  ZMC_E_BUSY if the request has not finished.  A
 * server keeps every unreleased ticket until zmc_server_destroy, so a
 * long-running caller releases each request once it has read its result. */
zmc_status zmc_server_release(zmc_server* server, uint64_t ticket);

/* Cancels a request that has not been admitted yet: it finishes with status
 * ZMC_E_CANCELLED (poll and wait report it; its d_f and d_sigma are never
 * written) and leaves the queue.  ZMC_E_BUSY if it has already been admitted
 * (it then runs to completion) or has finished; ZMC_E_INVALID for an unknown
 * ticket.  For callers whose client went away while the request queued. */
zmc_status zmc_server_cancel(zmc_server* server, uint64_t ticket);

zmc_status zmc_server_get_stats(zmc_server* server, zmc_server_stats* stats);

/* Finishes every submitted request (the queued ones included), stops the
 * thread, frees the server.  Callers must first return from every other call
 * on this server (a thread still blocked in zmc_server_wait would wake on
 * freed memory). */
zmc_status zmc_server_destroy(zmc_server* server);

#ifdef __cplusplus
}
#endif

#endif /* ZMC_H */
