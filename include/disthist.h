/*
 * disthist.h -- C ABI of libdisthist, particle-pair distance histograms on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (Reuter & Koefinger, "CADISHI: Fast parallel calculation of
 * particle-pair distance histograms on CPUs and GPUs", arXiv:1808.01478):
 *
 *   For a frame of particles grouped into species, and for every unordered
 *   species pair (s, t), count the pairs whose distance falls into each of
 *   n_bins half-open bins [k*dr, (k+1)*dr), dr = r_max / n_bins
 *   (Sec. 2.1, Eq. 4). For s != t all N_s*N_t pairs are counted, for s == t
 *   the N_s(N_s-1)/2 pairs with j > i (Sec. 2.2, Algorithm 1 and the
 *   single-species variant). The distance is the Euclidean length of the
 *   difference vector x_j - x_i after the minimum image convention for
 *   periodic cells (Sec. 2.3, Eq. 5; for triclinic cells beyond half the
 *   smallest cell width the 26 neighbouring images are searched as well).
 *   The bin index is (int)(n_bins * r / r_max) (Algorithm 1), evaluated as
 *   t = r * s with s = n_bins / r_max; pairs with t >= n_bins are out of
 *   range and are not counted in any bin.
 *
 * Conventions shared by every entry point
 *   coords        [N][3] binary64 Cartesian coordinates, C-contiguous,
 *                 species-contiguous: species s is rows
 *                 [offsets[s], offsets[s+1]).
 *   offsets       host int64 [n_species+1], offsets[0] = 0, non-decreasing,
 *                 N = offsets[n_species] <= 2^31 - 1.
 *   n_species     1..64.
 *   box_type      DH_BOX_NONE, DH_BOX_ORTHO or DH_BOX_TRICLINIC.
 *   box           host binary64 [3][3], rows are the cell vectors a, b, c.
 *                 Ignored (may be NULL) for DH_BOX_NONE. Orthorhombic: a
 *                 positive diagonal and zero off-diagonal entries.
 *                 Triclinic: lower triangular (a_y = a_z = b_z = 0) with a
 *                 positive diagonal, reduced so that |b_x| <= a_x/2,
 *                 |c_x| <= a_x/2 and |c_y| <= b_y/2.
 *   r_max         finite, > 0.
 *   n_bins        1..2^24 for DH_FP64, 1..2^22 for DH_FP32 (beyond 2^22 a
 *                 binary32 t is spaced half a bin or more apart).
 *   precision     DH_FP64: the canonical binary64 evaluation below; counts
 *                 are exactly those of that op sequence.
 *                 DH_FP32: a binary32 evaluation; a pair may change bin
 *                 only if its binary64 distance lies within a few binary32
 *                 ulps of the bin edge. The bin is taken from the bits of
 *                 t + (2^23 - 1/2) rounded to nearest, which is floor(t)
 *                 except that an exactly integer odd t counts one bin
 *                 lower (a tie); in a cube r * s and the offset are one
 *                 fused operation. Every device path (LDS histograms, bin
 *                 windows, global atomics, batches) bins alike, so binary32
 *                 counts do not depend on the launch shape.
 *   histograms    uint64 [H][n_bins], H = n_species*(n_species+1)/2, in the
 *                 order (0,0),(1,1),...,(k-1,k-1), then (s,t) for s < t in
 *                 lexicographic order. Always overwritten.
 *
 * Canonical binary64 arithmetic (IEEE-754 round to nearest even, nothing
 * fused except the fma() written, correctly rounded sqrt):
 *   d = x_j - x_i
 *   orthorhombic: n_c = rint(d_c * (1/L_c)); d_c = fma(-L_c, n_c, d_c)
 *   triclinic:    sc = dz*h33; sb = fma(dz, h23, dy*h22);
 *                 sa = fma(dz, h13, fma(dy, h12, dx*h11)); n = rint(s);
 *                 dz = fma(-cz, nc, dz); dy = fma(-cy, nc, fma(-by, nb, dy));
 *                 dx = fma(-cx, nc, fma(-bx, nb, fma(-ax, na, dx)))
 *                 with h11 = 1/ax, h22 = 1/by, h33 = 1/cz, h12 = -bx/(ax*by),
 *                 h23 = -cy/(by*cz), h13 = (bx*cy - by*cx)/(ax*by*cz)
 *   q = fma(dz, dz, fma(dy, dy, dx*dx)); when 2*r_max >= w_min*(1 - 1e-9)
 *   in a triclinic cell (w_min: smallest face-to-face width), q is the
 *   minimum of that expression over d + S for the 27 shifts
 *   S = i*a + j*b + k*c, i, j, k in {-1, 0, 1};
 *   t = sqrt(q) * (n_bins / r_max); bin floor(t) if t < n_bins.
 * The device square root is the compiler's own binary64 sequence (rsq seed,
 * Goldschmidt step, two fused Newton corrections); for about 2^-44 of
 * arguments it may return the neighbour of the correctly rounded root, which
 * moves a count only if t also sits within about 2^-52 of a bin edge.
 *
 * Errors: every entry point returns DH_OK (0) or a negative DH_E* code.
 * Argument errors (DH_EINVAL) are detected before anything is written or
 * launched. dh_strerror() gives a static description of a code, and
 * dh_ctx_last_error() the message of the last failure on a context.
 *
 * Threading: a context may be used by one host thread at a time, and the
 * calls on one context are ordered on the streams they are issued on; give
 * each concurrent stream its own context.
 */
#ifndef DISTHIST_H
#define DISTHIST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DH_OK 0
#define DH_EINVAL (-1)      /* invalid argument; nothing written */
#define DH_ENOMEM (-2)      /* device or pinned host allocation failed */
#define DH_EDEVICE (-3)     /* a HIP call failed; see dh_ctx_last_error */
#define DH_EBUDGET (-4)     /* the job does not fit the context's memory budget */
#define DH_EUNSUPPORTED (-5)

#define DH_BOX_NONE 0
#define DH_BOX_ORTHO 1
#define DH_BOX_TRICLINIC 2

#define DH_FP32 0
#define DH_FP64 1

typedef struct dh_ctx dh_ctx;

/* A hipStream_t. NULL is the null stream of the context's device. */
typedef void *dh_stream;

/* Library version as "major.minor.patch". */
const char *dh_version(void);

/* Static text for a status code. */
const char *dh_strerror(int code);

/*
 * Validates the arguments of a histogram call on the host without touching
 * any device: the rules listed above, plus finiteness of the coordinates when
 * coords is a host pointer (pass coords = NULL to skip that check).
 * Returns DH_OK or DH_EINVAL.
 */
int dh_check_args(const double *coords, const int64_t *offsets, int32_t n_species,
                  int32_t box_type, const double *box, double r_max, int32_t n_bins,
                  int32_t precision);

/*
 * Synchronous histogram of one frame from host memory (Sec. 2.2,
 * Algorithm 1; Sec. 3.2 on staging a whole frame in one transfer).
 *   coords   host [N][3] binary64.
 *   out      host uint64 [H][n_bins], overwritten.
 * Runs on the current HIP device through a library-owned context whose
 * device buffers are allocated at the first call and reused (Sec. 3.2).
 * The call returns when the result is in out. Thread-safe (calls on one
 * device are serialised).
 */
int dh_histo(const double *coords, const int64_t *offsets, int32_t n_species,
             int32_t box_type, const double *box, double r_max, int32_t n_bins,
             int32_t precision, uint64_t *out);

/*
 * Creates a context on HIP device `device` (the per-device state of the
 * paper's GPU kernel: the device buffers it keeps between calls and reuses
 * for every frame, Sec. 3.2). The context owns device scratch (staged
 * coordinates, sort keys, work lists, counters) that grows on demand and is
 * reused; it never frees caller memory.
 *   hbm_budget_bytes  the most device memory the context may hold: its
 *                     scratch plus the buffers of its live batches; 0 for no
 *                     limit. A call or dh_batch_create that would need more
 *                     fails with DH_EBUDGET and the context stays usable;
 *                     no output has been written, unless the call was
 *                     tuning its launch shape (DH_TUNE_ON), whose trial
 *                     runs write the output. Caller buffers do not count.
 * *ctx receives the handle (NULL on failure); DH_EINVAL for a negative
 * budget or a device index out of range, DH_ENOMEM or DH_EDEVICE if the
 * device cannot be set up.
 */
int dh_ctx_create(int32_t device, int64_t hbm_budget_bytes, dh_ctx **ctx);

/* Releases a context and its scratch (synchronises its device first). */
void dh_ctx_destroy(dh_ctx *ctx);

/* The message of the last failed call on ctx ("" if none). With ctx = NULL,
 * the message of the last failure on the calling thread (for failures that
 * have no context, such as dh_ctx_create or dh_histo). */
const char *dh_ctx_last_error(const dh_ctx *ctx);

/*
 * Asynchronous histogram of one frame already resident in device memory
 * (Algorithm 1 with Eq. 5's minimum image, Sec. 2.2; the GPU kernel of
 * Sec. 3.2: coordinates staged once per frame, pairs counted into
 * sub-histograms in shared memory and summed into d_out).
 *   d_coords         device [N][3] binary64; read by kernels on `stream`
 *                    after the call returns, so it must stay valid until
 *                    the stream reaches this work.
 *   offsets, box     host memory, read during the call only.
 *   d_out            device uint64 [H][n_bins], overwritten on `stream`.
 *   d_out_of_range   device uint64 [H] or NULL: pairs of each histogram
 *                    in no bin (t >= n_bins; binary32 by its bin rule).
 * The work is enqueued on `stream` and the call returns without waiting.
 * Device coordinates are not checked for finiteness; non-finite input
 * yields meaningless counts but never out-of-bounds accesses.
 */
int dh_histo_async(dh_ctx *ctx, dh_stream stream, const double *d_coords,
                   const int64_t *offsets, int32_t n_species, int32_t box_type,
                   const double *box, double r_max, int32_t n_bins, int32_t precision,
                   uint64_t *d_out, uint64_t *d_out_of_range);

/*
 * dh_histo_async without any allocation, for callers that cannot allocate
 * device or pinned memory: work under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. No context: the call runs on the
 * current HIP device, enqueues its kernels on `stream` and returns without
 * waiting. Arguments, layouts and validation as for dh_histo_async; the
 * counts are the same as dh_histo_async's (built-in launch shape, no tuning).
 * Scratch: one fixed device array per device, 48 MiB, held by every device
 * the library runs on until the process ends (frame constants, work list,
 * counters and the staged coordinates, 16 bytes per point in binary32 and 32
 * in binary64: about 1.4 million binary64 or 2.9 million binary32 points;
 * frames of at least 65,536 points staged in spatial order, triclinic ones
 * and binary64 orthorhombic ones, take 32 bytes per point and sort keys:
 * about 1.0 million points).
 * A frame that does not fit gets DH_EINVAL before anything is enqueued.
 * Calls share that array: calls that overlap on one device (several streams
 * or host threads) race and must be serialised by the caller. Failures
 * without a context: message via dh_ctx_last_error(NULL).
 */
int dh_histo_noalloc(dh_stream stream, const double *d_coords, const int64_t *offsets,
                     int32_t n_species, int32_t box_type, const double *box, double r_max,
                     int32_t n_bins, int32_t precision, uint64_t *d_out,
                     uint64_t *d_out_of_range);

/*
 * Scaled distances t = r * n_bins / r_max of explicit particle pairs,
 * evaluated with the device arithmetic that the histogram kernels use for
 * the given precision and box (Algorithm 1 without the increment): exactly
 * in binary64; in binary32 with periodic cells the pair kernel takes the c
 * differences of two i-particles from one 64-bit addition, which can lower
 * the second one by one fixed-point unit (2^-32 of the cell vector), and in
 * a cube it fuses the final scale with the bin offset, so the returned t is
 * the unfused product.
 * For checking sampled pairs of frames too large for an exhaustive CPU
 * comparison.
 *   d_coords   device [n][3] binary64 (one species; n <= 2^31 - 1).
 *   d_pi, d_pj device int32 [n_pairs] particle indices in [0, n).
 *   d_t        device binary64 [n_pairs] output (binary32 results widened).
 * Asynchronous on `stream`; indices are not range-checked on the device
 * beyond clamping into [0, n).
 */
int dh_pair_t_async(dh_ctx *ctx, dh_stream stream, const double *d_coords, int64_t n,
                    int32_t box_type, const double *box, double r_max, int32_t n_bins,
                    int32_t precision, const int32_t *d_pi, const int32_t *d_pj,
                    int64_t n_pairs, double *d_t);

/* ---------------------------------------------------------------------------
 * Batches: many frames (a trajectory, or frames of unrelated jobs) planned
 * once and run as one graph of launches. All species pairs of all frames
 * become work items of persistent pair kernels (one launch per class of
 * frames with the same minimum-image kind and bin-window mode), so frames of
 * very different sizes share the GPU without a launch per frame (the paper
 * launches per coordinate tile and keeps frames independent, Sec. 3.2.2 and
 * Sec. 3.2.4). Items of large frames are scheduled first.
 */
typedef struct dh_batch dh_batch;

typedef struct {
  const double *d_coords;      /* device [N][3] binary64; read at every launch   */
  const int64_t *offsets;      /* host [n_species+1]; copied at creation         */
  int32_t n_species;
  int32_t box_type;
  const double *box;           /* host [3][3] or NULL; copied at creation        */
  double r_max;
  int32_t n_bins;
  uint64_t *d_out;             /* device [H][n_bins]; overwritten at every launch */
  uint64_t *d_out_of_range;    /* device [H] or NULL                              */
} dh_frame_desc;

/* dh_batch_create flags */
#define DH_BATCH_GRAPH 1       /* capture the launch sequence in a hipGraph */

/*
 * Plans a batch of n_frames (1..65535) frames in one precision. The device
 * pointers of every frame are baked into the plan: each dh_batch_launch reads
 * the coordinates currently in d_coords and overwrites d_out, so a caller
 * streams a trajectory by refilling the same buffers between launches.
 * Frame shapes (species sizes, box, r_max, n_bins) are fixed at creation.
 * Validation as for dh_histo_async (DH_EINVAL before anything is allocated).
 * The batch owns its device memory (staged coordinates, work list); it keeps
 * a reference to ctx, which must outlive it.
 */
int dh_batch_create(dh_ctx *ctx, const dh_frame_desc *frames, int32_t n_frames,
                    int32_t precision, int32_t flags, dh_batch **batch);

/* Enqueues the whole batch on `stream` (a graph replay with DH_BATCH_GRAPH). */
int dh_batch_launch(dh_batch *batch, dh_stream stream);

/* Work items, pair-kernel launches per run, and pairs per run of a batch. */
int dh_batch_info(const dh_batch *batch, int64_t *n_items, int32_t *n_launches,
                  double *total_pairs);

/* Releases a batch (synchronises its device first). */
void dh_batch_destroy(dh_batch *batch);

/* ---------------------------------------------------------------------------
 * Serving: a request loop that runs histogram jobs of mixed sizes, boxes and
 * bin counts on one GPU with continuous batching. A scheduler thread admits
 * queued jobs while a slot is free and the job's device footprint fits the
 * HBM budget (see dh_sched_select for the order); an admitted job's frame is
 * copied to the device, staged and zeroed on a setup stream while other
 * jobs compute, and stays resident in its slot. Every pair-kernel launch is
 * then built from the work items of all ready jobs that share a kernel
 * variant (precision, minimum-image kind, accumulation mode, launch shape),
 * taken in policy order up to a bounded amount of work per launch (about 10
 * ms), with at most two launches on the device: a job admitted while others
 * run joins the next launch, its items computed in the same launch as pieces
 * of the running jobs. The default policy takes the job with the least work
 * left first (shortest remaining work); DH_SCHED_ARRIVAL uses arrival order
 * for admission and launches (with one slot: one job at a time, FIFO). When
 * a launch carries a job's last items, its results are copied out after
 * that launch; completion is detected with events. The paper's counterpart
 * is its producer/consumer engine that feeds frames to GPU workers through
 * queues (Sec. 3.3); here the unit handed to the device is a work item, so
 * one launch computes several frames.
 */
typedef struct dh_server dh_server;

#define DH_JOB_DONE 0
#define DH_JOB_QUEUED 1
#define DH_JOB_RUNNING 2

/*
 * Creates a server on `device` with `max_inflight` (1..64) slots (jobs
 * resident at once) and an HBM budget in bytes for the footprints of
 * resident jobs (coordinates, staged copy, histograms, out-of-range and
 * pair counts). head_wait_limit_s < 0 selects 1 second.
 */
int dh_server_create(int32_t device, int64_t hbm_budget_bytes, int32_t max_inflight,
                     double head_wait_limit_s, dh_server **server);

/*
 * Queues one job (arguments as dh_histo, host memory, copied before return)
 * and returns its id. DH_EINVAL for invalid arguments, DH_EBUDGET when the
 * job's footprint alone exceeds the budget; neither queues anything.
 */
int dh_server_submit(dh_server *server, const double *coords, const int64_t *offsets,
                     int32_t n_species, int32_t box_type, const double *box, double r_max,
                     int32_t n_bins, int32_t precision, int64_t *job_id);

#define DH_SCHED_SHORTEST 0 /* least work first (the default) */
#define DH_SCHED_ARRIVAL 1  /* arrival order */

/* Sets the order in which queued jobs are admitted and admitted jobs'
 * launches are issued; takes effect at the next scheduling step. DH_EINVAL
 * for another value. */
int dh_server_set_policy(dh_server *server, int32_t policy);

/* DH_JOB_QUEUED, DH_JOB_RUNNING, DH_JOB_DONE, or the job's negative error;
 * DH_EINVAL for an unknown id. */
int dh_server_status(dh_server *server, int64_t job_id);

/*
 * Waits for a job, copies its histograms (uint64 [H][n_bins]) and
 * out-of-range counts ([H]) to host memory (either may be NULL) and releases
 * it. times[3] (may be NULL) = seconds queued, seconds running, and the
 * latency from submission to completion. Returns the job's status.
 */
int dh_server_wait(dh_server *server, int64_t job_id, uint64_t *out, uint64_t *out_of_range,
                   double *times);

/*
 * stats[6] = jobs submitted, completed, failed, the largest number of jobs
 * running at once, the largest sum of admitted footprints (bytes), and the
 * budget (bytes).
 */
int dh_server_stats(const dh_server *server, int64_t *stats);

/*
 * Pair-kernel launches issued so far, how many of them carried the work
 * items of more than one job, and the most jobs one launch carried.
 */
int dh_server_launch_stats(const dh_server *server, int64_t *launches,
                           int64_t *shared_launches, int64_t *max_jobs_per_launch);

/* Finishes running jobs, drops queued ones, releases the server. */
void dh_server_destroy(dh_server *server);

/*
 * The admission policy of the server as a pure host function (no device):
 * given the queued jobs in arrival order (footprints, seconds waited and,
 * optionally, their work in pairs), the free budget and the free slots,
 * writes the queue positions to start now into admit[] (ascending) and
 * returns how many. Jobs that have waited at least head_wait_limit_s come
 * first, oldest first, and one of them that does not fit stops all
 * admissions (the memory running jobs free goes to it). The others follow
 * in order of increasing work (arrival order when work is NULL), each if it
 * fits: small jobs do not queue behind large ones, and the wait limit
 * bounds how long a large one can be passed over.
 */
int32_t dh_sched_select(const int64_t *need_bytes, const double *waited_s, const double *work,
                        int32_t n_queued, int64_t free_bytes, int32_t free_slots,
                        double head_wait_limit_s, int32_t *admit);

/*
 * The image lists of the 27-image search for a triclinic cell (Sec. 2.3's
 * neighbouring images beyond half the smallest width), as a pure host
 * function (no device). For each octant o of a reduced vector's fractional
 * coordinates (bit k of o set when component k is negative), the shift
 * indices m = 9(i+1) + 3(j+1) + (k+1) of the images i a + j b + k c that can
 * be nearer than the vector itself, ascending: the other images are farther
 * at every point of the octant's box by more than a margin, so the minimum
 * over the list equals the minimum over all 27. The pair kernels search only
 * these lists, except that an octant whose list is longer than 12 searches
 * all 27 images (full_mask bit o).
 *   box        host [3][3], rows a, b, c, as for a histogram call.
 *   lists      host int32 [8][26], overwritten; entries past an octant's
 *              count hold 13 (the zero shift).
 *   counts     host int32 [8], the list lengths.
 *   full_mask  host int32, the octants searched in full.
 * Returns DH_OK, or DH_EINVAL for a null pointer or a box a histogram call
 * would reject.
 */
int dh_search_images(const double *box, int32_t *lists, int32_t *counts, int32_t *full_mask);

/* ---------------------------------------------------------------------------
 * Tuned CPU kernel (the paper's cache-blocked CPU kernel, Sec. 3.1: tiles
 * sized for the L2, triangular tiles on the diagonal, coordinates as
 * separate arrays for the vectorizer, bin indices of a row buffered then
 * scattered into thread-private histograms). Host memory only, no device.
 * Same arguments and outputs as dh_histo (out [H][n_bins] overwritten;
 * out_of_range [H] optional, may be NULL); n_threads = 0 uses the CPUs of
 * the process's affinity mask, at most OMP_NUM_THREADS when that is set.
 * binary64 follows the canonical sequence (counts equal to the GPU path's);
 * binary32 rounds coordinates and constants once and runs the same sequence
 * in binary32, with bin floor(t) (the device's binary32 bin rule differs
 * from it only at integer t). DH_EINVAL as dh_histo.
 */
int dh_cpu_histo(const double *coords, const int64_t *species_offsets, int32_t n_species,
                 int32_t box_type, const double *box, double r_max, int32_t n_bins,
                 int32_t precision, int32_t n_threads, uint64_t *out_u64,
                 uint64_t *out_of_range);

/* ---------------------------------------------------------------------------
 * Trajectory engine (the paper's frame-parallel engine reads frames, runs
 * them on its workers and sums the histograms over intervals of frames in
 * its writer, Sec. 3.3 and Sec. 4.4; this is its one-GPU form).
 *
 * Trajectory file (little-endian): a 64-byte header
 *   char magic[8] = "DHTRAJ01"; int64 n_frames; int64 n_points;
 *   int32 box_type; zero padding to 64 bytes
 * then n_frames frames of (double box[9], rows a, b, c; zeros for
 * DH_BOX_NONE) followed by double coords[n_points][3]. The species layout
 * (offsets) is the same for every frame and passed to dh_traj_histo.
 * dh_traj_open checks the header and the file size (DH_EINVAL otherwise);
 * the handle reads the file, it never writes it.
 */
typedef struct dh_traj dh_traj;
int dh_traj_open(const char *path, dh_traj **out);
int dh_traj_info(const dh_traj *t, int64_t *n_frames, int64_t *n_points, int32_t *box_type);
void dh_traj_close(dh_traj *t);

/*
 * Histograms of frames [frame_begin, frame_end), summed over consecutive
 * intervals of `interval` frames (the last interval may be shorter). A host
 * thread reads frames into pinned buffers, the copy of frame f + 1 to the
 * device overlaps the histogram of frame f, and each frame runs the same
 * path as dh_histo_async (its own box, tuned shapes of ctx), adding into the
 * interval's sums.
 *
 * results_path receives a 128-byte header (magic "DHRES001", a hash of all
 * parameters and the species offsets, then the parameters) followed by one
 * record per finished interval: uint64 hist[H][n_bins], uint64
 * out_of_range[H], uint64 frames_in_interval. Each record is written and
 * synced before the next interval starts, so the file is the checkpoint: a
 * call with the same parameters and an existing file skips the intervals
 * already recorded (a partial trailing record is cut off and redone); a
 * file of other parameters gives DH_EINVAL. max_intervals > 0 stops after
 * that many new intervals (0: run to frame_end). *intervals_done receives
 * the number of complete records in the file on return. An invalid frame
 * (its box) stops the run with that frame's error before its interval is
 * recorded. Blocks until done; ctx must not be used by another thread
 * meanwhile.
 */
int dh_traj_histo(dh_ctx *ctx, dh_traj *t, const int64_t *species_offsets, int32_t n_species,
                  double r_max, int32_t n_bins, int32_t precision, int64_t frame_begin,
                  int64_t frame_end, int64_t interval, const char *results_path,
                  int64_t max_intervals, int64_t *intervals_done);

/*
 * dh_traj_histo with a CPU worker beside the GPU (the paper's hybrid of CPU
 * and GPU workers, Sec. 3.3 and Table 4): a host thread runs dh_cpu_histo on
 * `cpu_threads` threads over whole frames taken from the end of each
 * interval while the GPU takes them from the start, and the interval's
 * record adds both (binary64 counts are the same either way; binary32 frames
 * computed on the CPU follow the canonical sequence in binary32 and stay
 * within the binary32 tolerance). The CPU takes a frame only when its
 * measured time per frame (before the first one: 2e8 pairs per second per
 * thread) is below the GPU's measured time for the other unclaimed frames of
 * the interval, so it cannot hold an interval back by much more than one GPU
 * frame; flags = DH_HYBRID_GREEDY lifts that rule (every frame the CPU
 * worker can claim, for tests). cpu_threads = 0 is dh_traj_histo.
 * *cpu_frames (may be NULL) receives the number of frames the CPU computed.
 */
#define DH_HYBRID_GREEDY 1
int dh_traj_histo_hybrid(dh_ctx *ctx, dh_traj *t, const int64_t *species_offsets,
                         int32_t n_species, double r_max, int32_t n_bins, int32_t precision,
                         int64_t frame_begin, int64_t frame_end, int64_t interval,
                         const char *results_path, int64_t max_intervals, int32_t cpu_threads,
                         int32_t flags, int64_t *intervals_done, int64_t *cpu_frames);

/* ---------------------------------------------------------------------------
 * Launch tuning. The launch shape of a frame (i-particles per lane, LDS
 * sub-histogram copies, j-tile length, unclamped interior blocks, workgroups
 * per CU, work items per workgroup, workgroup size, and for histograms wider
 * than LDS the choice between LDS bin windows and uint64 global atomics)
 * changes speed only: every shape gives the same counts (the paper picks its
 * block size by fixed heuristics, Sec. 3.2.4, and its shared- or
 * global-memory kernel by the number of bins, Sec. 4.2).
 *
 *   DH_TUNE_OFF     built-in defaults
 *   DH_TUNE_CACHED  use cached shapes, never measure
 *   DH_TUNE_ON      on a cache miss, time candidate shapes on the call's own
 *                   frame (the call blocks until done), cache the fastest
 * Shapes are cached per bucket (architecture, precision, minimum-image
 * kind, ceil(log2 n_bins), ceil(log2 N), species up to 4). With a
 * cache_path, existing entries are loaded now and new ones saved as JSON.
 * Environment defaults for new contexts: DH_TUNE (mode), DH_TUNE_CACHE.
 */
#define DH_TUNE_OFF 0
#define DH_TUNE_CACHED 1
#define DH_TUNE_ON 2
int dh_ctx_set_tuning(dh_ctx *ctx, int32_t mode, const char *cache_path);

/*
 * Forces a launch shape for every later call on ctx and for batches created
 * on it (NULL restores tuning):
 * knobs[8] = {r (4|8), copies (1|2|4), tj (128|256), noclamp (0|1),
 * occ_cap (0..16, 0 = as many as fit), items_per_wg (1..64),
 * threads (256|512|1024, or 0 = the smallest workgroup that gives every SIMD
 * four waves within the LDS limit on workgroups per CU; the 27-image search
 * always runs 256),
 * wide (0..65536: count with uint64 global atomics instead of LDS
 * sub-histograms when the histogram would need at least this many LDS bin
 * windows; 0 = never, 1 = always)}.
 * Invalid knob values give DH_EINVAL.
 */
int dh_ctx_set_config(dh_ctx *ctx, const int32_t *knobs);

/*
 * The shape of the last single-frame launch on ctx: out[13] = the first six
 * knobs, the workgroup size launched, the wide knob, the grid size, LDS
 * bytes per workgroup, bin-window sweeps, work items, and the accumulation
 * mode (0 LDS histogram, 1 LDS bin windows, 2 global atomics).
 */
int dh_ctx_last_config(const dh_ctx *ctx, int32_t *out);

/*
 * Splits every later histogram on ctx into pair-kernel launches of at most
 * max_pairs pairs (0 = one launch per frame, the default; otherwise at least
 * 2^24). Counts are unchanged. A persistent launch holds every CU until its
 * work list is drained; bounded launches let work queued on other streams
 * start between them (the serving loop runs its jobs this way). DH_EINVAL
 * for a negative or too small limit.
 */
int dh_ctx_set_launch_pairs(dh_ctx *ctx, int64_t max_pairs);

/*
 * Kernel timing. When enabled, every histogram launch on ctx records a pair
 * of HIP events on its stream around the pair kernel (the dominant kernel of
 * the path); batches are not timed this way. dh_ctx_profile_read() waits for the recorded launches, returns
 * the summed kernel time in milliseconds and the number of launches, and
 * resets both. Enabling or disabling also resets them.
 */
int dh_ctx_profile(dh_ctx *ctx, int32_t enable);
int dh_ctx_profile_read(dh_ctx *ctx, double *kernel_ms, int64_t *launches);

/*
 * Pairs that went through the 27-image search (Sec. 2.3, the neighbouring
 * cells beyond half the smallest width; Sec. 4.1, the three-fold loop over
 * neighbouring boxes) in the last single-frame histogram on ctx
 * (dh_histo_async or dh_histo through ctx): the pairs whose Eq. 5 reduced
 * vector is at least half the shortest lattice vector long, counted by the
 * pair kernel. 0 when that call ran no search (r_max below half the smallest
 * width, or no triclinic cell) or the frame was added into an accumulating
 * sum. The caller must have waited for that call's stream; this reads the
 * device counter with a blocking copy. DH_EINVAL for a null argument.
 */
int dh_ctx_searched_pairs(dh_ctx *ctx, uint64_t *searched);

/*
 * Images evaluated for those pairs in the same call (Sec. 2.3's neighbouring
 * images; the kernel evaluates for each searched vector only the images of
 * its octant list, or all 27, and a wave runs to its longest list, so this
 * is the arithmetic actually spent on the search). 0 as for
 * dh_ctx_searched_pairs; same waiting rule and errors.
 */
int dh_ctx_searched_images(dh_ctx *ctx, uint64_t *images);

#ifdef __cplusplus
}
#endif

#endif /* DISTHIST_H */
