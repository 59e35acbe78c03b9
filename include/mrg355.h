/*
 * mrg355.h -- C ABI of the MI355X (gfx950) multi-stream MRG32k3a generator.
 *
 * The calls follow the problem as the clrng paper states it (Xu, Brown,
 * L'Ecuyer, "clrng: A tool set for parallel random number generation on GPUs
 * in R"): create streams from a 6-integer seed (Section 2.1), generate n
 * numbers of a distribution and dtype from explicit streams (Sections 2.2,
 * 3.1, 3.2), save and restore stream state (Section 2.2, save/restore
 * example).  The generator is MRG32k3a (L'Ecuyer 1999), the one the paper
 * names as prior art and future work (Sections 1, 2, 6).
 *
 * Conventions (every entry point):
 *   - Returns mrg_status: MRG_OK (0) or a negative error.  mrg_last_error()
 *     returns a thread-local message for the last failing call.
 *   - Arguments are validated before any side effect: on error no kernel is
 *     launched, no device memory is written and no creator is advanced.
 *   - Device work is enqueued asynchronously on the caller's hipStream_t
 *     (NULL = the default stream).  Faults of already enqueued kernels
 *     surface at the next synchronising HIP call.
 *   - The caller owns every device buffer (stream records, outputs).  The
 *     library allocates no device memory in these calls.
 *   - "device pointer" means memory from hipMalloc (or a torch CUDA tensor);
 *     "host pointer" means ordinary host memory.
 *   - Not thread-safe per stream array: two calls that touch the same stream
 *     records must be ordered by the caller (same hipStream or events).
 */
#ifndef MRG355_H
#define MRG355_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRG_ABI_VERSION 3

typedef enum {
    MRG_OK = 0,
    MRG_E_INVALID_ARG = -1,   /* null pointer, bad enum, size or alignment   */
    MRG_E_INVALID_SEED = -2,  /* seed violates the validity rule             */
    MRG_E_UNSUPPORTED = -3,   /* generator/dist/dtype combination not built  */
    MRG_E_HIP = -4,           /* a HIP runtime call failed                   */
    MRG_E_NOMEM = -5,         /* host allocation failed / buffer too small   */
    MRG_E_CORRUPT_STATE = -6, /* import: bad magic, version, length or words */
    MRG_E_BUSY = -7           /* mrg_server_poll: the request is not done yet */
} mrg_status;

/* Generators.  MRG32k3a: components mod m1 = 2^32-209 and m2 = 2^32-22853,
 * streams 2^127 apart, substreams 2^76 apart, state words oldest-first
 * (x1[n-3], x1[n-2], x1[n-1], x2[n-3], ...).  MRG31k3p (the paper's own,
 * Section 2): m1 = 2^31-1, m2 = 2^31-21069, streams 2^134 apart (Section
 * 2.1), substreams 2^72 apart, words newest-first (x1[n-1], x1[n-2],
 * x1[n-3], x2[n-1], ...) as in the stream table of Section 2.1, uniforms
 * z / 2^31.  Both run every stream, generate, save/restore and table call;
 * the batch and server calls run MRG32k3a only (MRG_E_UNSUPPORTED). */
typedef enum { MRG_GEN_MRG32K3A = 1, MRG_GEN_MRG31K3P = 2 } mrg_generator;

/* Distributions (Sections 2.2, 3.1, 3.2):
 *   MRG_UNIFORM      u = z / (m1 + 1), strictly inside (0,1)
 *   MRG_NORMAL       Box-Muller (Algorithm 1) on consecutive uniforms of one
 *                    stream: draws 2p, 2p+1 = R cos(2 pi u2), R sin(2 pi u2)
 *                    with R = sqrt(-2 log u1), (u1,u2) = steps 2p, 2p+1
 *   MRG_EXPONENTIAL  -log(u) / rate, rate = `param` (> 0, finite)
 *   MRG_RAW          the integer z in [1, m1] itself (dtype MRG_U32 only)  */
typedef enum { MRG_UNIFORM = 0, MRG_NORMAL = 1, MRG_EXPONENTIAL = 2, MRG_RAW = 3 } mrg_dist;

/* Output element types.  F32 uniforms are the double uniform rounded toward
 * zero (so they stay below 1); F32 normals/exponentials are the double value
 * rounded to nearest.  U32 pairs only with MRG_RAW, and MRG_RAW only with U32. */
typedef enum { MRG_F64 = 0, MRG_F32 = 1, MRG_U32 = 2 } mrg_dtype;

/* The creator: the state the next created stream starts from (the paper's
 * hidden .Random.seed.clrng object, Section 2.1), as an explicit value. */
typedef struct {
    uint32_t s[6];
} mrg_creator;

/* One stream (Section 2.1: current state and initial state; plus the start of
 * the current substream).  Each 6-word state is (x1[n-3], x1[n-2], x1[n-1],
 * x2[n-3], x2[n-2], x2[n-1]): oldest first per component.  72 bytes. */
typedef struct {
    uint32_t cur[6];
    uint32_t start[6];
    uint32_t sub[6];
} mrg_stream;

typedef enum {
    MRG_RESET_STREAM = 0,     /* cur = sub = start                 */
    MRG_RESET_SUBSTREAM = 1,  /* cur = sub                         */
    MRG_NEXT_SUBSTREAM = 2    /* sub = A^(2^76) sub; cur = sub      */
} mrg_reset_kind;

/* Launch shape of mrg_generate_ex.  Results never depend on it: the output
 * position and every value are functions of (stream, draw index) only.
 *   block            threads per block: 0 (automatic), 64, 128, 256, 512, 1024
 *   chunk            draws (normal: pairs) per work-item; 0 = automatic
 *   nontemporal      1 = stream the output with non-temporal stores
 *   arith            0 = automatic, 1 = 32x32->64 integer mod arithmetic,
 *                    2 = the same integers carried exactly in fp64 FMA registers
 *   streams_per_lane 0 = automatic, 1, 2 or 4: a request; the value used is
 *                    the largest not above it that keeps a store within 16
 *                    bytes and divides n_streams, with the output aligned to
 *                    the store width
 *   xcd_remap        1 = give each XCD a contiguous range of row segments
 *   lockstep         1 = the waves of a block write each draw index together
 *                    (a workgroup barrier per row); ignored unless every wave
 *                    of the grid holds 64*streams_per_lane streams           */
typedef struct {
    uint32_t block;
    uint32_t chunk;
    uint32_t nontemporal;
    uint32_t arith;
    uint32_t streams_per_lane;
    uint32_t xcd_remap;
    uint32_t lockstep;
} mrg_launch_cfg;

int         mrg_abi_version(void);
const char* mrg_status_string(mrg_status status);
const char* mrg_last_error(void);

/* Seed rule (RngStreams'; the paper states none): words 0-2 below m1, words
 * 3-5 below m2, neither triple all zero.  MRG_E_INVALID_SEED otherwise; a
 * seed is never reduced mod m.  `seed` is a host pointer to 6 words. */
mrg_status mrg_seed_check(mrg_generator gen, const uint32_t seed[6]);

/* setBaseCreator (Section 2.1): creator := seed after mrg_seed_check. */
mrg_status mrg_creator_init(mrg_generator gen, mrg_creator* creator, const uint32_t seed[6]);

/* createStreamsCpu (Section 2.1): n streams into host memory `host_out`
 * (n records).  Stream i starts at the creator advanced i * 2^127 steps
 * (cur = start = sub); the creator then advances n * 2^127 steps.  n = 0 is
 * a no-op. */
mrg_status mrg_streams_create_host(mrg_generator gen, mrg_creator* creator, size_t n,
                                   mrg_stream* host_out);

/* createStreamsGpu (Section 2.1): the same n streams written by a kernel to
 * device memory `dev_out` (n records, 4-byte aligned, n <= 2^36).  Identical
 * records to mrg_streams_create_host; the creator (host value) advances the
 * same way once the launch has been enqueued. */
mrg_status mrg_streams_create_device(mrg_generator gen, mrg_creator* creator, size_t n,
                                     mrg_stream* dev_out, hipStream_t stream);

/* Substreams (Section 2.1): the period is cut into streams Z steps apart,
 * and each stream can be cut further into substreams, which the paper notes
 * clrng does not implement; the record keeps the start of the current
 * substream as in RngStreams, the package Section 2.1 builds on.  The
 * substream length is 2^76 steps (MRG32k3a) or 2^72 (MRG31k3p).  This call
 * applies one of the mrg_reset_kind operations to n device stream records
 * (4-byte aligned).  n = 0 is a no-op. */
mrg_status mrg_streams_reset(mrg_generator gen, mrg_stream* dev, size_t n, mrg_reset_kind kind,
                             hipStream_t stream);

/* Jump-ahead (Section 2.1, which creates streams by advancing the state Z
 * steps with a matrix power): the current state of each of n device stream
 * records advances by `steps` steps (any count below 2^64), as if that many
 * numbers had been drawn; initial and substream states stay.  n = 0 or
 * steps = 0 is a no-op. */
mrg_status mrg_streams_advance(mrg_generator gen, mrg_stream* dev, size_t n, uint64_t steps,
                               hipStream_t stream);

/* runifGpu / rnormGpu / rexpGpu (Sections 2.2, 3.1, 3.2): n numbers from
 * the n_streams device stream records `dev` into device memory `dev_out`.
 * Stream s makes cnt_s = floor(n/S) + (s < n mod S) draws and draw k of
 * stream s is stored at element k*S + s (S = n_streams): the output is a
 * dense array of n elements whose layout does not depend on the launch.
 * Each stream's current state advances by the steps it consumed (cnt_s;
 * normals 2*ceil(cnt_s/2)).  `param` is the rate of MRG_EXPONENTIAL and is
 * ignored otherwise.  dev_out must be aligned to its element size.
 * n = 0 is a no-op.  Errors: MRG_E_INVALID_ARG (null pointers, n_streams = 0
 * with n > 0, dist/dtype mismatch, bad rate, misalignment, n_streams above
 * 2^31, 2^46 or more draws per stream). */
mrg_status mrg_generate(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t n,
                        mrg_dist dist, mrg_dtype dtype, double param, void* dev_out,
                        hipStream_t stream);

/* mrg_generate with an explicit launch shape (NULL = automatic).  Bitwise the
 * same results for every valid cfg. */
mrg_status mrg_generate_ex(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t n,
                           mrg_dist dist, mrg_dtype dtype, double param, void* dev_out,
                           const mrg_launch_cfg* cfg, hipStream_t stream);

/* Host only: the launch shape mrg_generate_ex would use for these arguments
 * and `cfg` (NULL = automatic) with an output aligned to 256 bytes, written
 * to host struct `*resolved` (all zero for n = 0; arith 0 for MRG31k3p,
 * which has one arithmetic form).  Same argument checks and errors as
 * mrg_generate_ex, pointers aside; nothing is launched. */
mrg_status mrg_generate_plan(mrg_generator gen, size_t n_streams, uint64_t n, mrg_dist dist, mrg_dtype dtype,
                             double param, const mrg_launch_cfg* cfg, mrg_launch_cfg* resolved);

/* Save/restore (Section 2.2, saveRDS/readRDS example).  Byte format,
 * little-endian: "MRG3", u32 version = 1, u32 generator, u32 flags (bit 0:
 * a creator follows the streams), u64 n, n x 18 u32 (cur, start, sub),
 * [6 u32 creator].
 *
 * mrg_streams_export_size: bytes needed for n streams (+ creator).
 * mrg_streams_export: copies n device records to host memory `host_buf`
 * (capacity `cap` bytes), appends `creator` when non-NULL, sets *len, and
 * returns after `stream` has been synchronised.
 * mrg_streams_import: validates the whole buffer (magic, version, generator,
 * length, every state word below its modulus, no all-zero triple) and only
 * then copies its n records to `dev` (room for `n` records required) and,
 * when `creator` is non-NULL and the buffer holds one, restores it.  Returns
 * after the copy has completed.  *n_out (optional) receives the count. */
mrg_status mrg_streams_export_size(size_t n, int with_creator, size_t* bytes);
mrg_status mrg_streams_export(mrg_generator gen, const mrg_stream* dev, size_t n,
                              const mrg_creator* creator, void* host_buf, size_t cap, size_t* len,
                              hipStream_t stream);
mrg_status mrg_streams_import(mrg_generator gen, const void* host_buf, size_t len, mrg_stream* dev,
                              size_t n, size_t* n_out, mrg_creator* creator, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The paper's own kernel geometry (Listing 1 of Section 2.2, Listing 2 of
 * Section 3.1), for code that relies on where clrng puts each number.
 *
 * The output is an nrow x ncol block of a row-major buffer with row stride
 * npad (elements; npad >= ncol; the other npad - ncol columns are not
 * written).  A g0size x g1size lattice of work-items (clrng's Nglobal) covers
 * it: work-item (g0, g1) owns the cells (g0 + i*g0size, g1 + j*g1size),
 * visits them row by row (i ascending, then j ascending) and stores its next
 * value in each.  Its stream is number g0 + g0size*g1 for MRG_UNIFORM and
 * MRG_RAW (Listing 1) and g0*g1size + g1 for MRG_NORMAL and MRG_EXPONENTIAL
 * (Listing 2; the exponential matrix printed in Section 3.2 needs this
 * index).  Normals pair the work-items (g0, 2p) and (g0, 2p+1): each visit
 * takes U1 from the first one's stream and U2 from the second one's, X goes
 * to the first one's cell and Y to the second one's (Algorithm 1); g1size
 * and ncol must be even.  A vector is one row (nrow = 1), as in the printed
 * runifGpu example.
 *
 * Needs n_streams >= g0size*g1size; a stream advances by the number of
 * visits of its work-item and the others do not move.  Values and rounding
 * are those of mrg_generate (f32 uniforms round toward zero).  nrow, ncol
 * < 2^31; nrow == 0 or ncol == 0 is a no-op.
 * ------------------------------------------------------------------------ */
mrg_status mrg_generate_paper(mrg_generator gen, mrg_stream* dev, size_t n_streams, uint64_t nrow, uint64_t ncol,
                              uint64_t npad, uint32_t g0size, uint32_t g1size, mrg_dist dist, mrg_dtype dtype,
                              double param, void* dev_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * The Monte-Carlo Fisher test of Section 4: random contingency tables with
 * fixed margins, one stream per table.  Entries are drawn row by row in
 * row-major order, each by inversion of its hypergeometric distribution given
 * the entries before it, with one uniform of the table's stream: entry (i,j)
 * is the smallest x in [lo, hi] with u*W <= w(lo)+...+w(x), where w(lo) = 1,
 * w(x+1) = w(x)*((K-x)(n-x))/((x+1)(N'-K-n+x+1)) in double precision, n the
 * row's remaining total, K column j's remaining total, N' the units left in
 * columns j.. of rows i..; the last entry of each row and the last row are
 * determined.  A table uses (I-1)(J-1) steps of its stream, which advances.
 * The statistic of a table is -sum log(n_ij!), summed row-major.
 * ------------------------------------------------------------------------ */

/* n tables: table t has shape I[t] x J[t] (1..5 each), row totals
 * rows[5t..5t+I-1], column totals cols[5t..5t+J-1] (all device int32), and
 * uses stream t of `dev_streams`.  Writes tables[25t..25t+24] (5 x 5,
 * row-major, zero padded) and stats[t] (optional, may be NULL).  A table with
 * a shape out of range, a negative margin, unequal row and column sums or a
 * grand total above 2^20 gets zeros and a NaN statistic and does not advance
 * its stream. */
mrg_status mrg_tables_sample(mrg_generator gen, mrg_stream* dev_streams, size_t n, const int32_t* dev_I,
                             const int32_t* dev_J, const int32_t* dev_rows, const int32_t* dev_cols,
                             int32_t* dev_tables, double* dev_stats, hipStream_t stream);

/* fisher.sim (Section 4): B replicates of the margins of `observed` (host,
 * I x J row-major, 1 <= I, J <= 32, non-negative, grand total <= 2^20),
 * replicate b from stream b.  *dev_count (device) receives the number of
 * replicates whose statistic is <= observed / (1 + 64 eps) (ties counted as
 * stats::fisher.test does); stats (device, B entries, optional) the
 * replicates' statistics; *observed_stat (host, optional) the observed one.
 * The p-value is (1 + count) / (B + 1) (mrg_fisher_pvalue).  Asynchronous;
 * no memset, so it may be captured in a graph. */
mrg_status mrg_fisher_sim(mrg_generator gen, mrg_stream* dev_streams, uint64_t B, int I, int J,
                          const int32_t* observed, uint64_t* dev_count, double* dev_stats,
                          double* observed_stat, hipStream_t stream);
double     mrg_fisher_pvalue(uint64_t count, uint64_t B);

/* ------------------------------------------------------------------------
 * Diagnostics.  Neither call reads or changes any stream.
 * ------------------------------------------------------------------------ */

/* Functions mrg_transform_accuracy checks.  The normal (Algorithm 1 of
 * Section 3.1) and exponential (Section 3.2) transforms evaluate them with the
 * library's own code, which leaves out the range reduction and special cases
 * of the general functions (a uniform lies in [2^-33, 1) and is never zero,
 * subnormal or non-finite).  Draws stored as MRG_F32 use shorter evaluations
 * of the same functions (the _F32OUT entries: about 1e-7 relative, since the
 * result is rounded to float). */
typedef enum {
    MRG_CHECK_LOG = 0,    /* log(u), u = z/(m1+1): exponential draws, Box-Muller radius */
    MRG_CHECK_SQRT = 1,   /* sqrt(x), x = -2 log(u): the Box-Muller radius R          */
    MRG_CHECK_SINPI = 2,  /* sin(pi t), t = 2u: the Box-Muller angle                   */
    MRG_CHECK_COSPI = 3,  /* cos(pi t), t = 2u                                         */
    MRG_CHECK_LOG_F32OUT = 4,    /* the same four, as the fp32 outputs evaluate them */
    MRG_CHECK_SQRT_F32OUT = 5,
    MRG_CHECK_SINPI_F32OUT = 6,
    MRG_CHECK_COSPI_F32OUT = 7
} mrg_check_fn;

/* For every integer z in [z_begin, z_end), the generator output a step can
 * produce (1 <= z_begin <= z_end <= m1 + 1), evaluate function `fn` at the
 * input that z gives the transforms, once with the library's code and once
 * with the HIP device math library (log, sqrt, sincospi; the square root
 * checks feed both the library's full-precision -2 log(u)), and count how
 * many doubles apart the two results are (a relative error e is about
 * e * 2^52 to e * 2^53 doubles).  dev_result (device, 8 uint64, 8-byte aligned) receives:
 * [0]..[3] the number of inputs 0, 1, 2, 3 apart, [4] 4 or more apart,
 * [5] (largest distance << 32) | the largest z at that distance (distance
 * capped at 2^32 - 1), [6] and [7] zero.  The call clears dev_result itself
 * with a kernel (no memset).  Asynchronous on `stream`. */
mrg_status mrg_transform_accuracy(mrg_generator gen, mrg_check_fn fn, uint64_t z_begin, uint64_t z_end,
                                  uint64_t* dev_result, hipStream_t stream);

/* Store-only ceiling of mrg_generate: writes 0.5 into the n elements of
 * dev_out (MRG_F64 or MRG_F32, aligned to its element size) with exactly the
 * store pattern of mrg_generate for MRG_UNIFORM draws of that dtype from
 * n_streams streams -- the same grid, per-lane store width, row order,
 * per-row barriers and cache policy -- and computes nothing else.  Its time
 * is what that write layout allows by itself.  n must be a multiple of
 * n_streams (whole rows).  Asynchronous on `stream`. */
mrg_status mrg_store_ceiling(size_t n_streams, uint64_t n, mrg_dtype dtype, void* dev_out, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batching: many generation requests of uneven lengths, each on its own
 * streams, in one persistent launch (graph-capturable).  Every request gives
 * exactly the numbers and final states that mrg_generate would give for it.
 * The paper launches once per call with a fixed work-item grid (Section 2.2);
 * batching is this library's own extension of that call.
 * ------------------------------------------------------------------------ */

/* One request: as the arguments of mrg_generate.  `streams` (device, room for
 * n_streams records) and `out` (device, n elements) belong to the caller;
 * different requests of one plan must not share stream records or output
 * bytes. */
typedef struct {
    mrg_stream* streams;
    uint32_t n_streams;
    uint64_t n;
    mrg_dist dist;
    mrg_dtype dtype;
    double param;
    void* out;
} mrg_request;

/* Batch launch shape (0 = automatic for every field).  Results never depend
 * on it.
 *   tile_units      most draws (normal: pairs) one wave makes in one tile
 *   waves_per_simd  waves per SIMD of the persistent grid (1..16), capped at
 *                   what the kernel's registers allow to be resident at once
 *   wide_stores     1 = one stream per lane; 2 = stores up to 16 bytes
 *                   wide (several streams per lane) where a request allows,
 *                   unless a narrower width leaves fewer lanes idle;
 *                   0 = automatic: 1 in gang mode, 2 otherwise.  In gang
 *                   mode a plan of one-stream tiles runs a kernel holding
 *                   only their code, which fits up to six waves per SIMD
 *                   (the kernel with every width fits three)
 *   gang_waves      1 = every wave takes tiles on its own, from one queue per
 *                   class (normal, exponential, uniform/raw); 2, 4 or 8 = a
 *                   block of that many waves takes a gang of that many tiles
 *                   -- neighbouring stream blocks of one request -- and its
 *                   waves write rows together (a barrier every three rows), from
 *                   one queue that interleaves the classes              */
typedef struct {
    uint32_t tile_units;
    uint32_t waves_per_simd;
    uint32_t wide_stores;
    uint32_t gang_waves;
} mrg_batch_cfg;

typedef struct mrg_batch_plan mrg_batch_plan;  /* opaque, owned by the library */

/* Host-only: validate the requests (as mrg_generate does, plus disjoint
 * stream ranges), cut them into tiles (request, block of 64 x SPL streams,
 * <= tile_units draw units) sorted by estimated cost, longest first. */
mrg_status mrg_batch_plan_create(mrg_generator gen, const mrg_request* reqs, size_t n_req,
                                 const mrg_batch_cfg* cfg, mrg_batch_plan** plan);
void       mrg_batch_plan_destroy(mrg_batch_plan* plan);

/* Device workspace the caller provides for a plan (256-byte aligned), and
 * the plan's tile count. */
mrg_status mrg_batch_workspace_size(const mrg_batch_plan* plan, size_t* bytes);
mrg_status mrg_batch_tile_count(const mrg_batch_plan* plan, size_t* tiles);

/* Copy the plan's static tables into `dev_workspace` (once per workspace and
 * plan; returns after the copy completed). */
mrg_status mrg_batch_upload(const mrg_batch_plan* plan, void* dev_workspace, hipStream_t stream);

/* Enqueue the batch on `stream`: a counter-reset kernel, the persistent
 * kernel and (when a request is split over chunks) a state-advance kernel.
 * No host synchronisation, no allocation, no memset: may be captured in a
 * hipGraph and replayed; one workspace serves one launch at a time. */
mrg_status mrg_batch_launch(const mrg_batch_plan* plan, void* dev_workspace, hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture
 * without an allocator, tight serving loops, harnesses that forbid hipMalloc):
 * mrg_batch_upload followed by mrg_batch_launch, with the workspace in a
 * static device array of the library (MRG_BATCH_STATIC_WORKSPACE_BYTES per
 * GPU, held until the process ends) instead of a caller buffer.  Enqueues on
 * `stream`, which must belong to the calling thread's current device: a copy
 * of the plan's tables into that array, then the launch.  The plan must stay
 * alive and unchanged until the launch has completed.  Allocates nothing
 * (no hipMalloc, hipFree, memset or allocating library call).  The array is
 * shared by every such call on a GPU and keeps the last call's contents (each
 * launch resets its own counters): calls that may overlap on one GPU race
 * and must be ordered by the caller (one stream, or events).
 * MRG_E_NOMEM when the plan's workspace (mrg_batch_workspace_size) exceeds
 * the array, checked before anything is enqueued. */
#define MRG_BATCH_STATIC_WORKSPACE_BYTES (16u << 20)
mrg_status mrg_batch_launch_static(const mrg_batch_plan* plan, hipStream_t stream);

/* After a launch has completed: host_ticks[0] = device real-time clock
 * (100 MHz) when the first tile was taken, host_ticks[1 + r] = when request r
 * finished storing its output (0 if it did not).  n_req + 1 entries.  Copies
 * and synchronises `stream`. */
mrg_status mrg_batch_request_times(const mrg_batch_plan* plan, const void* dev_workspace,
                                   uint64_t* host_ticks, hipStream_t stream);

/* Autotuner: time candidate shapes (tile_units in {192, 256, 512, ..., 8192}
 * x gang_waves in {1, 4, 8} x wide_stores in {1, 2} x waves_per_simd in
 * {2, 3, 4, 5, 6}; a waves setting that the kernel's registers cap to the grid of
 * the one before is skipped) of the plan on the GPU with its own requests,
 * in `dev_workspace` (capacity `workspace_bytes`; shapes whose workspace would
 * not fit are skipped: mrg_batch_autotune_workspace_size gives the capacity
 * that fits every candidate), keep
 * the fastest in the plan (re-cut and uploaded again) and report it in
 * `best` / `best_ms` (optional).  Every request's stream records are saved to
 * host memory first and restored at the end, so the streams are left as they
 * were; the outputs are overwritten.  Synchronises `stream`. */
mrg_status mrg_batch_autotune(mrg_batch_plan* plan, void* dev_workspace, size_t workspace_bytes,
                              hipStream_t stream, mrg_batch_cfg* best, double* best_ms);

/* Host only: the largest workspace any autotuner candidate of `plan` needs
 * (at least mrg_batch_workspace_size of the plan as it is). */
mrg_status mrg_batch_autotune_workspace_size(const mrg_batch_plan* plan, size_t* bytes);

/* ------------------------------------------------------------------------
 * Serving: a request loop over sessions whose stream state stays on the
 * device.  Section 2.1 keeps streams explicit and on the GPU so that
 * interrupted and restored sessions stay reproducible; the server keeps each
 * session's streams resident and assigns every request its position in the
 * session's sequence when it arrives.
 *
 *   - Session i owns streams_per_session streams created from `seed` (session
 *     i takes streams i*S .. i*S+S-1 of one creator).  A request of n draws
 *     on a session uses all its S streams: draw k of stream s is element
 *     k*S + s of the request's output, exactly as mrg_generate lays it out.
 *   - Positions are assigned at submission, in submission order: a request
 *     starts where the session's previous request ended, and advances every
 *     stream of the session by ceil(n/S) steps (normals: rounded up to even).
 *     Its numbers are those mrg_generate gives for the session's streams
 *     advanced to that position, whatever else is running.
 *   - Requests are admitted in submission order as output memory in the pool
 *     frees up, batched as they arrive into persistent launches (up to
 *     `lanes` of them in flight on separate HIP streams, overlapping on the
 *     device), and completed individually: the kernel flags each request in
 *     host-visible memory when its output is stored.
 *   - mode 1 replaces batching by one plain launch per request at admission,
 *     in submission order on one HIP stream (the comparison baseline).
 * Memory: the caller owns the device memory -- the output pool and a
 * workspace (mrg_server_workspace_size bytes, 256-byte aligned) that holds
 * the session stream records and one batch workspace per lane.  The library
 * allocates, in mrg_server_create and nowhere else, only pinned host memory
 * for the per-lane completion flags (host-visible, written by the kernels)
 * and table staging, plus HIP streams and events.
 * ------------------------------------------------------------------------ */

typedef struct {
    uint32_t n_sessions;
    uint32_t streams_per_session;  /* 0 = 64 */
    uint32_t seed[6];
    void* pool;                    /* device memory for request outputs (caller-owned) */
    size_t pool_bytes;
    uint32_t lanes;                /* launches in flight at once (0 = 4) */
    uint32_t max_batch;            /* requests per launch at most (0 = 256) */
    uint32_t mode;                 /* 0 = continuous batching, 1 = one plain launch per request */
    uint32_t tile_units;           /* 0 = 2048 */
    void* workspace;               /* device memory for session streams and lane workspaces
                                      (caller-owned, 256-byte aligned, not overlapping the pool) */
    size_t workspace_bytes;        /* at least mrg_server_workspace_size(cfg) */
} mrg_server_cfg;

typedef struct {
    uint64_t submitted, completed, released, rejected;
    uint64_t samples_completed;
    uint64_t launches;             /* batches (mode 0) or plain launches (mode 1) */
    uint64_t pool_in_use, pool_peak;
    uint64_t max_in_flight;        /* most requests on the device at once */
    uint64_t max_lanes_busy;       /* most lanes with a launch in flight at once (mode 0) */
} mrg_server_stats;

typedef struct mrg_server mrg_server;  /* opaque */

uint64_t   mrg_now_ns(void);           /* the steady clock the server uses */

/* Bytes of device workspace a server with this configuration needs (the
 * workspace fields of cfg are not read).  Host only. */
mrg_status mrg_server_workspace_size(const mrg_server_cfg* cfg, size_t* bytes);

/* Creates the session streams (in the workspace) and starts the scheduler
 * thread.  MRG_E_NOMEM when the workspace is smaller than
 * mrg_server_workspace_size; MRG_E_INVALID_ARG when the pool or workspace is
 * missing, misaligned or the two overlap. */
mrg_status mrg_server_create(const mrg_server_cfg* cfg, mrg_server** srv);
void       mrg_server_destroy(mrg_server* srv);  /* waits for work in flight */

/* Queue a request (thread-safe, never blocks on the GPU).  `t_arrival_ns`
 * (mrg_now_ns clock) is when the request arrived; latency is measured from
 * it.  MRG_E_NOMEM when the output alone exceeds the pool (nothing queued,
 * no position assigned).  *ticket identifies the request; *offset_out
 * (optional) receives its starting position in the session. */
mrg_status mrg_server_submit(mrg_server* srv, uint32_t session, uint64_t n, mrg_dist dist,
                             mrg_dtype dtype, double param, uint64_t t_arrival_ns, uint64_t* ticket,
                             uint64_t* offset_out);

/* Non-blocking query.  MRG_OK with *done = 1 once the output is in the
 * pool; then *dev_out points at it (n elements) and *t_done_ns is when the
 * server saw it complete.  MRG_E_BUSY with *done = 0 while the request is
 * queued or running (not an error: poll again). */
mrg_status mrg_server_poll(mrg_server* srv, uint64_t ticket, int* done, void** dev_out,
                           uint64_t* t_done_ns);

/* Give the output memory of a completed request back to the pool. */
mrg_status mrg_server_release(mrg_server* srv, uint64_t ticket);

/* Counters of the server so far (host struct).  The struct type already
 * carries the name mrg_server_stats, hence the _get. */
mrg_status mrg_server_stats_get(mrg_server* srv, mrg_server_stats* out);

/* Open-loop replay on the calling thread: request i (session[i], n_draws[i]
 * draws of dist/dtype/param) arrives t_arrival_ns[i] after the start; it is
 * submitted at that time, and released as soon as it completes.  Fills
 * latency_ns[i] (completion seen - arrival) and *span_ns (start to the last
 * completion).  Returns when every request has completed. */
mrg_status mrg_server_drive(mrg_server* srv, size_t n, const uint64_t* t_arrival_ns,
                            const uint32_t* session, const uint64_t* n_draws, mrg_dist dist,
                            mrg_dtype dtype, double param, uint64_t* latency_ns, uint64_t* span_ns);

#ifdef __cplusplus
}
#endif

#endif /* MRG355_H */
