/*
 * ebcc.h — C ABI of the EBCC GPU library (libebcc.so, HIP for gfx950).
 *
 * EBCC is the two-layer error-bounded compressor of arXiv 2510.22265: a
 * JPEG2000-style base layer (9/7 lifting DWT, dead-zone quantisation, EBCOT
 * tier-1 with the MQ coder, rate allocation to a base compression ratio r)
 * and a residual layer (DWT of input minus decoded base, SPIHT bit-plane
 * coding truncated at the first plane where every point meets the bound).
 * The operation is the problem statement of the paper's Algorithm 1 (EBCC
 * Compression Process): input a 2-D array, a max error target eps and a base
 * ratio; output a byte sequence that decodes with max|x - x_hat| <= eps.
 * Fields are float32 only (Implementation Details) and 2-D after flattening
 * (Method section, first paragraph).
 *
 * Conventions for every entry point:
 *  - Pointers prefixed d_ are device pointers (HBM of the current HIP
 *    device); h_ are host pointers.  The caller owns every buffer passed in.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; entry points that return a size or a status read it back and
 *    therefore synchronise that stream before returning (the asynchronous
 *    decoder leaves its statuses in device memory instead).
 *  - The library keeps per-device scratch workspaces and per-shape plans
 *    between calls (grown on demand, freed by ebcc_release).  Calls on
 *    different streams are safe to make from different host threads.
 *  - Return values are ebcc_status codes (0 = success, negative = error);
 *    ebcc_last_error() gives a human-readable detail for the calling thread.
 *  - Output streams are byte-identical to the CPU oracle's for the same
 *    input and parameters (the stream format is described with the design
 *    notes of this repository).
 */
#ifndef EBCC_H
#define EBCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EBCC_OK = 0,
  EBCC_EINVAL = -1,    /* bad argument, non-finite input, dims mismatch */
  EBCC_ENOSPC = -2,    /* output capacity too small; *out_len = size needed */
  EBCC_ECORRUPT = -3,  /* stream fails magic/version/length/checksum checks */
  EBCC_ENOMEM = -4,    /* device allocation failed */
  EBCC_EHIP = -5,      /* a HIP runtime call failed (see ebcc_last_error) */
  EBCC_ENOTIMPL = -6   /* a parameter value the library does not implement */
} ebcc_status;

enum { EBCC_BOUND_REL = 0, EBCC_BOUND_ABS = 1 };

/* Stream modes (byte 5 of the 48-byte header). */
enum { EBCC_MODE_CONST = 0, EBCC_MODE_RAW = 1, EBCC_MODE_CODED = 2 };

typedef struct {
  uint32_t struct_size;   /* sizeof(ebcc_params), for ABI versioning */
  uint32_t bound_mode;    /* EBCC_BOUND_REL: err_bound is a fraction of (max - min)
                             (range-relative, Benchmarks section); EBCC_BOUND_ABS: absolute */
  double err_bound;       /* > 0 and finite */
  double base_ratio;      /* r >= 1: header + base section <= floor(4 * ny * nx / r) bytes */
  double q;               /* 0: the base layer runs at base_ratio.  q in (0, 1]: Algorithm 1's
                             feedback search from r0 = base_ratio for the ratio at which the
                             proportion q of samples meets the bound in the base alone (the
                             paper uses 1 - 1e-5), plus its base-only fallback.  Else EINVAL. */
  uint32_t levels;        /* DWT levels (default 5), clamped to floor(log2(min(ny, nx))) */
  uint32_t cblk_log2w;    /* code-block width  = 2^cblk_log2w, 2..6 (default 5) */
  uint32_t cblk_log2h;    /* code-block height = 2^cblk_log2h, 2..6 (default 5); w*h <= 4096 */
  uint32_t spiht_tile;    /* SPIHT tile side in coarsest-LL roots, 1..64 (default 1) */
  uint32_t trunc;         /* residual truncation (Algorithm 1's second binary search): 0 = at the
                             end of a bit-plane (default); 1 = at a byte position of the tiles'
                             codes read as one embedded sequence (plane by plane, the sorting
                             passes of every tile before their refinement passes), searched
                             within the last plane the plane search keeps */
  uint32_t bypass;        /* tier-1 arithmetic-coding bypass (JPEG2000 Part 1, D.6, the "lazy"
                             mode): 0 = every coding pass MQ coded (default); 1 = the
                             significance-propagation and refinement passes after a block's
                             first ten send their decisions as raw bits (cleanup passes stay MQ
                             coded); a block's codeword after k > 10 passes is then u16 raw byte
                             count, MQ codeword, raw bits.  Any other value: EINVAL */
} ebcc_params;

/* Fill p with the defaults: range-relative 1% bound, r = 30, 5 levels,
 * 32x32 code-blocks, one-root SPIHT tiles, q = 0, truncation at plane ends,
 * no tier-1 bypass. */
void ebcc_params_default(ebcc_params* p);

/* Largest stream ebcc_compress can produce for an ny x nx field (a coded
 * stream never exceeds the raw one): 48 + 4 * ny * nx bytes. */
size_t ebcc_compress_bound(size_t ny, size_t nx);

/* Compress one float32 field.
 *   d_x      [ny][nx] row-major float32, device.  1 <= ny, nx <= 2^24,
 *            ny * nx < 2^31.  All values must be finite (else EBCC_EINVAL).
 *   p        parameters (host); NULL = defaults.
 *   d_out    device buffer of out_cap bytes receiving the stream.
 *   out_len  host: stream length on success, or the size needed on ENOSPC.
 * Synchronises `stream` (the truncation search reads back a few scalars and
 * the final length). */
int ebcc_compress(const float* d_x, size_t ny, size_t nx, const ebcc_params* p,
                  uint8_t* d_out, size_t out_cap, size_t* out_len, void* stream);

/* Decompress one stream (device bytes d_in[0..in_len)) into d_x [ny][nx]
 * float32.  ny, nx must match the stream header (else EBCC_EINVAL).  Corrupt
 * streams return EBCC_ECORRUPT (the output is then unspecified).
 * Synchronises `stream`. */
int ebcc_decompress(const uint8_t* d_in, size_t in_len, float* d_x, size_t ny, size_t nx,
                    void* stream);

/* ---------------------------------------------------------------------------
 * Batched execution.  A climate dataset is many 2-D fields of uneven sizes
 * (the paper compresses each variable/level slice independently; Benchmarks
 * section), and one small field does not fill the GPU.  These entry points
 * run every stage of the pipeline once over all fields of the batch: one
 * launch per stage covers every field's code-blocks, SPIHT tiles and DWT
 * tiles, and the per-field truncation searches of Algorithm 1 advance in
 * lockstep (one launch and one read-back per search round for the batch).
 * Each field's stream is byte-identical to what ebcc_compress /
 * ebcc_decompress produce for it alone.  Large batches are processed in
 * chunks of at most 2^27 samples or 4096 fields.
 * ------------------------------------------------------------------------- */

/* Compress n fields.
 *   d_x[i]        device pointer of field i, [ny[i]][nx[i]] float32 (host
 *                 arrays d_x, ny, nx of n entries).
 *   err_bounds    host [n]: per-field error bound (same bound_mode), or NULL
 *                 for p->err_bound for every field.
 *   p             shared parameters (host); NULL = defaults.
 *   d_out         device buffer of out_cap bytes; the streams are written
 *                 back to back in field order.
 *   h_offsets, h_lengths  host [n]: byte offset in d_out and length of each
 *                 stream.
 *   h_status      host [n] (may be NULL): each field's status.  A field
 *                 whose arguments are invalid or whose input is not finite
 *                 gets EBCC_EINVAL there and no stream (length 0); the other
 *                 fields are still compressed and their streams are the same
 *                 as without it.
 * Returns the first error (EBCC_OK if every field was compressed).
 * out_cap >= sum of ebcc_compress_bound(ny[i], nx[i]) always suffices; a
 * smaller buffer may fail with EBCC_ENOSPC after earlier chunks were
 * written.  Synchronises `stream`. */
int ebcc_compress_batch(int n, const float* const* d_x, const size_t* ny, const size_t* nx,
                        const double* err_bounds, const ebcc_params* p, uint8_t* d_out,
                        size_t out_cap, uint64_t* h_offsets, uint64_t* h_lengths, int* h_status,
                        void* stream);

/* Decompress n streams: d_in[i] (device, in_len[i] bytes) into d_x[i]
 * [ny[i]][nx[i]] float32.  h_status (host [n], may be NULL) receives each
 * stream's status; a stream that is corrupt or does not match its size is
 * reported there and the others are still decoded.  Streams of different
 * code-block sizes may be mixed: the library decodes each code-block size
 * in its own launch sequence.  Returns the first error, or EBCC_OK.
 * Synchronises `stream`. */
int ebcc_decompress_batch(int n, const uint8_t* const* d_in, const size_t* in_len,
                          float* const* d_x, const size_t* ny, const size_t* nx, int* h_status,
                          void* stream);

/* Decompress n streams without waiting for the device (the decoder of
 * Algorithm 1's problem statement, batched): every step is enqueued on
 * `stream` and the call returns; stream offsets, lengths and the per-stream
 * statuses stay in device memory.  The host knows the streams' shapes and
 * the parameters they were coded with, not their bytes.
 *   d_in          device buffer holding the streams.
 *   d_offsets, d_lengths  device [n]: stream i is d_in[d_offsets[i] ..
 *                 + d_lengths[i]); each such range must lie inside the
 *                 caller's allocation (the lengths written by a batched
 *                 compression, for instance).
 *   d_x, ny, nx   host [n]: device pointer and shape of output field i.
 *   p             the parameters the streams were coded with (host; NULL =
 *                 defaults): levels, cblk_log2w/h and spiht_tile must be
 *                 those of every coded stream; trunc = 1 and bypass = 1
 *                 allow streams with byte-cut residuals and with the tier-1
 *                 bypass (streams without them decode too); the other
 *                 fields are not used.
 *   d_status      device int32 [n]: set, when the work has run, to each
 *                 stream's status: EBCC_OK, EBCC_ECORRUPT (the checks of
 *                 ebcc_decompress_batch: header, lengths, tables, checksum)
 *                 or EBCC_EINVAL (shape not the stream's, or coding
 *                 parameters other than p's).  A stream that fails the
 *                 header checks leaves its output untouched; one found
 *                 corrupt by its tables or checksum has been decoded all the
 *                 same (its output is meaningless); the others decode.
 * Returns EBCC_EINVAL for bad arguments (NULL arrays, shapes out of range,
 * invalid p) before anything is enqueued, EBCC_ENOMEM / EBCC_EHIP when
 * enqueuing fails (the statuses of streams not yet enqueued then stay
 * unwritten), EBCC_OK otherwise.  Does not synchronise `stream`: the inputs
 * must stay unchanged and the outputs and statuses must not be read until
 * the stream has reached this point.  A call may wait for an earlier
 * call's table uploads (at most four calls' uploads are in flight per
 * stream), and waits when its stream's workspace has to grow. */
int ebcc_decompress_batch_async(int n, const uint8_t* d_in, const uint64_t* d_offsets,
                                const uint64_t* d_lengths, float* const* d_x, const size_t* ny,
                                const size_t* nx, const ebcc_params* p, int32_t* d_status,
                                void* stream);

/* Compress one float32 field without allocating: for callers that cannot
 * allocate memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same arguments, results and stream
 * bytes as ebcc_compress; the call's workspace is a static device array of
 * the library, 256 MiB on each device the library runs on (held until the
 * process ends), instead of an allocated one.  It calls no device or pinned
 * host allocation: host tables reach the device as kernel arguments (no
 * staging buffer), every stage runs on `stream` (no extra streams or
 * events), and the per-shape tables are written into the scratch by each
 * call.
 *   - A field whose workspace does not fit in the array fails with
 *     EBCC_EINVAL before any work is queued (fields up to 721 x 1440 at the
 *     default parameters fit; the truncation search then evaluates fewer
 *     bisection levels per round, with the same result).
 *   - Every call on a device shares that device's array and leaves its
 *     contents behind; a call rewrites everything it reads.  Calls are
 *     serialised by a host lock per device and each returns only after its
 *     stream has drained, so they do not overlap.  A caller that touches
 *     the array by other means while a call runs would race with it.
 * Synchronises `stream`. */
int ebcc_compress_noalloc(const float* d_x, size_t ny, size_t nx, const ebcc_params* p,
                          uint8_t* d_out, size_t out_cap, size_t* out_len, void* stream);

/* ---------------------------------------------------------------------------
 * Device memory.  The library keeps one workspace per (device, stream),
 * grown on demand by a call and reused by the next calls on that stream, and
 * small per-shape tables (plans).  These queries let a caller that budgets
 * HBM (a serving loop) know and bound what the library takes.  No device
 * memory is touched by the size queries.
 * ------------------------------------------------------------------------- */

/* Device bytes one ebcc_compress call of an ny x nx field with parameters p
 * (NULL = defaults) allocates at most: its workspace (search candidates
 * included) plus the shape's plan tables.  0 for invalid arguments.  A
 * decompression of the stream takes no more. */
size_t ebcc_workspace_size(size_t ny, size_t nx, const ebcc_params* p);

/* Workspace bytes one batched call allocates at most (the largest over its
 * internal chunks; plan tables not included):
 *   h_hdrs == NULL: ebcc_compress_batch of n fields [ny[i]][nx[i]] with p;
 *   h_hdrs != NULL: ebcc_decompress_batch of n streams whose first 48 bytes
 *                   are h_hdrs[48*i .. 48*i+47] (host) and whose lengths are
 *                   in_len[i], into fields [ny[i]][nx[i]] (p is not used).
 * 0 for invalid arguments. */
size_t ebcc_workspace_size_batch(int n, const size_t* ny, const size_t* nx, const ebcc_params* p,
                                 const uint8_t* h_hdrs, const size_t* in_len);

/* Make the workspace of `stream` on the current device exactly `bytes` now
 * (0 frees it): calls whose workspace fits then allocate nothing, a call
 * that needs more grows it again.  EBCC_ENOMEM if the allocation fails.
 * Synchronises `stream` if an existing workspace is replaced. */
int ebcc_workspace_reserve(size_t bytes, void* stream);

/* Device bytes the library holds on the current device: every stream's
 * workspace and the plan tables. */
size_t ebcc_device_bytes(void);

/* Header fields of a stream, read from host memory (the first 48 bytes). */
int ebcc_stream_info(const uint8_t* h_hdr, size_t len, size_t* ny, size_t* nx, int* mode);

/* Free the calling process's cached plans and workspaces on the current
 * device (the next call re-creates them). */
void ebcc_release(void);

const char* ebcc_status_str(int status);
/* Detail of the last error raised on the calling host thread ("" if none). */
const char* ebcc_last_error(void);

/* ---------------------------------------------------------------------------
 * Stage trace (for stage-by-stage comparison with the CPU oracle).
 * Runs ebcc_compress and copies intermediate device results into the given
 * device buffers (any may be NULL):
 *   d_coef  [ny*nx] f32  forward DWT of the normalised field
 *   d_abase [ny*nx] f32  base-layer reconstruction (normalised domain)
 *   d_cres  [ny*nx] f32  forward DWT of the residual
 *   d_kb    [nblocks] u8 coding passes kept per code-block
 *   d_pb    [nblocks] u8 magnitude bit-planes per code-block
 *   h_info  [11] i32 (host): mode, levels, e0, e_r, n_max, n_s, nblocks,
 *           ntiles, base_bytes, resid_bytes, feasibility checks
 * ------------------------------------------------------------------------- */
int ebcc_compress_trace(const float* d_x, size_t ny, size_t nx, const ebcc_params* p,
                        uint8_t* d_out, size_t out_cap, size_t* out_len, void* stream,
                        float* d_coef, float* d_abase, float* d_cres, uint8_t* d_kb,
                        uint8_t* d_pb, int32_t* h_info);

/* ---------------------------------------------------------------------------
 * Stage profiling.  When enabled, every call records HIP events on its
 * stream at stage boundaries (base DWT, tier-1 encode, rate allocation, ...)
 * and adds each stage's device time to process-wide accumulators.  A call
 * only records its events; they are read once the device has passed them
 * (at a later call, or in ebcc_profile_read / ebcc_profile_enable, which
 * wait for the outstanding ones), so profiling adds no synchronisation.
 *   ebcc_profile_enable(on)   enable/disable and reset the accumulators
 *   ebcc_profile_read(ms, calls, n)  copy up to n stage totals (milliseconds,
 *                             number of timed occurrences); returns the
 *                             number of stages
 *   ebcc_profile_stage_name(i)  the stage's name (static string)
 * ------------------------------------------------------------------------- */
void ebcc_profile_enable(int on);
int ebcc_profile_read(double* ms, long* calls, int n);
const char* ebcc_profile_stage_name(int i);

/* ---------------------------------------------------------------------------
 * Kernel tuning (process-wide).  These choices never change a stream: every
 * kernel variant produces the same bytes; they only trade latency for
 * throughput.  The autotuner of the Python package measures them (with the
 * code-block size and SPIHT tile, which do change the stream) on a sample of
 * the caller's fields.
 *   t1_encoder, t1_decoder  0 = by work size, 1 = one wavefront per
 *                           code-block (latency), 2 = several code-blocks per
 *                           wavefront, one per lane (throughput)
 *   t1_wave_max             by work size: one wavefront per code-block up to
 *                           this many code-blocks in a launch, lanes beyond
 *   spiht                   0 = SPIHT tiles in LDS (by capacity class, the
 *                           largest tiles with global-memory lists), 1 =
 *                           global-memory lists for every tile
 *   t1_lanes                lanes-per-block coders: code-blocks per
 *                           wavefront, 0 = by work size, or 1, 4, 16, 64
 *   t1_split                percent (0..100, default 10) of a lanes-per-block
 *                           encoder launch's code-blocks given to the
 *                           wave-per-block coder on a second stream (scalar
 *                           and vector units then work at the same time);
 *                           not used by persistent launches
 *   t1_persist              1 (default) = lanes-per-block coders as one
 *                           persistent launch: code-blocks ordered by the
 *                           bit-planes they code (most first), workgroups the
 *                           device keeps resident taking groups of them from
 *                           a work counter until none is left; 0 = one
 *                           workgroup per group of blocks in block order
 * ebcc_tuning_set returns EBCC_EINVAL for out-of-range values.
 * ------------------------------------------------------------------------- */
typedef struct {
  uint32_t struct_size;   /* sizeof(ebcc_tuning) */
  int32_t t1_encoder;
  int32_t t1_decoder;
  int32_t t1_wave_max;
  int32_t spiht;
  int32_t t1_lanes;
  int32_t t1_split;
  int32_t t1_persist;
} ebcc_tuning;
int ebcc_tuning_get(ebcc_tuning* t);
int ebcc_tuning_set(const ebcc_tuning* t);

#ifdef __cplusplus
}
#endif
#endif /* EBCC_H */
