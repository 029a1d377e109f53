/*
 * polarscs.h -- C-ABI of the MI355X (gfx950) successive-cancellation stack decoder.
 *
 * Polar codes PC(N, K) and their SCS decoding as in H. Aurora, W. Gross, "Towards
 * Practical Software Stack Decoding of Polar Codes" (Section 2.1 for the code, Section
 * 2.2 for SC / SCS decoding, Section 3 for the tree memory and the reduced-memory stack
 * scheme).  Plain pointers and sizes only; no framework types cross this boundary.
 *
 * Conventions shared by every call
 *   - Bits are uint8_t values 0 or 1, one per byte.
 *   - N = 2^n with 2 <= N <= 2048.  K counts every information position, CRC bits
 *     included; the first K - crc_bits information positions (ascending index) carry
 *     the payload and the last crc_bits carry the CRC remainder, most significant bit
 *     first.
 *   - CRC: crc_bits is 0 or 16; CRC-16 with polynomial 0x1021, initial register 0, bits
 *     most significant first, no reflection, no final xor (check value 0x31C3 over the
 *     ASCII string "123456789").
 *   - Return value: POLAR_OK (0) or a negative POLAR_E* code.  Argument errors are
 *     detected on the host before anything is enqueued, and nothing is written then.
 *   - Device pointers must be valid for the device of the context (or the current
 *     device for calls without a context) and stay alive until the stream reaches the
 *     enqueued work.  The caller owns every buffer it passes.
 */
#ifndef POLARSCS_H
#define POLARSCS_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
  POLAR_OK = 0,
  POLAR_EINVAL = -1,       /* invalid argument */
  POLAR_ENOMEM = -2,       /* host or device allocation failed */
  POLAR_EDEVICE = -3,      /* a HIP runtime call failed */
  POLAR_EUNSUPPORTED = -4, /* valid request outside what the library supports */
  POLAR_ETOOLARGE = -5     /* request beyond a fixed capacity (scs_decode_mixed_noalloc) */
};

/* Per-frame status bits written by the decoders. */
enum {
  SCS_STATUS_OK = 1,        /* output path passed the CRC (or there is no CRC) */
  SCS_STATUS_FALLBACK = 2,  /* every complete path failed the CRC; the first one is output */
  SCS_STATUS_EXHAUSTED = 4  /* decoding stopped because the stack emptied */
  /* a status byte of 0: the safeguard bound was reached (L N + L + 1 searches of the stack,
   * each followed by at most N + 1 extensions; the L counters keep every search far below
   * it, so it is not expected); payload unspecified */
};

/* LLR element types. */
enum { SCS_LLR_F32 = 0, SCS_LLR_I8 = 1 };

/* -- code construction (Section 2.1) ------------------------------------------------ */

typedef struct polar_code polar_code; /* opaque, host-owned, immutable once built */

/* Build PC(N, K): the information set is the K synthetic channels with the smallest
 * Bhattacharyya parameter for BPSK on AWGN at design_ebn0_db with rate K / N
 * (z0 = exp(-R Eb/N0); the f child of z is 2z - z^2, the g child is z^2; the first
 * split is the most significant bit of the index; ties go to the larger index).  The
 * paper takes its set from the 3GPP sequence; this construction stands in for it.
 * crc_bits: 0 or 16, counted inside K (K > crc_bits).  On success *out receives a new
 * code released with polar_code_free.  Errors: POLAR_EINVAL for N not a power of two in
 * [2, 2048], K outside [1, N], crc_bits not 0/16 or >= K, or a NULL out. */
int polar_construct(int32_t N, int32_t K, int32_t crc_bits, double design_ebn0_db,
                    polar_code** out);

/* Build PC(N, K) from an explicit information set (for example the paper's, taken from the
 * 3GPP reliability order, Section 5): info_mask holds N bytes, 1 for an information
 * position and 0 for a frozen one; K is their count and includes crc_bits (0 or 16), whose
 * bits are the last crc_bits information positions.  Errors: POLAR_EINVAL for N not a
 * power of two in [2, 2048], a NULL pointer, a mask byte other than 0 / 1, K < 1 or
 * crc_bits >= K. */
int polar_construct_set(int32_t N, const uint8_t* info_mask, int32_t crc_bits,
                        polar_code** out);

/* A systematic twin of `code` (Section 2.2.2, last paragraph; Section 4): the same N, K,
 * information set and CRC, but the encoders put the message (payload, then CRC) into the
 * codeword itself at the information positions (two passes of the transform: message at
 * the information positions of v, u = v F^(x)n cleared at the frozen positions, c =
 * u F^(x)n), and every decoder checks the CRC on, and reads the payload from, the
 * estimated codeword at the information positions.  The decoders' search itself is
 * unchanged.  On success *out receives a new code released with polar_code_free.
 * Errors: POLAR_EINVAL for NULL arguments; POLAR_EUNSUPPORTED when the two-pass encoder
 * does not show every message at this information set (checked on the unit messages; a
 * set with a frozen index between two information indices in the bit-subset order may
 * fail, constructed sets never do). */
int polar_code_systematic(const polar_code* code, polar_code** out);

/* 1 for a systematic code, 0 otherwise; POLAR_EINVAL for NULL. */
int polar_code_is_systematic(const polar_code* code);

/* Read back the parameters; any output pointer may be NULL.  info_mask_or_null, if
 * given, receives N bytes: 1 for an information position, 0 for a frozen one. */
int polar_code_query(const polar_code* code, int32_t* N, int32_t* K, int32_t* crc_bits,
                     uint8_t* info_mask_or_null);

void polar_code_free(polar_code* code);

/* -- encoding (Section 2.1: u at the information set, zeros elsewhere, c = u F^(x)n) -- */

/* Host encoder.  payload: B x (K - crc_bits) bits, row-major; codeword: B x N bits,
 * row-major.  The CRC remainder of each payload is appended when crc_bits = 16.  A
 * systematic code (polar_code_systematic) is encoded systematically. */
int polar_encode(const polar_code* code, const uint8_t* payload, uint8_t* codeword,
                 int64_t B);

/* Device encoder with the same layout and result, enqueued on hip_stream (a
 * hipStream_t; NULL = the default stream) of the current device.  Allocates nothing; the
 * code's tables travel as kernel arguments. */
int polar_encode_device(const polar_code* code, const uint8_t* payload_dev,
                        uint8_t* codeword_dev, int64_t B, void* hip_stream);

/* -- SCS decoding (Section 2.2.5; reduced-memory stack of Section 3.3) -------------- */

typedef struct scs_ctx scs_ctx; /* per-device decoder context */

/* Create a context on HIP device `device`.  It owns the device-side code tables and frame
 * descriptors of mixed batches, their work counter and a pinned staging buffer; after
 * creation it allocates only when a mixed batch needs more table space than any earlier
 * one.  Errors: POLAR_EINVAL for a bad device, POLAR_EDEVICE if HIP fails. */
int scs_ctx_create(int device, scs_ctx** out);
void scs_ctx_destroy(scs_ctx* ctx);

/* Wavefronts per workgroup of the decoder launches: 1, 2 or 4, or 0 for the library's
 * choice (4, fewer when their LDS state would exceed 64 KB).  A launch never uses more
 * than fit.  Results do not depend on this setting.  Errors: POLAR_EINVAL otherwise. */
int scs_ctx_set_waves_per_block(scs_ctx* ctx, int32_t waves_per_block);

/* Compute units' worth of workgroups a persistent mixed launch of this context takes (the
 * grid is this many CUs times the workgroups one CU holds): 0 = every CU of the device (the
 * default), else 1 .. the device's CU count.  Several contexts whose launches share the GPU
 * (a server's slots, one stream each) can each take a part, so that one batch's last
 * frames do not leave the rest of the GPU to wait for the next launch.  Results do not
 * depend on this setting.  Errors: POLAR_EINVAL for a negative value or one above the
 * device's CU count. */
int scs_ctx_set_grid_cus(scs_ctx* ctx, int32_t cus);

/* Per-frame counters (optional output of the decoders), one record per frame. */
typedef struct {
  uint32_t iterations;  /* leaf estimates (path extensions) */
  uint32_t switches;    /* extensions whose path was not the one held in the tree */
  uint32_t completions; /* length-N paths taken off the stack */
  uint32_t sc_elems;    /* sum of 2^(tz(i)+1) - 1 over extensions at i > 0, N - 1 at i = 0 */
  uint32_t fg_elems;    /* f/g element evaluations actually performed by the kernel */
  uint32_t evictions;   /* worst paths replaced in a full stack */
  uint32_t drops;       /* children discarded by a full stack */
  uint32_t prunes;      /* L-counter prune events */
} scs_stats;

/* Decode n_frames frames of one code with stack depth D and list parameter L.
 *
 * Per frame the decoder runs the stack search of Section 2.2.5: the best path (key:
 * path metric ascending, length descending, creation order ascending) is extended by
 * one leaf estimate (eq. llrcalc / scest), an information bit yields the hard-decision
 * child and the flipped child (eq. PMupd), a full stack keeps the D best paths, and
 * after L extensions at one length every path that short or shorter is dropped.  A
 * complete path is output if it passes the CRC; after L failures (or an empty stack)
 * the first complete path is output with SCS_STATUS_FALLBACK.
 *
 *   llr_dtype   SCS_LLR_F32: float LLRs, binary32 tree arithmetic;
 *               SCS_LLR_I8 : int8 LLRs in [-127, 127], saturating int8 tree, int16
 *                            saturating path metric.
 *   llr_dev     n_frames x N elements, row-major (frame f at f * N).
 *   payload_dev n_frames x (K - crc_bits) output bits, row-major.
 *   status_dev  n_frames status bytes (SCS_STATUS_*).
 *   stats_dev   NULL, or n_frames scs_stats records.
 *   D in [1, 256] (up to 64 slots per 64-lane bank of the stack), L in [1, 255].
 * Enqueued on hip_stream of the context's device; returns before the work runs.  The
 * result of a frame depends only on that frame's LLRs and (code, D, L).  Non-finite
 * LLRs give an unspecified output but the kernel still terminates (a frame makes at most
 * L N extensions and L completions; a safeguard bound stops it in any case). */
int scs_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t D, int32_t L,
                     int32_t llr_dtype, const void* llr_dev, int64_t n_frames,
                     uint8_t* payload_dev, uint8_t* status_dev, scs_stats* stats_dev,
                     void* hip_stream);

/* One frame of a mixed batch. */
typedef struct {
  int32_t code;    /* index into the codes array */
  int32_t D;       /* stack depth, [1, 64] in mixed batches */
  int32_t L;       /* list parameter, [1, 255] */
  int32_t _pad;    /* must be 0 */
  int64_t llr_off; /* element offset of the frame's N LLRs in llr_dev */
  int64_t out_off; /* byte offset of the frame's K - crc_bits payload bits */
} scs_frame;

/* Decode frames of different codes, depths and list sizes in one persistent launch.
 * frames_host: n_frames descriptors in host memory, validated on the host and copied with
 * the code tables into the context's device buffers on hip_stream.  Frame f writes
 * status_dev[f] and, if stats_dev is not NULL, stats_dev[f]; its payload goes to
 * payload_dev + out_off.  The result of every frame equals what scs_decode_batch gives for
 * it alone.  Equivalent to scs_mixed_prepare followed by scs_mixed_launch.  Errors:
 * POLAR_EINVAL for a bad code index, D, L, _pad, a negative offset or a NULL buffer;
 * POLAR_EUNSUPPORTED when one frame's decoder state would not fit 64 KB of LDS. */
int scs_decode_mixed(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                     const scs_frame* frames_host, int64_t n_frames, int32_t llr_dtype,
                     const void* llr_dev, uint8_t* payload_dev, uint8_t* status_dev,
                     scs_stats* stats_dev, void* hip_stream);

/* The two halves of scs_decode_mixed.  prepare validates and uploads a batch plan (it may
 * allocate, growing the context's buffers, and waits for the previous upload to finish);
 * launch enqueues the decoding of the prepared plan and neither allocates, copies nor
 * sets memory from the host, so a caller can capture it in a HIP graph and replay it while
 * the plan and the buffers stay the same.  The codes passed to prepare must outlive the
 * last launch of that plan.
 * Streams: a context holds one plan and one work counter.  Outside graph capture the
 * context orders its own mixed calls whatever streams they use: prepare and launch make
 * their stream wait (on the device) for the context's previous launch.  Launches captured
 * into a graph are not tracked: their replays must be ordered against the context's other
 * mixed calls by the caller (one stream, or events).  Contexts are independent. */
int scs_mixed_prepare(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                      const scs_frame* frames_host, int64_t n_frames, void* hip_stream);
int scs_mixed_launch(scs_ctx* ctx, int32_t llr_dtype, const void* llr_dev, uint8_t* payload_dev,
                     uint8_t* status_dev, scs_stats* stats_dev, void* hip_stream);

/* Fixed capacity of scs_decode_mixed_noalloc. */
#define SCS_NOALLOC_SCRATCH_BYTES (16u << 20) /* per device, held while the library is loaded */
#define SCS_NOALLOC_MAX_CODES 64

/* For callers that cannot allocate device memory (code under HIP graph capture of its own
 * stream work, tight serving loops, harnesses that forbid hipMalloc): scs_decode_mixed
 * without any allocation.  The batch plan -- work counter, the codes' tables and CRC
 * syndrome tables (64 N bytes per CRC code that a frame uses), and the n_frames
 * descriptors (24 bytes each) -- goes into one fixed array of SCS_NOALLOC_SCRATCH_BYTES that
 * the library keeps on every device it runs on, instead of buffers the context grows.  The
 * call makes no hipMalloc / hipFree and no host-side allocation; it copies the plan from host
 * memory with hipMemcpyAsync on hip_stream (pageable sources are read before the call
 * returns, after the stream's earlier work), zeroes the counter with a kernel and launches
 * the persistent decoder.  Frames are taken in descriptor order (scs_decode_mixed takes the
 * largest first); every frame's outputs equal what scs_decode_mixed gives.
 * Arguments, outputs and errors as scs_decode_mixed, plus: POLAR_ETOOLARGE when n_codes
 * exceeds SCS_NOALLOC_MAX_CODES or the plan exceeds SCS_NOALLOC_SCRATCH_BYTES (nothing is
 * enqueued then).  All calls on one device share its array and the last call's contents stay
 * there: calls that overlap on one device (other streams, other contexts, other threads)
 * race and must be ordered by the caller; calls on one stream are ordered by the stream. */
int scs_decode_mixed_noalloc(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                             const scs_frame* frames_host, int64_t n_frames, int32_t llr_dtype,
                             const void* llr_dev, uint8_t* payload_dev, uint8_t* status_dev,
                             scs_stats* stats_dev, void* hip_stream);

/* The fast simplified schedule of a code (Sections 2.2.2 and 3): nodes_out[N] receives,
 * for the first leaf i of every node, (class << 4) | lambda (the node covers leaves
 * [i, i + 2^lambda); classes 0 R-0, 1 R-1, 2 REP, 3 SPC) and 0xFF at every other position.
 * A block of leaves is one node when all its leaves are frozen (R-0), all carry information
 * (R-1), only its last leaf carries information (REP, 2 or more leaves) or only its first
 * leaf is frozen (SPC, 4 or more leaves); any other block is split in halves.
 * Errors: POLAR_EINVAL for NULL arguments. */
int polar_code_schedule(const polar_code* code, uint8_t* nodes_out);

/* Fast simplified stack decoding, FSSCS-RM (Section 4): the SCS search of scs_decode_batch
 * where one extension decodes a whole node of the schedule above and puts every candidate
 * of the node's list rule (Section 2.2.4) on the stack: R-0 one (all 0); REP two (all 0,
 * all 1); R-1 four (hard decisions, and flips of the one or two least reliable positions;
 * two for a single leaf); SPC eight (the flip patterns of the four least reliable positions
 * that give even parity).  A candidate's metric adds |alpha| of every position where it
 * differs from the hard decision.  Stack depth D, L counter (indexed by the node's first
 * leaf), CRC check, outputs, status bits and statistics as scs_decode_batch (iterations =
 * node extensions; a path switch = a winner that is not a candidate of the last
 * extension).  Errors: as scs_decode_batch; POLAR_EUNSUPPORTED when L times the candidates
 * of one pass over the schedule exceeds 2^20 - 2. */
int fsscs_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t D, int32_t L,
                       int32_t llr_dtype, const void* llr_dev, int64_t n_frames,
                       uint8_t* payload_dev, uint8_t* status_dev, scs_stats* stats_dev,
                       void* hip_stream);

/* CA-SCL decoding (Section 2.2.3): successive cancellation keeping a list of L paths (L = 1,
 * 2, 4 or 8).  At a frozen position every path takes 0 and its metric grows by |alpha| when
 * the hard decision is 1 (eq. PMupd); at an information position every path l (in list
 * order) offers u = 0 and u = 1 (candidate numbers 2 l and 2 l + 1), and the L candidates
 * with the smallest (metric, candidate number) form the new list in that order.  At the end
 * the paths are taken in ascending (metric, list position) and the first that passes the
 * CRC is the output (status SCS_STATUS_OK); if none passes, the first path with status
 * SCS_STATUS_FALLBACK.  Without a CRC the best path, status OK.  Buffers and statistics as
 * scs_decode_batch (iterations = path extensions, L per leaf once the list is full;
 * completions = CRC checks; the other counters 0).  At L <= 4 a wavefront decodes 8 / L
 * frames together; each frame's outputs do not depend on the other frames of the batch.
 * Errors: POLAR_EINVAL for another L or a bad argument; POLAR_EUNSUPPORTED when the LDS
 * state of one wavefront (eight list entries) would exceed 64 KB (it does not for
 * N <= 2048). */
int scl_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t L, int32_t llr_dtype,
                     const void* llr_dev, int64_t n_frames, uint8_t* payload_dev,
                     uint8_t* status_dev, scs_stats* stats_dev, void* hip_stream);

/* Last HIP error seen by a call on this context (POLAR_OK if none), then cleared. */
int scs_ctx_last_error(scs_ctx* ctx);

/* Text for a status code. */
const char* polar_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
