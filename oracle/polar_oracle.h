/*
 * polar_oracle.h -- plain CPU reference ("oracle") for polar-code construction,
 * encoding, SC, SCS, fast simplified stack (FSSCS-RM) and list (CA-SCL) decoding.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the HIP decoder.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links, loads or calls it, and the two share no code.
 *
 * Everything here is written to be read against the paper (Aurora & Gross, "Towards
 * Practical Software Stack Decoding of Polar Codes"): each function cites the passage
 * it implements.  Nothing is blocked, fused or reordered for speed.
 *
 * Conventions
 *   - bit vectors are arrays of uint8_t holding 0 or 1;
 *   - info_mask[i] = 1 iff i is in the information set A (|A| = K, CRC bits included);
 *   - the first K-r information positions (ascending) carry the payload, the last r
 *     carry the CRC-16 remainder, most significant bit first;
 *   - "mode" selects the arithmetic of the LLR tree: ORC_F32 (IEEE binary32, the
 *     paper's alpha type), ORC_F64 (binary64, for closed-form pins), ORC_FIX
 *     (saturating int8 LLRs with int16 path metrics).
 *   - return values: 0 ok, negative = invalid argument.
 */
#ifndef POLAR_ORACLE_H
#define POLAR_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1, ORC_FIX = 2 };

/* SCS status bits (same meaning as the library's). */
enum { ORC_ST_OK = 1, ORC_ST_FALLBACK = 2, ORC_ST_EXHAUSTED = 4 };

typedef struct {
  uint64_t iterations;   /* leaf estimates made (one per path extension) */
  uint64_t switches;     /* iterations whose winner was not the path held in alpha/beta memory */
  uint64_t completions;  /* length-N paths popped from the stack */
  uint64_t f_ops;        /* f evaluations performed (paper's schedule, root recompute on switch) */
  uint64_t g_ops;        /* g evaluations performed */
  uint64_t sc_elems;     /* sum over iterations of 2^(tz(i)+1)-1 (SC-schedule work, i>0), N-1 for i=0 */
  uint64_t evictions;    /* worst-path replacements in a full stack */
  uint64_t drops;        /* children discarded because the stack was full and they were worse */
  uint64_t prunes;       /* L-counter prune events */
} orc_stats;

/* Bhattacharyya construction (log domain) at design Eb/N0 with rate K/N; writes
 * info_mask[N].  Ties in the parameter go to the larger index. */
int orc_construct(int N, int K, double design_ebn0_db, uint8_t* info_mask);
/* Same, also returning the log-Bhattacharyya parameter of every synthetic channel. */
int orc_bhattacharyya_log(int N, double rate, double design_ebn0_db, double* lz);

/* CRC-16, polynomial 0x1021, init 0, MSB first, no reflection, no final xor,
 * over nbits bits (0/1 bytes). */
uint16_t orc_crc16_bits(const uint8_t* bits, int nbits);

/* c = u F^{(x)n} with F = [[1,0],[1,1]] (in-place XOR butterfly). */
int orc_polar_transform(int N, const uint8_t* u, uint8_t* c);
/* Build u from payload (+ CRC) and encode; payload[B][K-r] -> codeword[B][N]. */
int orc_encode_batch(int N, const uint8_t* info_mask, int crc_bits,
                     const uint8_t* payload, int64_t B, uint8_t* codeword);

/* SC decoding of one frame.  llr points to N values of the mode's input type
 * (float for F32, double for F64, int8_t for FIX).  Writes u_hat[N] and, if
 * leaf_llr is not NULL, the leaf LLR of every position as double. */
/* Systematic encoding of B payloads (Section 2.2.2, last paragraph; Section 4): the codeword
 * shows the message (payload, then CRC) at the information positions.  The decoders'
 * `systematic` flag checks the CRC on, and reads the payload from, the codeword estimate. */
int orc_encode_systematic_batch(int N, const uint8_t* info_mask, int crc_bits,
                                const uint8_t* payload, int64_t B, uint8_t* codeword);

int orc_sc_decode(int mode, int N, const uint8_t* info_mask, const void* llr,
                  uint8_t* u_hat, double* leaf_llr);

/* Leaf LLR alpha_(0,i) for an arbitrary decided prefix u[0..i-1], computed from the
 * root through the tree (populate beta, then alpha from the root). */
double orc_leaf_llr(int mode, int N, const void* llr, const uint8_t* prefix, int i);

/* SCS decoding of one frame with stack depth D, list parameter L, crc_bits 0 or 16.
 * Writes u_hat[N] (the output path), *status, optional stats, and *pm_out (the output
 * path's metric as double).  */
int orc_scs_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                   const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                   orc_stats* st, int systematic);

/* Batch helper: frames [B][N] -> payload[B][K-r], status[B], per-frame stats
 * (may be NULL; layout orc_stats[B]). */
int orc_scs_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int D,
                         int L, const void* llr, int64_t B, uint8_t* payload,
                         uint8_t* status, orc_stats* st, int systematic);

/* Fast simplified decoding (Sections 2.2.2, 2.2.4, 3 and 4).  Node classes: */
enum { ORC_NODE_R0 = 0, ORC_NODE_R1 = 1, ORC_NODE_REP = 2, ORC_NODE_SPC = 3 };
/* `types`: bit t allows class t above the leaves (0xF: all; 0: leaves only). */
#define ORC_TYPES_ALL 0xF

/* FSSC schedule: the nodes in decoding order (first leaf, lambda, class), at most
 * max_nodes written; returns the number of nodes. */
int orc_fssc_schedule(int N, const uint8_t* info_mask, int types, int32_t* start, int32_t* lam,
                      int32_t* type, int max_nodes);

/* FSSCL candidates of one node (class, lambda) with node LLRs alpha[2^lambda] (converted
 * to the mode's type) and path metric pm: writes each candidate's 2^lambda estimates and
 * its metric, in creation order; returns the number of candidates. */
int orc_node_candidates(int mode, int type, int lam, const double* alpha, double pm,
                        uint8_t* beta_out, double* pm_out, int max_out);

/* As orc_scs_decode / orc_fsscs_decode, and also the paths taken off the stack, in order:
 * creation number, length and metric of each (the first cap of them).  Returns the number
 * of paths taken (which may exceed cap), or -1 for bad arguments. */
int orc_scs_trace(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                  const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                  orc_stats* st, uint32_t* seq, int32_t* pl, double* pm, int cap,
                  int systematic);
int orc_fsscs_trace(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                    int types, const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                    orc_stats* st, uint32_t* seq, int32_t* pl, double* pm, int cap,
                    int systematic);

/* FSSCS-RM decoding of one frame (stack rules as orc_scs_decode, one iteration per node). */
int orc_fsscs_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                     int types, const void* llr, uint8_t* u_hat, uint8_t* status,
                     double* pm_out, orc_stats* st, int systematic);
int orc_fsscs_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int D,
                           int L, int types, const void* llr, int64_t B, uint8_t* payload,
                           uint8_t* status, orc_stats* st, int systematic);

/* CA-SCL decoding of one frame (Section 2.2.3): list size L, CRC selection among the final
 * paths (status OK, or FALLBACK when every path fails the CRC). */
int orc_scl_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int L,
                   const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                   orc_stats* st, int systematic);
int orc_scl_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int L,
                         const void* llr, int64_t B, uint8_t* payload, uint8_t* status,
                         orc_stats* st, int systematic);

/* Brute-force ML over all 2^K information words (K <= 20): discrepancy
 * disc(c) = sum_{j: c_j != HD(llr_j)} |llr_j| in binary64.  Returns the minimum in
 * *disc_min, the number of minimisers in *n_min, and writes each minimiser's
 * u (N bits) into minimisers[n][N] for the first max_out of them. */
int orc_ml_decode(int N, const uint8_t* info_mask, const double* llr, double* disc_min,
                  int64_t* n_min, uint8_t* minimisers, int64_t max_out);

#ifdef __cplusplus
}
#endif
#endif
