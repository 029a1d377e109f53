// Batched successive-cancellation stack (SCS) decoding of polar codes on gfx950.
//
// Method: Aurora & Gross, "Towards Practical Software Stack Decoding of Polar Codes",
// Section 2.2.5 (stack search, L-counter pruning, CRC termination), Section 2.2.1
// (min-sum f/g, eq. minsum; leaf decision, eq. scest; partial sums, eq. bitcalc) and the
// reduced-memory stack of Section 3.3 (one alpha/beta state, paths store only PM, PL and
// their decided bits; a path switch recomputes the tree).
//
// Mapping (one wavefront of 64 lanes decodes one frame):
//   * alpha tree in LDS: stage lambda (Lambda = 2^lambda values) at word offset
//     Lambda - 1.  Stages with Lambda >= 64 are computed 64 values per instruction (value
//     e in lane e mod 64; the top two stages, rebuilt from the channel LLRs, give each lane
//     consecutive values instead); stages with Lambda <= 32 run in one register with the
//     partner value from lane e xor Lambda (DPP / ds_swizzle / ds_bpermute).  The channel
//     LLRs (stage n) are read from the input.
//   * bit vectors (the decided bits of the path in the tree) are one VGPR: lane w holds
//     bits 32w..32w+31.  The partial sums a g-node needs are the transform of its left
//     sibling's decided bits, computed when the g-node is evaluated.
//   * the stack (scs_stack.h): slot s is lane s mod 64 of bank s / 64 (one bank for
//     D <= 64, up to four for D <= 256), holding one 64-bit key (path metric, then
//     N - PL and the creation number); the decided bits of slot s are word w in entry s
//     of lane w's private array.  Best / worst path = wave-wide min / max reductions
//     (DPP), free slots and pruning = ballots; the CRC is checked on a complete path from
//     a byte table of syndrome shares.
//   * a switch recomputes only the stages whose node differs between the path held in
//     the tree and the new path (lowest common ancestor of the two leaves, and the first
//     bit where their decisions differ); the values are identical to the paper's
//     recompute from the root because every alpha is a function of the channel LLRs and
//     the decided prefix only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "polar_code.h"
#include "polarscs.h"

#include "scs_device.h"
#include "scs_launch.h"

#include "scs_stack.h"
#include "scs_tree.h"

namespace {

// One frame, one wavefront.  `lds` is this wave's private region of
// scs_lds_words_per_wave(N, D) words.
// PERSISTENT: called once per frame inside the persistent loop of the mixed kernel, which
// inlines one copy per code length.
template <int LOGN, class TR, bool STATS, int NB = 1, bool PERSISTENT = false>
__device__ __forceinline__ void decode_frame(const CodeArgs& code, const FrameJob& job,
                                             uint32_t* lds) {
  using LY = Layout<LOGN>;
  constexpr int N = LY::N;
  constexpr int W = LY::W;
  int lane = lane_id();
  if constexpr (PERSISTENT) {
    // A value the compiler cannot see through (an empty asm statement, no instruction):
    // nothing derived from the lane number (masks, LDS addresses) is hoisted out of the
    // persistent loop, where it would stay live for every code length at once; this takes
    // the mixed kernel from 162 to 88 VGPRs.
    asm volatile("" : "+v"(lane));
    __builtin_assume(lane >= 0 && lane < kWave);
  }
  const int D = job.D, L = job.L;
  const bool use_crc = code.crc != 0;
  const typename TR::In* __restrict__ root = (const typename TR::In*)job.llr;
  // decided bits of slot s: word w in prow[s] of lane w.  Every access is by the lane
  // that owns the word, so the array is private to the lane (scratch memory, cached) and
  // needs no ordering across lanes; entry kRow takes the stores of lanes that must not
  // store.
  constexpr int kRow = 64 * NB;
  uint32_t prow[kRow + 1];
  // Every stored row is zero past its path's length (rows are written whole from a tree
  // path that is zero there, or gain a single 1 at the decided position), so a decision of
  // 0 needs no store.  The empty path's row starts at zero.
  prow[0] = 0u;
  uint32_t* cnt32 = lds;               // N bytes: extensions per length
  uint32_t* al = cnt32 + (N + 3) / 4;  // alpha stages 0 .. n-1 (0 .. n-2 without KEEP_TOP)
  uint32_t* dummy = al + LY::ALPHA_WORDS;  // kWave words: stores of lanes that must not store

  const uint32_t infow = lane < W ? code.info[lane] : 0u;
  for (int j = lane; j < (N + 3) / 4; j += kWave) cnt32[j] = 0u;
  lds_order();

  // stack: one key per slot; a path's length is N - (low word >> kSeqBits)
  PathStack<NB> S;
  S.init(D, make_key(0u, key_lo(N, 0, 0u)));
  uint32_t next_seq = 1;

  // The path extended next: slot p with key pk.  After an extension these are its first
  // child (which took over the slot), and that child is extended without a search whenever
  // its key is below lb, a lower bound on every other live key; kNone forces a search.
  int p = 0;
  uint64_t pk = kNone, lb = 0ull;
  // exact worst live key, kNone when unknown
  uint64_t maxk = kNone;
  int max_slot = 0;

  // the path held in the tree: its length when alpha was last computed, its decided bits
  int wl = -1;
  uint32_t ucur = 0u;
  // after an even leaf wl of the held path: leaf wl + 1's LLR for each value of bit wl, and
  // the value the first child took (its continuation then needs no tree work)
  uint32_t g0 = 0u, g1 = 0u, ulast = 0u;

  uint32_t fb = 0u, out = 0u;
  bool have_fb = false;
  int fails = 0;
  uint32_t st = 0u;
  uint32_t n_it = 0, n_sw = 0, n_cp = 0, n_sc = 0, n_fg = 0, n_ev = 0, n_dr = 0, n_pr = 0;

  // The L counters bound the search to L N extensions and L completions; as a safeguard
  // every stack search (at most N + 1 extensions follow one) spends one unit of a budget of
  // L N + L + 1, so every wavefront leaves the loop whatever its inputs.
  uint32_t budget = (uint32_t)L * (uint32_t)N + (uint32_t)L + 1u;
  for (;;) {
    // ---- the best path -------------------------------------------------------------
    bool cont = true;  // the first child of the last extension, with no search
    if (!(pk < lb)) {
      if (budget == 0u) {
        st = 0u;
        break;
      }
      --budget;
      if (S.empty()) {
        st = SCS_STATUS_FALLBACK | SCS_STATUS_EXHAUSTED;
        out = fb;
        break;
      }
      const uint64_t cand = pk;
      S.best(lane, p, pk, lb);
      cont = pk == cand;
    }
    // the slot stays live while the path is extended: its first child takes it over
    if (max_slot == p) maxk = kNone;
    const int i = N - (int)((uint32_t)pk >> kSeqBits);  // length of the best path

    if (i == N) {
      // a complete path: the CRC decides (Section 2.2.5)
      pk = kNone;
      S.kill(p);
      if constexpr (STATS) ++n_cp;
      const uint32_t row = lane < W ? prow[p] : 0u;
      if (!use_crc || crc_syndrome(code.crc_tab, row, lane, W, (N + 7) / 8) == 0u) {
        st = SCS_STATUS_OK;
        out = row;
        break;
      }
      if (!have_fb) {
        fb = row;
        have_fb = true;
      }
      if (++fails >= L) {
        st = SCS_STATUS_FALLBACK;
        out = fb;
        break;
      }
      continue;
    }

    // ---- extend path p by leaf i ---------------------------------------------------
    if constexpr (STATS) {
      ++n_it;
      n_sc += (i == 0) ? (uint32_t)(N - 1) : ((2u << __builtin_ctz((uint32_t)i)) - 1u);
    }
    // L counter of length i; lane 0 adds, the others add 0 to their dummy word
    const uint32_t old = atomicAdd(lane == 0 ? &cnt32[i >> 2] : &dummy[lane],
                                   lane == 0 ? (1u << (8 * (i & 3))) : 0u);

    int top;
    if (cont) {
      top = __builtin_ctz((uint32_t)i);  // the SC schedule continues (i = wl + 1 > 0)
    } else {
      if constexpr (STATS) ++n_sw;
      const uint32_t nu = lane < W ? prow[p] : 0u;
      int A = LOGN, d = 0;
      if (wl >= 0) {
        const int lim = wl < i ? wl : i;
        const uint32_t x = (ucur ^ nu) & prefix_mask(lane, lim);
        const uint64_t bx = ballot(x != 0u);
        if (bx == 0ull) {
          d = lim;
        } else {
          const int w = __builtin_ctzll(bx);
          d = w * 32 + __builtin_ctz(readlane(x, w));
        }
        A = (wl == i) ? 0 : msb((uint32_t)(wl ^ i)) + 1;
      }
      const int Bm = (d >= i) ? 0 : msb((uint32_t)(i ^ d)) + 1;
      top = (A > Bm ? A : Bm) - 1;
      if (top < 0) top = 0;
      ucur = nu & prefix_mask(lane, i);  // the tree path is zero past its length
    }
    uint32_t a0;
    if (cont && top == 0) {
      // odd leaf i = wl + 1 continuing: made with leaf wl (leaf_pair)
      a0 = ulast ? g1 : g0;
      if constexpr (STATS) ++n_fg;
    } else if (cont && top <= LY::SMALL) {
      a0 = cont_dispatch<0, LOGN, TR, STATS>(top, i, ucur, root, al, dummy, lane, n_fg, g0, g1);
    } else {
      if (top >= 6) big_stages<LOGN - 1, LOGN, TR, STATS>(top, i, ucur, root, al, lane, n_fg);
      a0 = small_stages<LOGN, TR, STATS>(top, i, ucur, root, al, dummy, lane, n_fg, g0, g1);
    }

    // ---- leaf decision and children (eq. scest, eq. PMupd) ---------------------------
    const bool info = (readlane(infow, i >> 5) >> (i & 31)) & 1u;
    const bool h = TR::hd(a0);
    const uint32_t ppm = (uint32_t)(pk >> 32);
    const uint32_t pm1 = TR::pm_add(ppm, TR::mag(a0));  // metric against the decision
    const uint32_t lo0 = key_lo(N, i + 1, next_seq);
    const uint64_t k0 = make_key((!info && h) ? pm1 : ppm, lo0);
    next_seq += info ? 2u : 1u;
    const int wi = i >> 5;
    const uint32_t bitm = 1u << (i & 31);
    if (info && h) {  // a decided 1 (a 0 is already there)
      ucur = (lane == wi) ? (ucur | bitm) : ucur;
      prow[lane == wi ? p : kRow] = ucur;
    }
    S.rekey(p, k0, lane);
    if (k0 > maxk) {  // never true while the worst key is unknown
      maxk = k0;
      max_slot = p;
    }

    if (info) {
      // the flipped child, against the decision: metric pm1, next sequence number
      const uint64_t k1 = make_key(pm1, lo0 + 1u);
      int t = -1;
      if (S.count() < D) {
        t = S.first_free();
        if (k1 > maxk) {
          maxk = k1;
          max_slot = t;
        }
      } else {
        if (maxk == kNone) S.worst(lane, max_slot, maxk);
        if (k1 < maxk) {
          t = max_slot;
          maxk = kNone;
          if constexpr (STATS) ++n_ev;
        } else {
          if constexpr (STATS) ++n_dr;
        }
      }
      if (t >= 0) {
        prow[lane < W ? t : kRow] = ucur ^ (lane == wi ? bitm : 0u);
        S.put(t, k1, lane);
        if (k1 < lb) lb = k1;
      }
    }
    lds_order();

    // L-counter pruning: drop every path of length <= i
    if ((int)((readlane(old, 0) >> (8 * (i & 3))) & 0xFFu) + 1 == L) {
      if constexpr (STATS) ++n_pr;
      S.prune(N, i);
      maxk = kNone;
    }
    wl = i;
    ulast = (info && h) ? 1u : 0u;  // the first child's bit i
    pk = k0;  // slot p now holds the first child
  }

  // output: payload = the first K - r information bits of the output path (systematic
  // encoding: of its codeword, the path's bits re-encoded)
  if (code.systematic) out = polar_transform_row(out, lane, N, W);
  if (lane < W) {
    uint32_t iw = infow;
    int k = code.pre[lane];
    uint8_t* dst = job.payload;
    while (iw) {
      const int b = __builtin_ctz(iw);
      iw &= iw - 1u;
      if (k < code.kp) dst[k] = (uint8_t)((st ? (out >> b) : 0u) & 1u);
      ++k;
    }
  }
  if (lane == 0) *job.status = (uint8_t)st;
  if constexpr (STATS) {
    const uint32_t v[8] = {n_it, n_sw, n_cp, n_sc, n_fg, n_ev, n_dr, n_pr};
    if (lane < 8) {
      uint32_t x = v[0];
#pragma unroll
      for (int j = 1; j < 8; ++j) x = lane == j ? v[j] : x;
      reinterpret_cast<uint32_t*>(job.stats)[lane] = x;
    }
  }
}

// Wavefronts per SIMD the register allocation must allow: the one-bank kernels fit 7 (at
// most 72 VGPRs) and are held to it (the compiler takes 8 where it can); the two-bank
// kernels up to N = 1024 are held to 8 (64 VGPRs, without spilling), the other banked
// kernels to 6 (80 VGPRs, a few words spilled): left free, the top stages' loads raised
// them to 67-105 VGPRs and one or two wavefronts fewer, 1-9 % slower.
template <int NB, int LOGN>
constexpr int scs_waves_per_simd() { return NB == 1 ? 7 : NB == 2 && LOGN <= 10 ? 8 : 6; }

template <int LOGN, class TR, bool STATS, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(scs_waves_per_simd<NB, LOGN>())))
void scs_uniform_kernel(CodeArgs code, int D, int L,
                                                          const typename TR::In* __restrict__ llr,
                                                          int64_t n_frames,
                                                          uint8_t* __restrict__ payload,
                                                          uint8_t* __restrict__ status,
                                                          scs_stats* __restrict__ stats,
                                                          int wave_words) {
  extern __shared__ uint32_t lds[];
  const int wave = threadIdx.x >> 6;
  const int64_t frame = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (frame >= n_frames) return;
  constexpr int N = 1 << LOGN;
  FrameJob job;
  job.llr = llr + frame * N;
  job.payload = payload + frame * code.kp;
  job.status = status + frame;
  job.stats = STATS ? stats + frame : nullptr;
  job.D = D;
  job.L = L;
  decode_frame<LOGN, TR, STATS, NB>(code, job, lds + wave * wave_words);
}

// ------------------------------------------------------------------------------------
// Mixed batches: one persistent launch, frames of any code / D / L taken from an atomic
// work counter in the order given by `order` (largest frames first), one frame per wave.
// ------------------------------------------------------------------------------------
template <class TR, bool STATS>
__device__ __forceinline__ void decode_any(int logn, const CodeArgs& code, const FrameJob& job,
                                           uint32_t* lds) {
  switch (logn) {
    case 1: decode_frame<1, TR, STATS, 1, true>(code, job, lds); break;
    case 2: decode_frame<2, TR, STATS, 1, true>(code, job, lds); break;
    case 3: decode_frame<3, TR, STATS, 1, true>(code, job, lds); break;
    case 4: decode_frame<4, TR, STATS, 1, true>(code, job, lds); break;
    case 5: decode_frame<5, TR, STATS, 1, true>(code, job, lds); break;
    case 6: decode_frame<6, TR, STATS, 1, true>(code, job, lds); break;
    case 7: decode_frame<7, TR, STATS, 1, true>(code, job, lds); break;
    case 8: decode_frame<8, TR, STATS, 1, true>(code, job, lds); break;
    case 9: decode_frame<9, TR, STATS, 1, true>(code, job, lds); break;
    case 10: decode_frame<10, TR, STATS, 1, true>(code, job, lds); break;
    case 11: decode_frame<11, TR, STATS, 1, true>(code, job, lds); break;
    default: break;
  }
}

// Zeroes the work counter on the launch stream (a kernel, so that the launch can be
// captured in a graph without memset nodes).
__global__ void reset_counter_kernel(uint32_t* counter) { *counter = 0u; }

// At most 80 VGPRs (6 wavefronts per SIMD): measured faster than the unconstrained 88 (5 per
// SIMD) and than 72 (7 per SIMD, which spills).
template <class TR, bool STATS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6)))
void scs_mixed_kernel(const CodeArgs* __restrict__ codes,
                      const scs_frame* __restrict__ frames,
                      const int32_t* __restrict__ order,
                      uint32_t n_frames,
                      const typename TR::In* __restrict__ llr,
                      uint8_t* __restrict__ payload,
                      uint8_t* __restrict__ status,
                      scs_stats* __restrict__ stats,
                      uint32_t* __restrict__ counter,
                      int wave_words) {
  extern __shared__ uint32_t lds[];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  uint32_t* mine = lds + wave * wave_words;
  for (;;) {
    uint32_t k = 0u;
    if (lane == 0) k = atomicAdd(counter, 1u);
    k = readlane(k, 0);
    if (k >= n_frames) break;  // every wave leaves once the queue is empty
    const int f = order ? order[k] : (int)k;  // no order: descriptor order
    const scs_frame d = frames[f];
    const CodeArgs& code = codes[d.code];
    FrameJob job;
    job.llr = llr + d.llr_off;
    job.payload = payload + d.out_off;
    job.status = status + f;
    job.stats = STATS ? stats + f : nullptr;
    job.D = d.D;
    job.L = d.L;
    decode_any<TR, STATS>(code.logn, code, job, mine);
    lds_order();
  }
}

// ------------------------------------------------------------------------------------
// Fixed scratch of the no-allocation mixed decoder (scs_decode_mixed_noalloc): the work
// counter, the code tables, their CRC syndrome tables and the frame descriptors of one
// batch.  Each device holds its own copy while the library is loaded.  Host code reaches it
// only through the address hipGetSymbolAddress returns for the device (noalloc_scratch).
// ------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)SCS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

// ------------------------------------------------------------------------------------
// Device encoder: one wave per frame, lane w owns bits 32w..32w+31 of u.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void encode_kernel(CodeArgs code, const uint16_t* __restrict__ crc_unit,
                                                     const uint8_t* __restrict__ payload,
                                                     uint8_t* __restrict__ codeword, int64_t B) {
  const int lane = lane_id();
  const int64_t f = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (f >= B) return;
  const uint8_t* pl = payload + f * code.kp;
  // CRC remainder: xor of the remainders of the payload's one-bits (linear CRC)
  uint32_t r = 0u;
  if (code.crc) {
    for (int k = lane; k < code.kp; k += kWave)
      if (pl[k] & 1u) r ^= crc_unit[k];
    for (int m = 1; m < kWave; m <<= 1) r ^= xor_lane_rt(r, m);
  }
  uint32_t x = 0u;
  if (lane < code.W) {
    uint32_t iw = code.info[lane];
    int k = code.pre[lane];
    while (iw) {
      const int b = __builtin_ctz(iw);
      iw &= iw - 1u;
      uint32_t bit;
      if (k < code.kp) bit = pl[k] & 1u;
      else bit = (r >> (code.crc - 1 - (k - code.kp))) & 1u;
      x |= bit << b;
      ++k;
    }
  }
  // u F^(x)n.  Systematic encoding: the message placed this way is v; its transform,
  // cleared at the frozen positions, is the u that is sent through the transform.
  x = polar_transform_row(x, lane, code.N, code.W);
  if (code.systematic) {
    x &= lane < code.W ? code.info[lane] : 0u;
    x = polar_transform_row(x, lane, code.N, code.W);
  }
  if (lane < code.W) {
    uint8_t* dst = codeword + f * code.N + lane * 32;
    const int nb = code.N < 32 ? code.N : 32;
    for (int b = 0; b < nb; ++b) dst[b] = (uint8_t)((x >> b) & 1u);
  }
}

// ------------------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------------------
template <class TR>
using UniformKernel = void (*)(CodeArgs, int, int, const typename TR::In*, int64_t, uint8_t*,
                               uint8_t*, scs_stats*, int);

template <class TR, bool STATS, int NB>
UniformKernel<TR> uniform_kernel_for_t(int logn) {
  switch (logn) {
    case 1: return scs_uniform_kernel<1, TR, STATS, NB>;
    case 2: return scs_uniform_kernel<2, TR, STATS, NB>;
    case 3: return scs_uniform_kernel<3, TR, STATS, NB>;
    case 4: return scs_uniform_kernel<4, TR, STATS, NB>;
    case 5: return scs_uniform_kernel<5, TR, STATS, NB>;
    case 6: return scs_uniform_kernel<6, TR, STATS, NB>;
    case 7: return scs_uniform_kernel<7, TR, STATS, NB>;
    case 8: return scs_uniform_kernel<8, TR, STATS, NB>;
    case 9: return scs_uniform_kernel<9, TR, STATS, NB>;
    case 10: return scs_uniform_kernel<10, TR, STATS, NB>;
    case 11: return scs_uniform_kernel<11, TR, STATS, NB>;
  }
  return nullptr;
}

// stack banks of 64 slots for depth D: 1, 2 or kMaxBanks
inline int stack_banks(int D) { return D <= 64 ? 1 : (D <= 128 ? 2 : kMaxBanks); }

template <class TR>
UniformKernel<TR> uniform_kernel_for(int logn, bool stats, int nb) {
  if (nb == 1)
    return stats ? uniform_kernel_for_t<TR, true, 1>(logn) : uniform_kernel_for_t<TR, false, 1>(logn);
  if (nb == 2)
    return stats ? uniform_kernel_for_t<TR, true, 2>(logn) : uniform_kernel_for_t<TR, false, 2>(logn);
  return stats ? uniform_kernel_for_t<TR, true, kMaxBanks>(logn)
               : uniform_kernel_for_t<TR, false, kMaxBanks>(logn);
}

int waves_per_block(int N, int D) {
  const int bytes = scs_lds_words_per_wave(N, D) * 4;
  int wpb = 4;
  while (wpb > 1 && wpb * bytes > 64 * 1024) wpb >>= 1;
  return wpb;
}

}  // namespace

// The HIP runtime keeps the last error of any call in the thread until it is read, and the
// process may share the runtime with other libraries (PyTorch loads its own copy under the
// same soname).  Launch sites read and drop whatever an earlier call left there, so that
// the check after a launch reports that launch alone.
inline void clear_stale_error() { (void)hipGetLastError(); }

// Device copies of a code's host tables (CRC unit remainders for the encoder, the CRC
// syndrome table for the decoders), one per code, device and table, uploaded on first use
// and kept until the process ends: a code's tables are a few to 128 KB.
enum CodeTable { kTabCrcUnit = 0, kTabCrcSyn = 1, kTabNodes = 2 };

int device_table_bytes(const polar_code* code, CodeTable which, const void** out) {
  static std::mutex mu;
  static std::unordered_map<uint64_t, void*> tables;  // key: (uid * 64 + device) * 4 + table
  *out = nullptr;
  const void* src = nullptr;
  size_t bytes = 0;
  if (which == kTabCrcUnit) {
    src = code->crc_unit.data();
    bytes = code->crc_unit.size() * sizeof(uint16_t);
  } else if (which == kTabCrcSyn) {
    src = code->crc_syn.data();
    bytes = code->crc_syn.size() * sizeof(uint16_t);
  } else {
    src = code->nodes.data();
    bytes = code->nodes.size();
  }
  if (bytes == 0 || (which != kTabNodes && code->crc == 0)) return POLAR_OK;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return POLAR_EDEVICE;
  const uint64_t key = (code->uid * 64 + (uint64_t)dev) * 4 + (uint64_t)which;
  std::lock_guard<std::mutex> g(mu);
  auto it = tables.find(key);
  if (it != tables.end()) {
    *out = it->second;
    return POLAR_OK;
  }
  // the node table is read a 32-bit word at a time (wave-uniform scalar loads), so its
  // copy is zero-padded to whole words: codes as short as N = 2 have 2 bytes of it
  std::vector<uint8_t> padded;
  if (which == kTabNodes && bytes % 4 != 0) {
    padded.assign((const uint8_t*)src, (const uint8_t*)src + bytes);
    padded.resize((bytes + 3) & ~(size_t)3, 0);
    src = padded.data();
    bytes = padded.size();
  }
  void* tab = nullptr;
  if (hipMalloc(&tab, bytes) != hipSuccess) return POLAR_ENOMEM;
  if (hipMemcpy(tab, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(tab);
    return POLAR_EDEVICE;
  }
  tables[key] = tab;
  *out = tab;
  return POLAR_OK;
}

template <class T>
int device_table(const polar_code* code, CodeTable which, const T** out) {
  const void* p = nullptr;
  const int e = device_table_bytes(code, which, &p);
  *out = (const T*)p;
  return e;
}

struct scs_ctx {
  int device = 0;
  int wpb = 0;    // wavefronts per workgroup: 0 = automatic, else 1, 2 or 4
  int last_error = POLAR_OK;
  int cus = 0;    // compute units of the device
  int grid_cus = 0;  // CUs' worth of workgroups of a persistent launch: 0 = cus
  std::mutex mu;
  // mixed-batch plan: device copies of the code tables, descriptors and the frame order,
  // the work counter, and a pinned staging area for the uploads
  CodeArgs* d_codes = nullptr;
  size_t cap_codes = 0;
  scs_frame* d_frames = nullptr;
  int32_t* d_order = nullptr;
  size_t cap_frames = 0;
  uint32_t* d_counter = nullptr;
  char* h_stage = nullptr;
  size_t cap_stage = 0;
  hipEvent_t staged = nullptr;
  hipEvent_t launched = nullptr;  // the last mixed launch enqueued outside graph capture
  uint32_t plan_frames = 0;
  int plan_wave_words = 0;
  void* scratch = nullptr;  // device address of this device's fixed scratch array
};

namespace {

constexpr size_t kMaxLdsPerBlock = 64 * 1024;

// Device address of `scratch` per device, resolved once with that device current (the
// array's name in host code is only a stand-in for the symbol).  Null until resolved.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Resolves the scratch address of `device`, which is current.  Called at context creation.
int resolve_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return POLAR_EUNSUPPORTED;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return POLAR_EDEVICE;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return POLAR_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

extern "C" {

int scs_ctx_create(int device, scs_ctx** out) {
  if (!out) return POLAR_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return POLAR_EDEVICE;
  if (device < 0 || device >= n) return POLAR_EINVAL;
  scs_ctx* c = new (std::nothrow) scs_ctx;
  if (!c) return POLAR_ENOMEM;
  c->device = device;
  int dev0 = 0;
  (void)hipGetDevice(&dev0);
  if (hipSetDevice(device) != hipSuccess ||
      hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipMalloc(&c->d_counter, sizeof(uint32_t)) != hipSuccess ||
      hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->launched, hipEventDisableTiming) != hipSuccess ||
      resolve_scratch(device, &c->scratch) != POLAR_OK) {
    (void)hipFree(c->d_counter);
    if (c->staged) (void)hipEventDestroy(c->staged);
    if (c->launched) (void)hipEventDestroy(c->launched);
    delete c;
    (void)hipSetDevice(dev0);
    return POLAR_EDEVICE;
  }
  (void)hipSetDevice(dev0);
  *out = c;
  return POLAR_OK;
}

void scs_ctx_destroy(scs_ctx* ctx) {
  if (!ctx) return;
  // teardown: errors here cannot be acted on
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->d_codes);
  (void)hipFree(ctx->d_frames);
  (void)hipFree(ctx->d_order);
  (void)hipFree(ctx->d_counter);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->staged) (void)hipEventDestroy(ctx->staged);
  if (ctx->launched) (void)hipEventDestroy(ctx->launched);
  delete ctx;
}

int scs_ctx_set_waves_per_block(scs_ctx* ctx, int32_t waves_per_block) {
  if (!ctx) return POLAR_EINVAL;
  if (waves_per_block != 0 && waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4)
    return POLAR_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->wpb = waves_per_block;
  return POLAR_OK;
}

int scs_ctx_set_grid_cus(scs_ctx* ctx, int32_t cus) {
  if (!ctx || cus < 0 || cus > ctx->cus) return POLAR_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  ctx->grid_cus = cus;
  return POLAR_OK;
}

int scs_ctx_last_error(scs_ctx* ctx) {
  if (!ctx) return POLAR_EINVAL;
  std::lock_guard<std::mutex> g(ctx->mu);
  const int e = ctx->last_error;
  ctx->last_error = POLAR_OK;
  return e;
}

int scs_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t D, int32_t L,
                     int32_t llr_dtype, const void* llr_dev, int64_t n_frames,
                     uint8_t* payload_dev, uint8_t* status_dev, scs_stats* stats_dev,
                     void* hip_stream) {
  if (!ctx || !code) return POLAR_EINVAL;
  if (D < 1 || D > kMaxDepth || L < 1 || L > 255) return POLAR_EINVAL;
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (n_frames < 0) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (!llr_dev || !status_dev || (!payload_dev && code->payload_bits() > 0)) return POLAR_EINVAL;
  if (code->logn < 1 || code->logn > 11) return POLAR_EUNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;

  CodeArgs args = make_args(code);
  if (const int e = device_table(code, kTabCrcSyn, &args.crc_tab)) return e;
  hipStream_t s = (hipStream_t)hip_stream;
  int wpb = waves_per_block(code->N, D);
  if (ctx->wpb && ctx->wpb < wpb) wpb = ctx->wpb;
  const int wave_words = scs_lds_words_per_wave(code->N, D);
  const size_t lds = (size_t)wpb * wave_words * 4;
  const int64_t blocks = (n_frames + wpb - 1) / wpb;
  if (blocks > 0x7FFFFFFF) return POLAR_EUNSUPPORTED;
  clear_stale_error();
  if (llr_dtype == SCS_LLR_F32) {
    auto k = uniform_kernel_for<TrF32>(code->logn, stats_dev != nullptr, stack_banks(D));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, s, args, (int)D, (int)L,
                       (const float*)llr_dev, n_frames, payload_dev, status_dev, stats_dev,
                       wave_words);
  } else {
    auto k = uniform_kernel_for<TrI8>(code->logn, stats_dev != nullptr, stack_banks(D));
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, s, args, (int)D, (int)L,
                       (const int8_t*)llr_dev, n_frames, payload_dev, status_dev, stats_dev,
                       wave_words);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = POLAR_EDEVICE;
    return POLAR_EDEVICE;
  }
  return POLAR_OK;
}

int fsscs_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t D, int32_t L,
                       int32_t llr_dtype, const void* llr_dev, int64_t n_frames,
                       uint8_t* payload_dev, uint8_t* status_dev, scs_stats* stats_dev,
                       void* hip_stream) {
  if (!ctx || !code) return POLAR_EINVAL;
  if (D < 1 || D > kMaxDepth || L < 1 || L > 255) return POLAR_EINVAL;
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (n_frames < 0) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (!llr_dev || !status_dev || (!payload_dev && code->payload_bits() > 0)) return POLAR_EINVAL;
  if (code->logn < 1 || code->logn > 11) return POLAR_EUNSUPPORTED;
  // creation numbers: at most L extensions per node, each numbering all its candidates
  uint64_t per_round = 0;
  for (int j = 0; j < code->N; ++j) {
    const uint8_t nd = code->nodes[(size_t)j];
    if (nd == 0xFF) continue;
    const int cls = nd >> 4, lam = nd & 15;
    per_round += cls == 0 ? 1 : (cls == 2 ? 2 : (cls == 3 ? 8 : (lam == 0 ? 2 : 4)));
  }
  if (1 + (uint64_t)L * per_round > kSeqMask) return POLAR_EUNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;
  polarscs::FsscsLaunch a;
  a.code = make_args(code);
  if (const int e = device_table(code, kTabCrcSyn, &a.code.crc_tab)) return e;
  if (const int e = device_table(code, kTabNodes, &a.code.nodes)) return e;
  int wpb = waves_per_block(code->N, D);
  if (ctx->wpb && ctx->wpb < wpb) wpb = ctx->wpb;
  a.D = D;
  a.L = L;
  a.dtype = llr_dtype;
  a.waves_per_block = wpb;
  a.llr = llr_dev;
  a.n_frames = n_frames;
  a.payload = payload_dev;
  a.status = status_dev;
  a.stats = stats_dev;
  a.stream = (hipStream_t)hip_stream;
  if ((n_frames + wpb - 1) / wpb > 0x7FFFFFFF) return POLAR_EUNSUPPORTED;
  if (polarscs::launch_fsscs(a) != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = POLAR_EDEVICE;
    return POLAR_EDEVICE;
  }
  return POLAR_OK;
}

int scl_decode_batch(scs_ctx* ctx, const polar_code* code, int32_t L, int32_t llr_dtype,
                     const void* llr_dev, int64_t n_frames, uint8_t* payload_dev,
                     uint8_t* status_dev, scs_stats* stats_dev, void* hip_stream) {
  if (!ctx || !code) return POLAR_EINVAL;
  if (L != 1 && L != 2 && L != 4 && L != 8) return POLAR_EINVAL;
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (n_frames < 0) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (!llr_dev || !status_dev || (!payload_dev && code->payload_bits() > 0)) return POLAR_EINVAL;
  if (code->logn < 1 || code->logn > 11) return POLAR_EUNSUPPORTED;
  const size_t bytes = polarscs::scl_lds_bytes(code->N, L);
  if (bytes > kMaxLdsPerBlock) return POLAR_EUNSUPPORTED;
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;
  polarscs::SclLaunch a;
  a.code = make_args(code);
  if (const int e = device_table(code, kTabCrcSyn, &a.code.crc_tab)) return e;
  int wpb = 1;
  const int cap = ctx->wpb ? ctx->wpb : 4;
  while (wpb < cap && (size_t)(wpb * 2) * bytes <= kMaxLdsPerBlock) wpb *= 2;
  a.L = L;
  a.dtype = llr_dtype;
  a.waves_per_block = wpb;
  a.llr = llr_dev;
  a.n_frames = n_frames;
  a.payload = payload_dev;
  a.status = status_dev;
  a.stats = stats_dev;
  a.stream = (hipStream_t)hip_stream;
  if ((n_frames + wpb - 1) / wpb > 0x7FFFFFFF) return POLAR_EUNSUPPORTED;
  if (polarscs::launch_scl(a) != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = POLAR_EDEVICE;
    return POLAR_EDEVICE;
  }
  return POLAR_OK;
}

int polar_code_schedule(const polar_code* code, uint8_t* nodes_out) {
  if (!code || !nodes_out) return POLAR_EINVAL;
  std::memcpy(nodes_out, code->nodes.data(), (size_t)code->N);
  return POLAR_OK;
}

int scs_mixed_prepare(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                      const scs_frame* frames_host, int64_t n_frames, void* hip_stream) {
  if (!ctx || n_frames < 0 || n_codes < 0 || n_frames > 0x7FFFFFFF) return POLAR_EINVAL;
  if (n_frames > 0 && (!codes || n_codes < 1 || !frames_host)) return POLAR_EINVAL;
  for (int32_t c = 0; c < n_codes; ++c)
    if (!codes[c] || codes[c]->logn < 1 || codes[c]->logn > 11) return POLAR_EINVAL;
  int wave_words = 0;
  for (int64_t f = 0; f < n_frames; ++f) {
    const scs_frame& d = frames_host[f];
    if (d.code < 0 || d.code >= n_codes || d.D < 1 || d.D > 64 || d.L < 1 || d.L > 255 ||
        d._pad != 0 || d.llr_off < 0 || d.out_off < 0)
      return POLAR_EINVAL;
    wave_words = std::max(wave_words, scs_lds_words_per_wave(codes[d.code]->N, d.D));
  }
  if ((size_t)wave_words * 4 > 64 * 1024) return POLAR_EUNSUPPORTED;
  std::lock_guard<std::mutex> g(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  // largest frames first (N L), so that the work queue ends with short frames
  std::vector<int32_t> order((size_t)n_frames);
  std::vector<int32_t> weight((size_t)n_frames);
  for (int64_t f = 0; f < n_frames; ++f) {
    order[f] = (int32_t)f;
    weight[f] = codes[frames_host[f].code]->N * frames_host[f].L;
  }
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return weight[a] > weight[b]; });
  const size_t nc = (size_t)std::max(n_codes, 1), nf = (size_t)std::max<int64_t>(n_frames, 1);
  // grow-only device buffers (earlier launches may still read the old ones)
  if (nc > ctx->cap_codes || nf > ctx->cap_frames) {
    if (hipDeviceSynchronize() != hipSuccess) return POLAR_EDEVICE;
    if (nc > ctx->cap_codes) {
      (void)hipFree(ctx->d_codes);  // the device is idle (synchronized above)
      ctx->d_codes = nullptr;
      if (hipMalloc(&ctx->d_codes, nc * sizeof(CodeArgs)) != hipSuccess) return POLAR_ENOMEM;
      ctx->cap_codes = nc;
    }
    if (nf > ctx->cap_frames) {
      (void)hipFree(ctx->d_frames);
      (void)hipFree(ctx->d_order);
      ctx->d_frames = nullptr;
      ctx->d_order = nullptr;
      if (hipMalloc(&ctx->d_frames, nf * sizeof(scs_frame)) != hipSuccess ||
          hipMalloc(&ctx->d_order, nf * sizeof(int32_t)) != hipSuccess)
        return POLAR_ENOMEM;
      ctx->cap_frames = nf;
    }
  }
  const size_t bytes = nc * sizeof(CodeArgs) + nf * sizeof(scs_frame) + nf * sizeof(int32_t);
  if (hipEventSynchronize(ctx->staged) != hipSuccess) return POLAR_EDEVICE;  // staging free
  // the plan buffers may still be read by this context's last launch, on any stream
  if (hipStreamWaitEvent(s, ctx->launched, 0) != hipSuccess) return POLAR_EDEVICE;
  if (bytes > ctx->cap_stage) {
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    ctx->h_stage = nullptr;
    if (hipHostMalloc((void**)&ctx->h_stage, bytes, hipHostMallocDefault) != hipSuccess)
      return POLAR_ENOMEM;
    ctx->cap_stage = bytes;
  }
  CodeArgs* hc = (CodeArgs*)ctx->h_stage;
  scs_frame* hf = (scs_frame*)(ctx->h_stage + nc * sizeof(CodeArgs));
  int32_t* ho = (int32_t*)(ctx->h_stage + nc * sizeof(CodeArgs) + nf * sizeof(scs_frame));
  for (int32_t c = 0; c < n_codes; ++c) {
    hc[c] = make_args(codes[c]);
    if (const int e = device_table(codes[c], kTabCrcSyn, &hc[c].crc_tab)) return e;
  }
  if (n_frames) {
    std::memcpy(hf, frames_host, (size_t)n_frames * sizeof(scs_frame));
    std::memcpy(ho, order.data(), (size_t)n_frames * sizeof(int32_t));
  }
  if (hipMemcpyAsync(ctx->d_codes, hc, nc * sizeof(CodeArgs), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ctx->d_frames, hf, nf * sizeof(scs_frame), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(ctx->d_order, ho, nf * sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventRecord(ctx->staged, s) != hipSuccess)
    return POLAR_EDEVICE;
  ctx->plan_frames = (uint32_t)n_frames;
  ctx->plan_wave_words = wave_words;
  return POLAR_OK;
}

int scs_mixed_launch(scs_ctx* ctx, int32_t llr_dtype, const void* llr_dev, uint8_t* payload_dev,
                     uint8_t* status_dev, scs_stats* stats_dev, void* hip_stream) {
  if (!ctx) return POLAR_EINVAL;
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (ctx->plan_frames == 0) return POLAR_OK;
  if (!llr_dev || !status_dev || !payload_dev) return POLAR_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  const int ww = ctx->plan_wave_words;
  int wpb = ctx->wpb ? ctx->wpb : 4;
  while (wpb > 1 && (size_t)wpb * ww * 4 > 64 * 1024) wpb >>= 1;
  const size_t lds = (size_t)wpb * ww * 4;
  const bool st = stats_dev != nullptr;
  const void* kfun;
  if (llr_dtype == SCS_LLR_F32)
    kfun = st ? (const void*)scs_mixed_kernel<TrF32, true> : (const void*)scs_mixed_kernel<TrF32, false>;
  else
    kfun = st ? (const void*)scs_mixed_kernel<TrI8, true> : (const void*)scs_mixed_kernel<TrI8, false>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfun, 64 * wpb, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t need = ((int64_t)ctx->plan_frames + wpb - 1) / wpb;
  const int grid_cus = ctx->grid_cus ? ctx->grid_cus : ctx->cus;
  const unsigned blocks = (unsigned)std::min<int64_t>((int64_t)per_cu * grid_cus, need);
  // Launches of one context share its work counter: outside graph capture, a launch waits
  // for the context's previous one (on any stream) and is recorded for the next.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cap) != hipSuccess) return POLAR_EDEVICE;
  const bool track = cap == hipStreamCaptureStatusNone;
  if (track && hipStreamWaitEvent(s, ctx->launched, 0) != hipSuccess) return POLAR_EDEVICE;
  clear_stale_error();
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, ctx->d_counter);
  if (llr_dtype == SCS_LLR_F32) {
    auto k = st ? scs_mixed_kernel<TrF32, true> : scs_mixed_kernel<TrF32, false>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, s, ctx->d_codes, ctx->d_frames,
                       ctx->d_order, ctx->plan_frames, (const float*)llr_dev, payload_dev,
                       status_dev, stats_dev, ctx->d_counter, ww);
  } else {
    auto k = st ? scs_mixed_kernel<TrI8, true> : scs_mixed_kernel<TrI8, false>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, s, ctx->d_codes, ctx->d_frames,
                       ctx->d_order, ctx->plan_frames, (const int8_t*)llr_dev, payload_dev,
                       status_dev, stats_dev, ctx->d_counter, ww);
  }
  if (hipGetLastError() != hipSuccess || (track && hipEventRecord(ctx->launched, s) != hipSuccess)) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = POLAR_EDEVICE;
    return POLAR_EDEVICE;
  }
  return POLAR_OK;
}

int scs_decode_mixed(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                     const scs_frame* frames_host, int64_t n_frames, int32_t llr_dtype,
                     const void* llr_dev, uint8_t* payload_dev, uint8_t* status_dev,
                     scs_stats* stats_dev, void* hip_stream) {
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (n_frames > 0 && (!llr_dev || !status_dev || !payload_dev)) return POLAR_EINVAL;
  const int rc = scs_mixed_prepare(ctx, codes, n_codes, frames_host, n_frames, hip_stream);
  if (rc != POLAR_OK) return rc;
  return scs_mixed_launch(ctx, llr_dtype, llr_dev, payload_dev, status_dev, stats_dev, hip_stream);
}

int scs_decode_mixed_noalloc(scs_ctx* ctx, const polar_code* const* codes, int32_t n_codes,
                             const scs_frame* frames_host, int64_t n_frames, int32_t llr_dtype,
                             const void* llr_dev, uint8_t* payload_dev, uint8_t* status_dev,
                             scs_stats* stats_dev, void* hip_stream) {
  if (!ctx || n_frames < 0 || n_codes < 0) return POLAR_EINVAL;
  if (llr_dtype != SCS_LLR_F32 && llr_dtype != SCS_LLR_I8) return POLAR_EINVAL;
  if (n_frames == 0) return POLAR_OK;
  if (!codes || n_codes < 1 || !frames_host || !llr_dev || !status_dev || !payload_dev)
    return POLAR_EINVAL;
  if (n_codes > SCS_NOALLOC_MAX_CODES) return POLAR_ETOOLARGE;
  for (int32_t c = 0; c < n_codes; ++c)
    if (!codes[c] || codes[c]->logn < 1 || codes[c]->logn > 11) return POLAR_EINVAL;
  bool used[SCS_NOALLOC_MAX_CODES] = {};
  int wave_words = 0;
  for (int64_t f = 0; f < n_frames; ++f) {
    const scs_frame& d = frames_host[f];
    if (d.code < 0 || d.code >= n_codes || d.D < 1 || d.D > 64 || d.L < 1 || d.L > 255 ||
        d._pad != 0 || d.llr_off < 0 || d.out_off < 0)
      return POLAR_EINVAL;
    used[d.code] = true;
    wave_words = std::max(wave_words, scs_lds_words_per_wave(codes[d.code]->N, d.D));
  }
  if ((size_t)wave_words * 4 > kMaxLdsPerBlock) return POLAR_EUNSUPPORTED;
  // scratch layout: work counter | code tables | CRC syndrome tables | frame descriptors
  const size_t off_codes = 256;
  size_t off = align256(off_codes + (size_t)n_codes * sizeof(CodeArgs));
  size_t crc_off[SCS_NOALLOC_MAX_CODES] = {};
  for (int32_t c = 0; c < n_codes; ++c) {
    if (!used[c] || codes[c]->crc == 0) continue;
    crc_off[c] = off;
    off = align256(off + codes[c]->crc_syn.size() * sizeof(uint16_t));
  }
  const size_t off_frames = off;
  const size_t need = off_frames + (size_t)n_frames * sizeof(scs_frame);
  if ((uint64_t)n_frames > 0x7FFFFFFFull || need > kScratchBytes) return POLAR_ETOOLARGE;
  if (!ctx->scratch) return POLAR_EDEVICE;
  if (hipSetDevice(ctx->device) != hipSuccess) return POLAR_EDEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  uint8_t* base = (uint8_t*)ctx->scratch;
  // code tables, built on the host stack; their CRC tables point into the scratch array
  CodeArgs args[SCS_NOALLOC_MAX_CODES];
  for (int32_t c = 0; c < n_codes; ++c) {
    args[c] = make_args(codes[c]);
    args[c].crc_tab = crc_off[c] ? (const uint16_t*)(base + crc_off[c]) : nullptr;
  }
  // Host-to-device copies of pageable memory return once the source has been read, after
  // the stream's earlier work (which may still read the scratch array) has finished.
  clear_stale_error();
  if (hipMemcpyAsync(base + off_codes, args, (size_t)n_codes * sizeof(CodeArgs),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return POLAR_EDEVICE;
  for (int32_t c = 0; c < n_codes; ++c)
    if (crc_off[c] &&
        hipMemcpyAsync(base + crc_off[c], codes[c]->crc_syn.data(),
                       codes[c]->crc_syn.size() * sizeof(uint16_t), hipMemcpyHostToDevice,
                       s) != hipSuccess)
      return POLAR_EDEVICE;
  if (hipMemcpyAsync(base + off_frames, frames_host, (size_t)n_frames * sizeof(scs_frame),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return POLAR_EDEVICE;
  int wpb = ctx->wpb ? ctx->wpb : 4;
  while (wpb > 1 && (size_t)wpb * wave_words * 4 > kMaxLdsPerBlock) wpb >>= 1;
  const size_t lds = (size_t)wpb * wave_words * 4;
  const bool st = stats_dev != nullptr;
  const void* kfun;
  if (llr_dtype == SCS_LLR_F32)
    kfun = st ? (const void*)scs_mixed_kernel<TrF32, true> : (const void*)scs_mixed_kernel<TrF32, false>;
  else
    kfun = st ? (const void*)scs_mixed_kernel<TrI8, true> : (const void*)scs_mixed_kernel<TrI8, false>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfun, 64 * wpb, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t want = (n_frames + wpb - 1) / wpb;
  const int grid_cus = ctx->grid_cus ? ctx->grid_cus : ctx->cus;
  const unsigned blocks = (unsigned)std::min<int64_t>((int64_t)per_cu * grid_cus, want);
  uint32_t* counter = (uint32_t*)base;
  const CodeArgs* d_codes = (const CodeArgs*)(base + off_codes);
  const scs_frame* d_frames = (const scs_frame*)(base + off_frames);
  // the counter keeps the previous call's value: a kernel zeroes it on the stream
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
  if (llr_dtype == SCS_LLR_F32) {
    auto k = st ? scs_mixed_kernel<TrF32, true> : scs_mixed_kernel<TrF32, false>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, s, d_codes, d_frames,
                       (const int32_t*)nullptr, (uint32_t)n_frames, (const float*)llr_dev,
                       payload_dev, status_dev, stats_dev, counter, wave_words);
  } else {
    auto k = st ? scs_mixed_kernel<TrI8, true> : scs_mixed_kernel<TrI8, false>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, s, d_codes, d_frames,
                       (const int32_t*)nullptr, (uint32_t)n_frames, (const int8_t*)llr_dev,
                       payload_dev, status_dev, stats_dev, counter, wave_words);
  }
  if (hipGetLastError() != hipSuccess) {
    std::lock_guard<std::mutex> g(ctx->mu);
    ctx->last_error = POLAR_EDEVICE;
    return POLAR_EDEVICE;
  }
  return POLAR_OK;
}

int polar_encode_device(const polar_code* code, const uint8_t* payload_dev,
                        uint8_t* codeword_dev, int64_t B, void* hip_stream) {
  if (!code || B < 0) return POLAR_EINVAL;
  if (B == 0) return POLAR_OK;
  if (!codeword_dev || (!payload_dev && code->payload_bits() > 0)) return POLAR_EINVAL;
  const uint16_t* tab = nullptr;
  if (const int e = device_table(code, kTabCrcUnit, &tab)) return e;
  const CodeArgs args = make_args(code);
  const int64_t blocks = (B + 3) / 4;
  if (blocks > 0x7FFFFFFF) return POLAR_EUNSUPPORTED;
  clear_stale_error();
  hipLaunchKernelGGL(encode_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)hip_stream,
                     args, tab, payload_dev, codeword_dev, B);
  return hipGetLastError() == hipSuccess ? POLAR_OK : POLAR_EDEVICE;
}

}  // extern "C"
