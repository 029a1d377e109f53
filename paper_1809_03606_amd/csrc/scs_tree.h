// The alpha tree, the partial sums of a g-node's left sibling, path keys and the CRC
// syndrome: pieces shared by the stack decoders of this library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "scs_device.h"

namespace {

// ------------------------------------------------------------------------------------
// alpha tree in LDS: stage lambda (Lambda = 2^lambda values) at word offset Lambda - 1,
// stages 0 .. n-1 (N - 1 words); the channel LLRs (stage n) are read from the input.
// ------------------------------------------------------------------------------------
// From this code length up (N = 1024) the SCS decoder does not keep stage n-1 (N/2 words):
// stage n-2 is computed straight from the channel LLRs whenever it is needed, which halves
// the alpha tree's share of LDS and lets more wavefronts share a CU (measured: N = 2048
// +13 %, N = 1024 +2 %, shorter codes not measurably different).
constexpr int kTopFreeLogN = 10;

template <int LOGN>
struct Layout {
  static constexpr int N = 1 << LOGN;
  static constexpr int W = N >= 32 ? N / 32 : 1;         // 32-bit words per bit vector
  static constexpr int SMALL = LOGN < 6 ? LOGN - 1 : 5;  // highest stage kept lane-parallel
  static constexpr bool KEEP_TOP = LOGN < kTopFreeLogN;  // stage n-1 kept in LDS
  static constexpr int ALPHA_WORDS = KEEP_TOP ? N : N / 2;  // stages kept (+1 spare word)
};

constexpr uint32_t kLowMask[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu,
                                  0x0000FFFFu};

// Partial sums (eq. bitcalc carried through all LAM levels: the polar transform) of the
// block of 2^LAM decided bits [base, base + 2^LAM) of u, where lane w of u holds bits
// 32w..32w+31.  This is the beta of the left sibling that g needs (eq. llrcalc); it is
// computed when needed from the decided bits.  For blocks of <= 32 bits the result is a
// scalar word whose bit e belongs to position base + e.
template <int LAM>
__device__ __forceinline__ uint32_t sibling_small(uint32_t u, int base) {
  uint32_t x = readlane(u, base >> 5);
  if constexpr (LAM < 5) x = (x >> (base & 31)) & ((1u << (1 << LAM)) - 1u);
#pragma unroll
  for (int s = 0; s < LAM; ++s) x ^= (x >> (1 << s)) & kLowMask[s];
  return x;
}

template <int S, int LAM>
__device__ __forceinline__ void sibling_cross(uint32_t& x, int lane) {
  if constexpr (S < LAM) {
    constexpr int dw = 1 << (S - 5);
    const uint32_t y = xor_lane<dw>(x);
    if (!(lane & dw)) x ^= y;
    sibling_cross<S + 1, LAM>(x, lane);
  }
}

// Blocks of >= 64 bits: lane-per-word result, zero outside the block.
template <int LAM>
__device__ __forceinline__ uint32_t sibling_big(uint32_t u, int base, int lane) {
  constexpr int NW = (1 << LAM) / 32;
  const int w0 = base >> 5;
  uint32_t x = (lane >= w0 && lane < w0 + NW) ? u : 0u;
#pragma unroll
  for (int s = 0; s < 5; ++s) x ^= (x >> (1 << s)) & kLowMask[s];
  sibling_cross<5, LAM>(x, lane);
  return x;
}

// Word w of a lane-per-word vector, in every lane (w may differ between lanes).
__device__ __forceinline__ uint32_t lane_word(uint32_t x, int w) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(w << 2, (int)x);
}

// Stage n-2 of a code whose stage n-1 is not kept (Layout::KEEP_TOP false): value e of
// stage n-2 from values e and e + N/4 of stage n-1, each made on the spot from the channel
// LLRs x and x + N/2 (eq. llrcalc twice; the same operations on the same operands as when
// stage n-1 is stored, so the values are identical).
template <int LOGN, class TR, bool STATS>
__device__ __forceinline__ void top_two_stages(int i, uint32_t u,
                                               const typename TR::In* __restrict__ root,
                                               uint32_t* al, int lane, uint32_t& fg) {
  constexpr int L1 = LOGN - 1, L2 = LOGN - 2;
  constexpr int Lam1 = 1 << L1, Lam2 = 1 << L2;
  const bool odd1 = (i >> L1) & 1;                 // stage n-1: g-node (right half)
  const bool odd2 = (i >> L2) & 1;                 // stage n-2: g-node
  const int base2 = ((i >> L2) - 1) << L2;         // its left sibling block
  uint32_t b1 = 0u, b2 = 0u;
  if (odd1) b1 = sibling_big<L1>(u, 0, lane);      // partial sums of bits [0, N/2)
  if (odd2) b2 = sibling_big<L2>(u, base2, lane);
  uint32_t* dst = al + (Lam2 - 1);
  // Lane l makes values e = V l .. V l + V - 1: each operand is V consecutive channel LLRs,
  // and the partial-sum bits of those values sit in one word (V divides 32).
  constexpr int V = Lam2 / kWave;
  static_assert(V <= 32 && 32 % V == 0, "a lane's values share one partial-sum word");
  const int e0 = V * lane;
  uint32_t m1 = 0u, m1c = 0u, m2 = 0u;
  if (odd1) {
    m1 = lane_word(b1, e0 >> 5) >> (e0 & 31);
    m1c = lane_word(b1, (e0 + Lam2) >> 5) >> (e0 & 31);
  }
  if (odd2) m2 = lane_word(b2, (base2 >> 5) + (e0 >> 5)) >> (e0 & 31);
  uint32_t p0[V], p1[V];
  {
    uint32_t x[V], y[V];
#pragma unroll
    for (int k = 0; k < V; ++k) x[k] = TR::load(root, e0 + k);
#pragma unroll
    for (int k = 0; k < V; ++k) y[k] = TR::load(root, e0 + Lam1 + k);
#pragma unroll
    for (int k = 0; k < V; ++k) p0[k] = odd1 ? TR::g(x[k], y[k], (m1 >> k) & 1u) : TR::f(x[k], y[k]);
  }
  {
    uint32_t x[V], y[V];
#pragma unroll
    for (int k = 0; k < V; ++k) x[k] = TR::load(root, e0 + Lam2 + k);
#pragma unroll
    for (int k = 0; k < V; ++k) y[k] = TR::load(root, e0 + Lam2 + Lam1 + k);
#pragma unroll
    for (int k = 0; k < V; ++k) p1[k] = odd1 ? TR::g(x[k], y[k], (m1c >> k) & 1u) : TR::f(x[k], y[k]);
  }
#pragma unroll
  for (int k = 0; k < V; ++k)
    dst[e0 + k] = odd2 ? TR::g(p0[k], p1[k], (m2 >> k) & 1u) : TR::f(p0[k], p1[k]);
  if constexpr (STATS) fg += (uint32_t)(Lam1 + Lam2);
  lds_order();
}

// Stage LAM >= 6 (Lambda >= 64), then the stages below it down to 6: value e = 64 r + lane
// of stage lambda from values e and e + Lambda of its parent (eq. llrcalc): f for even
// phi = i >> lambda, g for odd phi with the partial sums of the left sibling block.
template <int LAM, int LOGN, class TR, bool STATS>
__device__ __forceinline__ void big_stages(int top, int i, uint32_t u,
                                           const typename TR::In* __restrict__ root,
                                           uint32_t* al, int lane, uint32_t& fg) {
  if constexpr (LAM + 1 == LOGN && !Layout<LOGN>::KEEP_TOP) {
    static_assert(LAM - 1 >= 6, "stage n-2 must be a wide stage");
    if (LAM - 1 <= top) top_two_stages<LOGN, TR, STATS>(i, u, root, al, lane, fg);
    big_stages<LAM - 2, LOGN, TR, STATS>(top, i, u, root, al, lane, fg);
  } else if constexpr (LAM >= 6) {
    if (LAM <= top) {
      constexpr int Lam = 1 << LAM;
      const bool odd = (i >> LAM) & 1;
      const int base = ((i >> LAM) - 1) << LAM;
      uint32_t bx = 0u;
      if (odd) bx = sibling_big<LAM>(u, base, lane);
      uint32_t* dst = al + (Lam - 1);
      const uint32_t* src = al + (2 * Lam - 1);
      if (!odd) {
#pragma unroll
        for (int r = 0; r < Lam / kWave; ++r) {
          const int e = r * kWave + lane;
          if constexpr (LAM + 1 == LOGN)
            dst[e] = TR::f(TR::load(root, e), TR::load(root, e + Lam));
          else
            dst[e] = TR::f(src[e], src[e + Lam]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < Lam / kWave; ++r) {
          const int e = r * kWave + lane;
          const int w0 = (base >> 5) + 2 * r;
          const uint32_t mlo = readlane(bx, w0), mhi = readlane(bx, w0 + 1);
          const uint32_t m = lane < 32 ? mlo : mhi;
          const bool u = (m >> (lane & 31)) & 1u;
          if constexpr (LAM + 1 == LOGN)
            dst[e] = TR::g(TR::load(root, e), TR::load(root, e + Lam), u);
          else
            dst[e] = TR::g(src[e], src[e + Lam], u);
        }
      }
      if constexpr (STATS) fg += (uint32_t)Lam;
      lds_order();
    }
    big_stages<LAM - 1, LOGN, TR, STATS>(top, i, u, root, al, lane, fg);
  }
}

// One register stage: value e of stage LAM in lane e from lanes e and e xor Lambda.
template <int LAM, class TR>
__device__ __forceinline__ uint32_t reg_stage(uint32_t x, int i, uint32_t u, int lane) {
  const uint32_t y = xor_lane<(1 << LAM)>(x);
  if ((i >> LAM) & 1) {
    const uint32_t m = sibling_small<LAM>(u, ((i >> LAM) - 1) << LAM);
    return TR::g(x, y, (m >> (lane & 31)) & 1u);
  }
  return TR::f(x, y);
}

template <int LAM, class TR, bool STATS>
__device__ __forceinline__ void small_chain(uint32_t& x, int start, int i, uint32_t u,
                                            uint32_t* al, uint32_t* dummy, int lane,
                                            uint32_t& fg) {
  if constexpr (LAM >= 1) {
    if (LAM <= start) {
      x = reg_stage<LAM, TR>(x, i, u, lane);
      // lanes past the stage store into the wave's dummy words instead of masking exec
      *(lane < (1 << LAM) ? &al[(1 << LAM) - 1 + lane] : &dummy[lane]) = x;
      if constexpr (STATS) fg += 1u << LAM;
    }
    small_chain<LAM - 1, TR, STATS>(x, start, i, u, al, dummy, lane, fg);
  }
}

// Leaf pair of an even leaf i: its own LLR f(a, b) and, for both values of its bit, the
// LLR g(a, b, bit) of the odd leaf i + 1 (a, b: the two stage-1 values, in lanes 0 and 1).
template <class TR>
__device__ __forceinline__ uint32_t leaf_pair(uint32_t x, uint32_t& g0, uint32_t& g1) {
  const uint32_t y = xor_lane<1>(x);
  g0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)TR::g(x, y, false));
  g1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)TR::g(x, y, true));
  return TR::f(x, y);
}

// Stages min(top, SMALL) .. 0 in one register; every computed stage above 0 is stored for
// later leaves.  Returns the leaf LLR (stage 0 is never a parent and is not stored); for an
// even leaf also the next leaf's LLR for each value of this leaf's bit (leaf_pair).
template <int LOGN, class TR, bool STATS>
__device__ __forceinline__ uint32_t small_stages(int top, int i, uint32_t u,
                                                 const typename TR::In* __restrict__ root,
                                                 uint32_t* al, uint32_t* dummy, int lane,
                                                 uint32_t& fg, uint32_t& g0, uint32_t& g1) {
  constexpr int SM = Layout<LOGN>::SMALL;
  const int start = top < SM ? top : SM;
  const int nin = 2 << start;  // values of stage start + 1, read into lanes < nin
  const int q = lane < nin ? lane : nin - 1;
  uint32_t x;
  if (start + 1 == LOGN)
    x = TR::load(root, q);
  else
    x = al[nin - 1 + q];
  if (start > 0) small_chain<SM, TR, STATS>(x, start, i, u, al, dummy, lane, fg);
  x = (i & 1) ? reg_stage<0, TR>(x, i, u, lane) : leaf_pair<TR>(x, g0, g1);
  if constexpr (STATS) fg += 1u;
  lds_order();
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// f-stages LAM .. 1 of a continuing schedule, each stored for later leaves, then stage 0
// (an even leaf: leaf_pair).
template <int LAM, class TR, bool STATS>
__device__ __forceinline__ uint32_t f_chain(uint32_t x, uint32_t* al, uint32_t* dummy, int lane,
                                            uint32_t& fg, uint32_t& g0, uint32_t& g1) {
  if constexpr (LAM >= 1) {
    x = TR::f(x, xor_lane<(1 << LAM)>(x));
    *(lane < (1 << LAM) ? &al[(1 << LAM) - 1 + lane] : &dummy[lane]) = x;
    if constexpr (STATS) fg += 1u << LAM;
    return f_chain<LAM - 1, TR, STATS>(x, al, dummy, lane, fg, g0, g1);
  } else {
    if constexpr (STATS) fg += 1u;
    return leaf_pair<TR>(x, g0, g1);
  }
}

// The SC schedule continuing at leaf i with ctz(i) = K <= SMALL: stage K is a g-node (bit K
// of i is 1, its left sibling is the block [i - 2^K, i)) and every stage below it is an
// f-node (those bits of i are 0), so the chain is straight-line code.  Returns the leaf LLR.
template <int K, int LOGN, class TR, bool STATS>
__device__ __forceinline__ uint32_t cont_chain(int i, uint32_t u,
                                               const typename TR::In* __restrict__ root,
                                               uint32_t* al, uint32_t* dummy, int lane,
                                               uint32_t& fg, uint32_t& g0, uint32_t& g1) {
  constexpr int nin = 2 << K;  // values of stage K + 1
  const int q = lane < nin ? lane : nin - 1;
  uint32_t x;
  if constexpr (K + 1 == LOGN)
    x = TR::load(root, q);
  else
    x = al[nin - 1 + q];
  const uint32_t m = sibling_small<K>(u, i - (1 << K));
  x = TR::g(x, xor_lane<(1 << K)>(x), (m >> (lane & 31)) & 1u);
  if constexpr (K >= 1) {
    *(lane < (1 << K) ? &al[(1 << K) - 1 + lane] : &dummy[lane]) = x;
    if constexpr (STATS) fg += 1u << K;
    x = f_chain<K - 1, TR, STATS>(x, al, dummy, lane, fg, g0, g1);
  } else {
    if constexpr (STATS) fg += 1u;
  }
  lds_order();
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

template <int K, int LOGN, class TR, bool STATS>
__device__ __forceinline__ uint32_t cont_dispatch(int top, int i, uint32_t u,
                                                  const typename TR::In* __restrict__ root,
                                                  uint32_t* al, uint32_t* dummy, int lane,
                                                  uint32_t& fg, uint32_t& g0, uint32_t& g1) {
  if constexpr (K < Layout<LOGN>::SMALL) {
    if (top == K) return cont_chain<K, LOGN, TR, STATS>(i, u, root, al, dummy, lane, fg, g0, g1);
    return cont_dispatch<K + 1, LOGN, TR, STATS>(top, i, u, root, al, dummy, lane, fg, g0, g1);
  } else {
    return cont_chain<K, LOGN, TR, STATS>(i, u, root, al, dummy, lane, fg, g0, g1);
  }
}

struct FrameJob {
  const void* llr;   // N values of the frame
  uint8_t* payload;  // kp output bits
  uint8_t* status;
  scs_stats* stats;  // may be null
  int D, L;
};

// LDS words per wave: per-length counters, alpha tree, dummy words.  The decided-bit
// rows of the stack live in lane-private memory (see decode_frame), so the LDS share of a
// frame does not depend on D.
inline int lds_words_per_wave(int N, int /*D*/) { return (N + 3) / 4 + N + kWave; }

// The same for the SCS decoder, which keeps only stages 0 .. n-2 from N = 2^kTopFreeLogN up
// (Layout::ALPHA_WORDS): 3.3 KB per frame at N = 1024, 6.3 KB at N = 2048.
inline int scs_lds_words_per_wave(int N, int /*D*/) {
  return (N + 3) / 4 + (N >= (1 << kTopFreeLogN) ? N / 2 : N) + kWave;
}

constexpr int kMaxD = 64;  // stack slots are lanes

// Path keys: one 64-bit word, path metric (a non-negative value whose 32-bit pattern
// orders like the value) in the high half and key_lo in the low half, so that unsigned
// order is (PM ascending, PL descending, creation order ascending).  kNone is above every
// key (a path metric never has the all-ones pattern).
constexpr uint64_t kNone = ~0ull;

__device__ __forceinline__ uint64_t make_key(uint32_t pm, uint32_t lo) {
  return ((uint64_t)pm << 32) | lo;
}

// CRC check of a complete path (Section 2.2.5): the CRC register has no initial value and
// no final xor, so it is linear in the information bits and the check is the xor of
// per-bit contributions; `tab` holds, for every byte of the bit vector and every byte
// value, the xor of the contributions of its information bits (zero for a valid word).
// Lane w holds bits 32w..32w+31 of the path.  Returns the wave-wide xor (0: check passed).
__device__ __forceinline__ uint32_t crc_syndrome(const uint16_t* __restrict__ tab, uint32_t row,
                                                 int lane, int W, int nbytes) {
  uint32_t acc = 0u;
  if (lane < W) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int b = 4 * lane + k;
      if (b < nbytes) acc ^= tab[b * 256 + ((row >> (8 * k)) & 0xFFu)];
    }
  }
  acc ^= dpp<0xB1>(acc);
  acc ^= dpp<0x4E>(acc);
  acc ^= dpp<0x141>(acc);  // row_half_mirror: lane i pairs with the other quad
  acc ^= dpp<0x140>(acc);  // row_mirror: the other half-row
  return readlane(acc, 0) ^ readlane(acc, 16) ^ readlane(acc, 32) ^ readlane(acc, 48);
}

}  // namespace
