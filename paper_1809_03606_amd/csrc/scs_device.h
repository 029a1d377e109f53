// Device helpers shared by the SCS decoder kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>

#include "polar_code.h"
#include "polarscs.h"

namespace polarscs {

// Kernel-argument copy of a code's tables.
struct CodeArgs {
  int32_t N, K, crc, logn, W, kp;
  int32_t systematic;  // read the payload from the re-encoded path (systematic encoding)
  uint32_t info[64];
  uint16_t pre[64];
  const uint16_t* crc_tab;  // device copy of polar_code::crc_syn (null without a CRC)
  const uint8_t* nodes;     // device copy of polar_code::nodes (fast simplified decoder),
                            // zero-padded to a multiple of 4 bytes
};

inline CodeArgs make_args(const polar_code* c) {
  CodeArgs a;
  std::memset(&a, 0, sizeof a);
  a.N = c->N;
  a.K = c->K;
  a.crc = c->crc;
  a.logn = c->logn;
  a.W = c->words();
  a.kp = c->payload_bits();
  a.systematic = c->systematic;
  std::memcpy(a.info, c->info_words, sizeof a.info);
  std::memcpy(a.pre, c->info_prefix, sizeof a.pre);
  return a;
}

}  // namespace polarscs

namespace {

using polarscs::CodeArgs;
using polarscs::make_args;


constexpr int kWave = 64;
constexpr uint32_t kSeqBits = 20;
constexpr uint32_t kSeqMask = (1u << kSeqBits) - 1;

// ------------------------------------------------------------------------------------
// Cross-lane primitives
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// v from lane (lane xor M), M a power of two <= 32.
template <int M>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  if constexpr (M == 1) {
    return dpp<0xB1>(v);  // quad_perm [1,0,3,2]
  } else if constexpr (M == 2) {
    return dpp<0x4E>(v);  // quad_perm [2,3,0,1]
  } else if constexpr (M <= 16) {
    // ds_swizzle bit mode: and_mask = 0x1F, or_mask = 0, xor_mask = M
    return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, (M << 10) | 0x1F);
  } else {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ M) << 2, (int)v);
  }
}

__device__ __forceinline__ uint32_t xor_lane_rt(uint32_t v, int m) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute((lane_id() ^ m) << 2, (int)v);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Wave-wide unsigned min / max; every lane contributes.  Butterfly over quads, then
// half-rows and rows by mirroring, then the four row results on the scalar unit.
__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
  v = min(v, dpp<0xB1>(v));
  v = min(v, dpp<0x4E>(v));
  v = min(v, dpp<0x141>(v));  // row_half_mirror
  v = min(v, dpp<0x140>(v));  // row_mirror
  return min(min(readlane(v, 0), readlane(v, 16)), min(readlane(v, 32), readlane(v, 48)));
}
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  v = max(v, dpp<0xB1>(v));
  v = max(v, dpp<0x4E>(v));
  v = max(v, dpp<0x141>(v));
  v = max(v, dpp<0x140>(v));
  return max(max(readlane(v, 0), readlane(v, 16)), max(readlane(v, 32), readlane(v, 48)));
}

__device__ __forceinline__ int msb(uint32_t x) { return 31 - __builtin_clz(x); }

// x = u F^(x)n of a bit vector held one 32-bit word per lane (lane w: bits 32w..32w+31,
// lanes >= W hold 0; Section 2.1): butterflies within each word, then between lanes.  Every
// lane of the wave takes part.
__device__ __forceinline__ uint32_t polar_transform_row(uint32_t x, int lane, int N, int W) {
  constexpr uint32_t kLow[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu, 0x0000FFFFu};
  for (int s = 0; s < 5 && (1 << s) < N; ++s) x ^= (x >> (1 << s)) & kLow[s];
  for (int dw = 1; dw < W; dw <<= 1) {
    const uint32_t y = xor_lane_rt(x, dw);
    if (!(lane & dw)) x ^= y;
  }
  return x;
}

// Bits [0, lim) of a lane-per-word bit vector.
__device__ __forceinline__ uint32_t prefix_mask(int lane, int lim) {
  const int lo = lane * 32;
  if (lo + 32 <= lim) return 0xFFFFFFFFu;
  if (lo >= lim) return 0u;
  return (1u << (lim - lo)) - 1u;
}

// ------------------------------------------------------------------------------------
// Arithmetic of the two precisions (values travel as 32-bit patterns).
// ------------------------------------------------------------------------------------
struct TrF32 {
  typedef float In;
  __device__ static __forceinline__ uint32_t load(const float* p, int64_t j) {
    return __float_as_uint(p[j]);
  }
  // f = sign(a) sign(b) min(|a|, |b|), sign from the IEEE sign bits.  The minimum of the
  // magnitudes is one v_min_f32 with absolute-value modifiers: the same value fminf gives for
  // every non-NaN input, without the two canonicalising instructions the compiler puts in
  // front of fminf for operands it cannot prove canonical (they arrive here as bit patterns).
  __device__ static __forceinline__ uint32_t f(uint32_t a, uint32_t b) {
    uint32_t m;
    asm("v_min_f32_e64 %0, |%1|, |%2|" : "=v"(m) : "v"(a), "v"(b));
    return m | ((a ^ b) & 0x80000000u);
  }
  // g = b + (-1)^u a, one binary32 addition.
  __device__ static __forceinline__ uint32_t g(uint32_t a, uint32_t b, bool u) {
    const float fa = __uint_as_float(a);
    return __float_as_uint(__uint_as_float(b) + (u ? -fa : fa));
  }
  __device__ static __forceinline__ bool hd(uint32_t a) { return __uint_as_float(a) < 0.0f; }
  __device__ static __forceinline__ uint32_t mag(uint32_t a) { return a & 0x7FFFFFFFu; }
  __device__ static __forceinline__ uint32_t pm_add(uint32_t pm, uint32_t m) {
    return __float_as_uint(__uint_as_float(pm) + __uint_as_float(m));
  }
};

struct TrI8 {
  typedef int8_t In;
  __device__ static __forceinline__ uint32_t load(const int8_t* p, int64_t j) {
    const int v = p[j];
    return (uint32_t)(v < -127 ? -127 : v);
  }
  // f = sign(a) sign(b) min(|a|, |b|) (0 when either is 0), computed as
  // max(min(a, b), -max(a, b)), four instructions instead of nine: both >= 0 gives min(a, b);
  // both <= 0 gives -max(a, b) = min(|a|, |b|); a < 0 < b gives max(a, -b) = -min(|a|, b)
  // (and symmetrically); no overflow for the int8 range these values stay in.
  __device__ static __forceinline__ uint32_t f(uint32_t a, uint32_t b) {
    const int ia = (int)a, ib = (int)b;
    return (uint32_t)max(min(ia, ib), -max(ia, ib));
  }
  __device__ static __forceinline__ uint32_t g(uint32_t a, uint32_t b, bool u) {
    const int s = (int)b + (u ? -(int)a : (int)a);
    return (uint32_t)min(max(s, -127), 127);
  }
  __device__ static __forceinline__ bool hd(uint32_t a) { return (int)a < 0; }
  __device__ static __forceinline__ uint32_t mag(uint32_t a) { return (uint32_t)abs((int)a); }
  __device__ static __forceinline__ uint32_t pm_add(uint32_t pm, uint32_t m) {
    return min(pm + m, 32767u);
  }
};

// Order LDS accesses of different lanes: the wave's LDS operations execute in issue
// order, so only the compiler has to be kept from reordering them.
__device__ __forceinline__ void lds_order() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ uint32_t crc_step(uint32_t reg, uint32_t bit) {
  const uint32_t top = ((reg >> 15) ^ bit) & 1u;
  reg = (reg << 1) & 0xFFFFu;
  return top ? (reg ^ 0x1021u) : reg;
}

// Low word of a path key: (N - PL) in the top 12 bits (PL descending), creation order in
// the low 20 bits.  Sequence numbers stay below 1 + 2 L N <= 1,044,481 < 2^20.
__device__ __forceinline__ uint32_t key_lo(int N, int pl, uint32_t seq) {
  return ((uint32_t)(N - pl) << kSeqBits) | (seq & kSeqMask);
}

__device__ __forceinline__ bool key_less(uint32_t ah, uint32_t al_, uint32_t bh, uint32_t bl) {
  return ah < bh || (ah == bh && al_ < bl);
}


}  // namespace
