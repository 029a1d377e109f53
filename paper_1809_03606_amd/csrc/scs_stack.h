// The path stack of one frame in one wavefront (Section 2.2.5, Section 3.3): up to 64 NB
// slots.  Slot s lives in lane s % 64 of bank s / 64: that lane holds the slot's 64-bit key
// (make_key) in key[s / 64], and bit s % 64 of live[s / 64] says the slot holds a path.
// Every operation is wave-uniform in its result.  NB = 1 (D <= 64) is the single-bank
// stack; a larger NB serves the deep stacks of the depth study (D <= 64 NB).
#pragma once

#include <hip/hip_runtime.h>

#include "scs_device.h"
#include "scs_tree.h"

namespace {

constexpr int kMaxBanks = 4;                 // the deepest stack: 4 banks
constexpr int kMaxDepth = 64 * kMaxBanks;    // 256 slots

template <int NB>
struct PathStack {
  uint64_t key[NB];
  uint64_t live[NB];
  uint64_t cap[NB];  // the slots below D

  __device__ __forceinline__ void init(int D, uint64_t k0) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      key[b] = k0;
      live[b] = 0ull;
      const int d = D - 64 * b;
      cap[b] = d >= 64 ? ~0ull : (d > 0 ? (1ull << d) - 1ull : 0ull);
    }
    live[0] = 1ull;  // the empty path in slot 0
  }

  __device__ __forceinline__ bool lane_live(int b, int lane) const {
    return (live[b] >> lane) & 1ull;
  }

  __device__ __forceinline__ bool empty() const {
    uint64_t a = 0ull;
#pragma unroll
    for (int b = 0; b < NB; ++b) a |= live[b];
    return a == 0ull;
  }

  __device__ __forceinline__ int count() const {
    int c = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) c += __builtin_popcountll(live[b]);
    return c;
  }

  // the lowest free slot below D (the caller has checked count() < D)
  __device__ __forceinline__ int first_free() const {
    if constexpr (NB == 1) {
      return __builtin_ctzll(~live[0] & cap[0]);
    } else {
      int s = -1;
#pragma unroll
      for (int b = NB - 1; b >= 0; --b) {
        const uint64_t f = ~live[b] & cap[b];
        if (f) s = 64 * b + __builtin_ctzll(f);
      }
      return s;
    }
  }

  __device__ __forceinline__ void kill(int s) {
    if constexpr (NB == 1) {
      live[0] &= ~(1ull << s);
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (b == (s >> 6)) live[b] &= ~(1ull << (s & 63));
    }
  }

  // slot s takes key k
  __device__ __forceinline__ void put(int s, uint64_t k, int lane) {
    if constexpr (NB == 1) {
      key[0] = (lane == s) ? k : key[0];
      live[0] |= 1ull << s;
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        key[b] = (b == (s >> 6) && lane == (s & 63)) ? k : key[b];
        if (b == (s >> 6)) live[b] |= 1ull << (s & 63);
      }
    }
  }

  // The smallest live key `pk` and its slot `p`; `lb` a lower bound on every other live
  // key.  The stack is not empty.
  __device__ __forceinline__ void best(int lane, int& p, uint64_t& pk, uint64_t& lb) const {
    if constexpr (NB == 1) {
      const uint32_t kh = lane_live(0, lane) ? (uint32_t)(key[0] >> 32) : 0xFFFFFFFFu;
      const uint32_t mh = wave_min(kh);
      const uint64_t tie = ballot(kh == mh) & live[0];
      uint32_t ml;
      if (__builtin_popcountll(tie) == 1) {
        p = __builtin_ctzll(tie);
        ml = readlane((uint32_t)key[0], p);
        lb = (uint64_t)wave_min(lane != p ? kh : 0xFFFFFFFFu) << 32;
      } else {
        const uint32_t kl = ((tie >> lane) & 1ull) ? (uint32_t)key[0] : 0xFFFFFFFFu;
        ml = wave_min(kl);
        p = __builtin_ctzll(ballot(kl == ml) & tie);
        lb = make_key(mh, ml + 1u);  // the other tied keys have larger low words
      }
      pk = make_key(mh, ml);
    } else {
      uint32_t kh = 0xFFFFFFFFu;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (lane_live(b, lane)) kh = min(kh, (uint32_t)(key[b] >> 32));
      const uint32_t mh = wave_min(kh);
      uint64_t tie[NB];
      int nt = 0, tb = 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        tie[b] = ballot(lane_live(b, lane) && (uint32_t)(key[b] >> 32) == mh);
        nt += __builtin_popcountll(tie[b]);
        if (tie[b]) tb = b;
      }
      uint32_t ml;
      if (nt == 1) {
        uint64_t t = 0ull;
        uint32_t lo = 0u;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          t = (b == tb) ? tie[b] : t;
          lo = (b == tb) ? (uint32_t)key[b] : lo;
        }
        const int pl = __builtin_ctzll(t);
        p = 64 * tb + pl;
        ml = readlane(lo, pl);
        uint32_t k2 = 0xFFFFFFFFu;  // the other live keys' high words
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if (lane_live(b, lane) && !(b == tb && lane == pl))
            k2 = min(k2, (uint32_t)(key[b] >> 32));
        lb = (uint64_t)wave_min(k2) << 32;
      } else {
        uint32_t kl = 0xFFFFFFFFu;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if ((tie[b] >> lane) & 1ull) kl = min(kl, (uint32_t)key[b]);
        ml = wave_min(kl);
        p = 0;
#pragma unroll
        for (int b = NB - 1; b >= 0; --b) {  // the low words of live keys are distinct
          const uint64_t m = ballot(((tie[b] >> lane) & 1ull) && (uint32_t)key[b] == ml);
          if (m) p = 64 * b + __builtin_ctzll(m);
        }
        lb = make_key(mh, ml + 1u);
      }
      pk = make_key(mh, ml);
    }
  }

  // The largest live key `k` and its slot `s`.  The stack is not empty.
  __device__ __forceinline__ void worst(int lane, int& s, uint64_t& k) const {
    if constexpr (NB == 1) {
      const uint32_t xh = lane_live(0, lane) ? (uint32_t)(key[0] >> 32) : 0u;
      const uint32_t Mh = wave_max(xh);
      const uint64_t tq = ballot(xh == Mh) & live[0];
      uint32_t Ml;
      if (__builtin_popcountll(tq) == 1) {
        s = __builtin_ctzll(tq);
        Ml = readlane((uint32_t)key[0], s);
      } else {
        const uint32_t xl = ((tq >> lane) & 1ull) ? (uint32_t)key[0] : 0u;
        Ml = wave_max(xl);
        s = __builtin_ctzll(ballot(xl == Ml) & tq);
      }
      k = make_key(Mh, Ml);
    } else {
      uint32_t xh = 0u;
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (lane_live(b, lane)) xh = max(xh, (uint32_t)(key[b] >> 32));
      const uint32_t Mh = wave_max(xh);
      uint64_t tq[NB];
      int nt = 0, tb = 0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        tq[b] = ballot(lane_live(b, lane) && (uint32_t)(key[b] >> 32) == Mh);
        nt += __builtin_popcountll(tq[b]);
        if (tq[b]) tb = b;
      }
      uint32_t Ml;
      if (nt == 1) {
        uint64_t t = 0ull;
        uint32_t lo = 0u;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          t = (b == tb) ? tq[b] : t;
          lo = (b == tb) ? (uint32_t)key[b] : lo;
        }
        const int sl = __builtin_ctzll(t);
        s = 64 * tb + sl;
        Ml = readlane(lo, sl);
      } else {
        uint32_t xl = 0u;
#pragma unroll
        for (int b = 0; b < NB; ++b)
          if ((tq[b] >> lane) & 1ull) xl = max(xl, (uint32_t)key[b]);
        Ml = wave_max(xl);
        s = 0;
#pragma unroll
        for (int b = NB - 1; b >= 0; --b) {
          const uint64_t m = ballot(((tq[b] >> lane) & 1ull) && (uint32_t)key[b] == Ml);
          if (m) s = 64 * b + __builtin_ctzll(m);
        }
      }
      k = make_key(Mh, Ml);
    }
  }

  // slot s, which holds a path, takes key k (the path is replaced by its first child)
  __device__ __forceinline__ void rekey(int s, uint64_t k, int lane) {
    if constexpr (NB == 1) {
      key[0] = (lane == s) ? k : key[0];
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b) key[b] = (b == (s >> 6) && lane == (s & 63)) ? k : key[b];
    }
  }

  // L-counter pruning: drop every path of length <= i
  __device__ __forceinline__ void prune(int N, int i) {
#pragma unroll
    for (int b = 0; b < NB; ++b)
      live[b] &= ~ballot(((uint32_t)key[b] >> kSeqBits) >= (uint32_t)(N - i));
  }
};

}  // namespace
