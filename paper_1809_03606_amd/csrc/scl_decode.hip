// Successive-cancellation list decoding with CRC selection (CA-SCL) on gfx950.
//
// Method: Aurora & Gross, Section 2.2.3 (SCL with the path metric of eq. PMupd, the CRC
// selecting among the final list) with one alpha tree per list entry (Section 3.2).
//
// Mapping: a wavefront holds LW = max(L, 8) list entries, F = LW / L frames of L entries
// each (L = 1, 2, 4 or 8; the entries of frame f are positions f L .. f L + L - 1).  The
// schedule of leaves, and with it the list size at every leaf, is the same for every
// frame of a code, so the frames of a wavefront advance in lockstep.  The LW entries share
// the 64 lanes, G = 64 / LW lanes each, and every stage of the SC schedule is computed for
// all entries at once (value e of entry p in lane p G + (e mod G)).  LDS holds, per
// physical slot (frame f owns slots f L .. f L + L - 1), the alpha tree below its top T
// stages (stage s at word offset 2^s - 1; T = 4 with one frame per wavefront, 3 with
// more), the partial sums of the left siblings of the top stages' current nodes, and the
// decided bits u (N bits); a list position points to a slot.  The top stages are
// recomputed from the channel LLRs and those partial sums whenever the first kept stage
// is computed (at leaves that are multiples of N / 2^(T + 1)), which keeps the LDS of a
// frame at about N / 2^T words per entry.  At an information leaf the 2n candidates of
// each frame (entry l with u = 0, then u = 1) sit in lanes; each finds its rank among its
// frame's candidates by key (metric, candidate number) and the L best form the frame's
// new list in rank order.  A parent's first surviving child keeps the parent's slot; any
// other child takes a free slot of its frame and copies the parent's alpha stages that
// later leaves read (above stage ctz(i + 1)) and its bits.  Partial sums of a g-node are
// the transform of the left sibling's decided bits (scratch words per entry for blocks of
// 64 bits and more).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "polarscs.h"
#include "scs_device.h"
#include "scs_launch.h"
#include "scs_tree.h"

namespace {

constexpr int kSclEntries = 8;  // list entries per wavefront (frames packed up to this)
// Top stages of the tree recomputed from the channel LLRs instead of kept per slot.  With
// one frame per wavefront every entry's recomputation reads the same LLRs, which stay in
// the caches; with several frames each frame's entries read their own, and one stage fewer
// halves those reads at twice the kept alpha words per slot.
constexpr int kSclTop = 4;
constexpr int kSclTopPacked = 3;

// List entries per wavefront for list size L.
__host__ __device__ constexpr int scl_entries(int L) { return L > kSclEntries ? L : kSclEntries; }

__host__ __device__ constexpr int scl_top(int logn, int L) {
  const int t = scl_entries(L) == L ? kSclTop : kSclTopPacked;
  return logn - 1 < t ? logn - 1 : t;
}

// Words of the partial sums kept for level k (stage n - k: the transform of the current
// node's left sibling, 2^(n-k) bits), and the per-slot words (each level padded by one) of
// the levels before k.
__host__ __device__ constexpr int scl_ps_words(int logn, int k) {
  return logn - k >= 5 ? 1 << (logn - k - 5) : 1;
}
__host__ __device__ constexpr int scl_ps_before(int logn, int k) {
  int o = 0;
  for (int j = 1; j < k; ++j) o += scl_ps_words(logn, j) + 1;
  return o;
}

// LDS words per wave of the list decoder with list size L (LW = scl_entries(L) entries and
// slots per wave): the kept alpha stages of LW slots, bit rows of LW slots, sibling scratch
// per entry, partial sums of the recomputed stages of LW slots, candidate exchange, dummy
// words.  Per-slot arrays are padded so that consecutive slots start in different banks:
// the G = 64 / LW lanes of a slot work on consecutive words of their own slot, and with
// unpadded power-of-two strides every slot's word e sits in the same bank.
__host__ __device__ inline int scl_words_per_wave(int N, int L) {
  int logn = 0;
  while ((1 << logn) < N) ++logn;
  const int LW = scl_entries(L);
  const int T = scl_top(logn, L);
  const int W = N >= 32 ? N / 32 : 1;
  const int S = N >> T;                                    // kept alpha words per slot
  const int SW = (N >> (T + 6)) > 1 ? (N >> (T + 6)) : 1;  // largest sibling block, words
  return LW * (S + kWave / LW) + LW * (W + 1) + LW * (SW + 1) + LW * scl_ps_before(logn, T + 1) +
         4 * 16 + kWave;
}

// f(integral_constant<int, s>) for s = S, S - 1, ..., 0 while s <= top.
template <int S, class F>
__device__ __forceinline__ void for_stages_desc(int top, F&& f) {
  if constexpr (S >= 0) {
    if (S <= top) f(std::integral_constant<int, S>());
    for_stages_desc<S - 1>(top, f);
  }
}

// The rank of a lane's key among the keys of its aligned group of G2 <= 16 lanes, by
// (key, lane): the number of lanes in the group with a smaller key, or an equal key and a
// lower lane.  Every other lane of the group is visited once through a DPP exchange inside
// the lane's row (lane xor m for groups of up to 8, a rotation of the 16-lane row for 16);
// the tie rule needs only whether the visited lane is the lower one, a fixed function of
// the lane number for each exchange.
template <int G2>
__device__ __forceinline__ int group_rank(uint32_t key, int lane) {
  int r = 0;
  auto count = [&](uint32_t o, bool lower) { r += (o < key || (o == key && lower)) ? 1 : 0; };
  if constexpr (G2 == 16) {
    const int g = lane & 15;
    // row_ror:n: the value of lane (g - n) mod 16 of the row, the lower lane when g >= n
    count(dpp<0x121>(key), g >= 1);
    count(dpp<0x122>(key), g >= 2);
    count(dpp<0x123>(key), g >= 3);
    count(dpp<0x124>(key), g >= 4);
    count(dpp<0x125>(key), g >= 5);
    count(dpp<0x126>(key), g >= 6);
    count(dpp<0x127>(key), g >= 7);
    count(dpp<0x128>(key), g >= 8);
    count(dpp<0x129>(key), g >= 9);
    count(dpp<0x12A>(key), g >= 10);
    count(dpp<0x12B>(key), g >= 11);
    count(dpp<0x12C>(key), g >= 12);
    count(dpp<0x12D>(key), g >= 13);
    count(dpp<0x12E>(key), g >= 14);
    count(dpp<0x12F>(key), g >= 15);
  } else {
    static_assert(G2 == 2 || G2 == 4 || G2 == 8, "groups of 2, 4, 8 or 16 lanes");
    // lane xor m is the lower lane when the lane has the highest bit of m set
    count(dpp<0xB1>(key), lane & 1);  // xor 1: quad_perm [1,0,3,2]
    if constexpr (G2 >= 4) {
      count(dpp<0x4E>(key), lane & 2);  // xor 2: quad_perm [2,3,0,1]
      count(dpp<0x1B>(key), lane & 2);  // xor 3: quad_perm [3,2,1,0]
    }
    if constexpr (G2 == 8) {
      const uint32_t m7 = dpp<0x141>(key);  // xor 7: row_half_mirror
      count(m7, lane & 4);
      count(dpp<0x1B>(m7), lane & 4);  // xor 4 = xor 7, then xor 3
      count(dpp<0x4E>(m7), lane & 4);  // xor 5 = xor 7, then xor 2
      count(dpp<0xB1>(m7), lane & 4);  // xor 6 = xor 7, then xor 1
    }
  }
  return r;
}

// Value x of stage n - K on a list entry's path at leaf i, recomputed from the channel
// LLRs (the entry's frame at root + rofs): f of the two halves of the stage above in an
// even node, g of them with the kept partial sums of the node's left sibling (level K of
// slot `slot`, L slots per level) in an odd node.
template <int LOGN, int K, class TR>
__device__ __forceinline__ uint32_t stage_rec(const typename TR::In* __restrict__ root, int rofs,
                                              int i, const uint32_t* PS, int L, int slot, int x) {
  if constexpr (K == 0) {
    return TR::load(root, rofs + x);
  } else {
    constexpr int half = 1 << (LOGN - K);
    const uint32_t a = stage_rec<LOGN, K - 1, TR>(root, rofs, i, PS, L, slot, x);
    const uint32_t b = stage_rec<LOGN, K - 1, TR>(root, rofs, i, PS, L, slot, x + half);
    if (!((i >> (LOGN - K)) & 1)) return TR::f(a, b);
    const uint32_t* ps =
        PS + L * scl_ps_before(LOGN, K) + slot * (scl_ps_words(LOGN, K) + 1);
    return TR::g(a, b, (ps[x >> 5] >> (x & 31)) & 1u);
  }
}

// The nf <= LW / L frames of one wavefront; `job` describes the first of them (the others
// follow it in the batch: LLRs N apart, payloads kp bytes apart).
template <int LOGN, class TR, bool STATS, int L, int LW>
__device__ __forceinline__ void scl_frames(const CodeArgs& code, const FrameJob& job, int nf,
                                           uint32_t* lds) {
  constexpr int N = 1 << LOGN;
  constexpr int W = N >= 32 ? N / 32 : 1;
  // The top T stages are not kept: stage n - T - 1 takes its inputs from stage_rec, the
  // same operations on the same inputs as if they had been kept.
  constexpr int T = scl_top(LOGN, L);
  constexpr int S = N >> T;
  constexpr int SW = (N >> (T + 6)) > 1 ? (N >> (T + 6)) : 1;
  const int lane = lane_id();
  // the list size and the entries per wave are compile-time constants: G lanes per entry,
  // loop trip counts and slot strides are constants
  constexpr int lgL = L == 1 ? 0 : (L == 2 ? 1 : (L == 4 ? 2 : 3));
  static_assert((1 << lgL) == L, "L is 1, 2, 4 or 8");
  constexpr int lgLW = LW == 8 ? 3 : (LW == 16 ? 4 : 5);
  static_assert((1 << lgLW) == LW && LW >= L && LW <= 16, "LW is 8 or 16, at least L");
  constexpr int F = LW / L;  // frames per wave
  constexpr int lgG = 6 - lgLW;
  constexpr int G = 1 << lgG;
  const int mypos = lane >> lgG, myj = lane & (G - 1);
  const int myp = mypos & (L - 1);  // position of the lane's entry in its frame's list
  // the lane's frame's LLRs (a frame past the end of the batch reads the last frame's)
  const int myf = mypos >> lgL;
  const int rofs = F == 1 ? 0 : (myf < nf ? myf : nf - 1) * N;
  // lane q < LW holds entry q's metric and slot; the frame of entry (or candidate) lanes
  const int qf = (lane & (LW - 1)) >> lgL;
  const int cf = (lane >> 1) >> lgL;
  // padded per-slot strides (see scl_words_per_wave)
  constexpr int SP = S + G;
  constexpr int WP = W + 1, SWP = SW + 1;
  const typename TR::In* __restrict__ root = (const typename TR::In*)job.llr;
  uint32_t* A = lds;                 // LW x SP: alpha of slot q at A + q SP (S used)
  uint32_t* U = A + LW * SP;         // LW x WP: decided bits of slot q (W used)
  uint32_t* SIB = U + LW * WP;       // LW x SWP: sibling partial sums of list entry p
  uint32_t* PS = SIB + LW * SWP;     // levels 1 .. T: LW x (words + 1) each, slot q
  uint32_t* XC = PS + LW * scl_ps_before(LOGN, T + 1);  // 2 x 32: candidate exchange
  uint32_t* dummy = XC + 64;         // kWave words

  for (int j = lane; j < LW * WP; j += kWave) U[j] = 0u;
  lds_order();

  int n = 1;                         // list size of every frame
  uint32_t pm = 0u;                  // lane q < LW, entry q in use: metric of entry q
  uint32_t phys = lane < LW ? (uint32_t)lane : 0u;  // lane q: slot of entry q
  uint32_t myslot = (uint32_t)__builtin_amdgcn_ds_bpermute(mypos << 2, (int)phys);
  uint32_t n_it = 0;
  const uint32_t infow = lane < W ? code.info[lane] : 0u;

  // the polar transform (partial sums) of the entry's 2^lg decided bits from bit b0 into
  // dst[0, max(1, 2^lg / 32)): one masked word for lg <= 5, else in-word steps and then
  // steps across words
  auto block_sums = [&](int b0, int lg, uint32_t* dst) {
    if (lg <= 5) {
      uint32_t x = U[myslot * WP + (b0 >> 5)] >> (b0 & 31);
      if (lg < 5) x &= (1u << (1 << lg)) - 1u;
      for (int t = 0; t < lg; ++t) x ^= (x >> (1 << t)) & kLowMask[t];
      *((myp < n) && myj == 0 ? dst : &dummy[lane]) = x;
    } else {
      const int nw = 1 << (lg - 5);
      for (int j = myj; j < nw; j += G) {
        uint32_t x = U[myslot * WP + (b0 >> 5) + j];
#pragma unroll
        for (int t = 0; t < 5; ++t) x ^= (x >> (1 << t)) & kLowMask[t];
        *((myp < n) ? &dst[j] : &dummy[lane]) = x;
      }
      lds_order();
      for (int d = 1; d < nw; d <<= 1) {
        for (int j = myj; j < nw; j += G) {
          const uint32_t y = (j & d) ? 0u : dst[j + d];
          if ((myp < n) && !(j & d)) dst[j] ^= y;
        }
        lds_order();
      }
    }
  };

  for (int i = 0; i < N; ++i) {
    const int top = i == 0 ? LOGN - 1 : __builtin_ctz((uint32_t)i);
    const bool active = myp < n;
    // ---- the SC schedule for every list entry: stages top .. 0 ---------------------
    // one instance of the body per stage, so that each stage's sizes are constants
    for_stages_desc<LOGN - 1>(top, [&](auto SC) {
      constexpr int s = decltype(SC)::value;
      constexpr int Lam = 1 << s;
      const bool odd = (i >> s) & 1;
      const int base = ((i >> s) - 1) << s;  // left sibling block (odd nodes)
      if constexpr (s >= LOGN - T) {  // a recomputed stage: keep its odd node's sibling sums
        if (odd) {
          constexpr int k = LOGN - s;
          block_sums(base, s, PS + LW * scl_ps_before(LOGN, k) + myslot * (scl_ps_words(LOGN, k) + 1));
        }
        lds_order();
        return;
      } else {
        uint32_t sw = 0u;  // blocks of <= 32 bits: transformed word
        if (odd) {
          if constexpr (Lam <= 32) {
            uint32_t x = U[myslot * WP + (base >> 5)] >> (base & 31);
            if constexpr (Lam < 32) x &= (1u << Lam) - 1u;
#pragma unroll
            for (int t = 0; t < s; ++t) x ^= (x >> (1 << t)) & kLowMask[t];
            sw = x;
          } else {
            constexpr int nw = Lam >> 5;
            // in-word transforms of the block's words, then across words, per entry
            for (int j = myj; j < nw; j += G) {
              uint32_t x = U[myslot * WP + (base >> 5) + j];
#pragma unroll
              for (int t = 0; t < 5; ++t) x ^= (x >> (1 << t)) & kLowMask[t];
              *(active ? &SIB[mypos * SWP + j] : &dummy[lane]) = x;
            }
            lds_order();
#pragma unroll
            for (int d = 1; d < nw; d <<= 1) {
              for (int j = myj; j < nw; j += G) {
                const uint32_t y = (j & d) ? 0u : SIB[mypos * SWP + j + d];
                if (active && !(j & d)) SIB[mypos * SWP + j] ^= y;
              }
              lds_order();
            }
          }
        }
        const int R = Lam > G ? (Lam >> lgG) : 1;
        uint32_t* dst = A + myslot * SP + (Lam - 1);
        const uint32_t* src = A + myslot * SP + (2 * Lam - 1);
        for (int r = 0; r < R; ++r) {
          const int e = r * G + myj;
          const bool ok = active && e < Lam;
          const int ee = ok ? e : 0;
          uint32_t a, b;
          if constexpr (s + T + 1 == LOGN) {  // inputs: the recomputed stage above (T = 0: LLRs)
            a = stage_rec<LOGN, T, TR>(root, rofs, i, PS, LW, myslot, ee);
            b = stage_rec<LOGN, T, TR>(root, rofs, i, PS, LW, myslot, ee + Lam);
          } else {
            a = src[ee];
            b = src[ee + Lam];
          }
          uint32_t v;
          if (!odd) {
            v = TR::f(a, b);
          } else {
            uint32_t word;
            if constexpr (Lam <= 32) word = sw;
            else word = SIB[mypos * SWP + (ee >> 5)];
            v = TR::g(a, b, (word >> (ee & 31)) & 1u);
          }
          *(ok ? &dst[ee] : &dummy[lane]) = v;
        }
        lds_order();
      }
    });
    // ---- leaf decision for every entry ------------------------------------------------
    const bool ent = lane < LW && (lane & (L - 1)) < n;  // lane q: entry q is in use
    const uint32_t a0 = ent ? A[phys * SP] : 0u;
    const bool info = (readlane(infow, i >> 5) >> (i & 31)) & 1u;
    if constexpr (STATS) n_it += (uint32_t)n;
    if (!info) {
      if (ent && TR::hd(a0)) pm = TR::pm_add(pm, TR::mag(a0));
      continue;  // u_i = 0 is already in every row
    }
    // candidates c = 2 q + u of entry q in lanes c < 2 LW; frame f's are lanes
    // 2 f L .. 2 f L + 2 L - 1
    const int cl = lane >> 1, cu = lane & 1;
    const bool cval = lane < 2 * LW && (cl & (L - 1)) < n;
    const uint32_t ca = (uint32_t)__builtin_amdgcn_ds_bpermute(cl << 2, (int)a0);
    const uint32_t cpm0 = (uint32_t)__builtin_amdgcn_ds_bpermute(cl << 2, (int)pm);
    const bool chd = TR::hd(ca);
    const uint32_t cpm = (cval && (cu != 0) != chd) ? TR::pm_add(cpm0, TR::mag(ca)) : cpm0;
    // rank among the frame's candidates (its aligned group of 2 L lanes) by (metric,
    // candidate number); unused candidates hold the largest key, above every metric, so
    // that they are never counted
    const uint32_t key = cval ? cpm : 0xFFFFFFFFu;
    const int rank = group_rank<2 * L>(key, lane);
    const int n2 = 2 * n < L ? 2 * n : L;
    const bool surv = cval && rank < n2;
    // the first child of a parent (the lower new position of the two candidates) keeps the
    // parent's slot; the two candidates of a parent are neighbouring lanes
    const bool sib_surv = xor_lane<1>((uint32_t)surv) != 0u;
    const int sib_rank = (int)xor_lane<1>((uint32_t)rank);
    const bool cfirst = surv && (!sib_surv || rank < sib_rank);
    // survivors: scatter (parent, bit, first) and the metric to their new positions
    const int npos = cf * L + rank;
    *(surv ? &XC[npos] : &dummy[lane]) = (uint32_t)(cl << 1 | cu) | (cfirst ? 0x100u : 0u);
    *(surv ? &XC[32 + npos] : &dummy[lane]) = cpm;
    // slots that stay in use: those of the parents with a surviving child
    const uint64_t sv = ballot(surv);
    uint32_t uv = (ent && ((sv >> ((lane & (LW - 1)) * 2)) & 3ull)) ? (1u << phys) : 0u;
    uv |= xor_lane<1>(uv);
    uv |= xor_lane<2>(uv);
    uv |= xor_lane<4>(uv);
    if constexpr (LW > 8) uv |= xor_lane<8>(uv);
    const uint32_t used = readlane(uv, 0);
    lds_order();
    const bool nent = lane < LW && (lane & (L - 1)) < n2;  // lane k: new entry k
    const uint32_t pcx = nent ? XC[lane] : 0u;
    const uint32_t pc = pcx & 0xFFu;                       // new entry k: 2 parent + bit
    const bool isfirst = nent && (pcx & 0x100u);
    const uint32_t npm = nent ? XC[32 + lane] : 0u;
    const int par = (int)(pc >> 1);
    const uint32_t pslot = (uint32_t)__builtin_amdgcn_ds_bpermute(par << 2, (int)phys);
    const uint64_t others = ballot(nent && !isfirst);
    // a non-first child takes its frame's free slots in increasing order, in order of new
    // position (never short: n2 <= L); it copies the parent's alpha stages that later leaves
    // read, its bit row and the kept partial sums
    uint32_t freeslots = (uint32_t)(~used) & ((1u << LW) - 1u);
    uint32_t nslot = pslot;
    const int keep_from = (i + 1 < N) ? (2 << __builtin_ctz((uint32_t)(i + 1))) - 1 : N;
    uint64_t todo = others;
    while (todo) {
      const int k = __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const uint32_t mine = F == 1 ? freeslots : freeslots & (((1u << L) - 1u) << (k & ~(L - 1)));
      const uint32_t to = (uint32_t)__builtin_ctz(mine);
      freeslots &= ~(1u << to);
      nslot = lane == k ? to : nslot;
      const uint32_t from = readlane(pslot, k);
      for (int w = keep_from + lane; w < S - 1; w += kWave) A[to * SP + w] = A[from * SP + w];
      for (int w = lane; w < W; w += kWave) U[to * WP + w] = U[from * WP + w];
      // partial sums of the recomputed stages whose current node is odd (the others are
      // rewritten before they are read)
#pragma unroll
      for (int k2 = 1; k2 <= T; ++k2) {
        if ((i >> (LOGN - k2)) & 1) {
          const int nw = scl_ps_words(LOGN, k2);
          uint32_t* ps = PS + LW * scl_ps_before(LOGN, k2);
          for (int w = lane; w < nw; w += kWave) ps[to * (nw + 1) + w] = ps[from * (nw + 1) + w];
        }
      }
    }
    lds_order();
    // bit i of every surviving entry
    if (nent && (pc & 1u)) atomicOr(&U[nslot * WP + (i >> 5)], 1u << (i & 31));
    lds_order();
    n = n2;
    pm = nent ? npm : 0u;
    phys = nent ? nslot : phys;
    // unused slots keep their numbers in the lanes of unused entries (never read)
    myslot = (uint32_t)__builtin_amdgcn_ds_bpermute(mypos << 2, (int)phys);
  }

  // ---- selection, per frame: entries in ascending (metric, position); the first to pass
  // the CRC ------------------------------------------------------------------------------
  const bool ent = lane < LW && (lane & (L - 1)) < n;
  int order = 0;
#pragma unroll
  for (int c = 0; c < LW; ++c) {
    if ((c & (L - 1)) < n) {
      const uint32_t o = readlane(pm, c);
      const bool mine = F == 1 || (c >> lgL) == qf;
      order += (mine && (o < pm || (o == pm && c < lane))) ? 1 : 0;
    }
  }
  const uint64_t entries = ballot(ent);
  for (int f = 0; f < nf; ++f) {
    const uint64_t fm = entries & ((((uint64_t)1 << L) - 1ull) << (f * L));
    uint32_t st = SCS_STATUS_OK;
    uint32_t n_cp = 0;
    int out = __builtin_ctzll(ballot(order == 0) & fm);
    if (code.crc) {
      st = SCS_STATUS_FALLBACK;
      for (int q = 0; q < n; ++q) {
        const int p = __builtin_ctzll(ballot(order == q) & fm);
        const uint32_t slot = readlane(phys, p);
        const uint32_t row = lane < W ? U[slot * WP + lane] : 0u;
        ++n_cp;
        if (crc_syndrome(code.crc_tab, row, lane, W, (N + 7) / 8) == 0u) {
          out = p;
          st = SCS_STATUS_OK;
          break;
        }
      }
    }
    const uint32_t oslot = readlane(phys, out);
    uint32_t orow = lane < W ? U[oslot * WP + lane] : 0u;
    // systematic encoding: the payload is read from the re-encoded path
    if (code.systematic) orow = polar_transform_row(orow, lane, N, W);
    if (lane < W) {
      uint32_t iw = infow;
      int k = code.pre[lane];
      uint8_t* dstp = job.payload + (int64_t)f * code.kp;
      while (iw) {
        const int b = __builtin_ctz(iw);
        iw &= iw - 1u;
        if (k < code.kp) dstp[k] = (uint8_t)((orow >> b) & 1u);
        ++k;
      }
    }
    if (lane == 0) job.status[f] = (uint8_t)st;
    if constexpr (STATS) {
      const uint32_t v[8] = {n_it, 0u, n_cp, 0u, 0u, 0u, 0u, 0u};
      if (lane < 8) {
        uint32_t x = v[0];
#pragma unroll
        for (int j = 1; j < 8; ++j) x = lane == j ? v[j] : x;
        reinterpret_cast<uint32_t*>(job.stats + f)[lane] = x;
      }
    }
  }
}

template <int LOGN, class TR, bool STATS, int L>
__global__ __launch_bounds__(256) void scl_uniform_kernel(CodeArgs code, int /*L: the template's*/,
                                                          const typename TR::In* __restrict__ llr,
                                                          int64_t n_frames,
                                                          uint8_t* __restrict__ payload,
                                                          uint8_t* __restrict__ status,
                                                          scs_stats* __restrict__ stats,
                                                          int wave_words) {
  extern __shared__ uint32_t lds[];
  constexpr int LW = scl_entries(L), F = LW / L;
  const int wave = threadIdx.x >> 6;
  const int64_t frame = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * F;
  if (frame >= n_frames) return;
  const int nf = n_frames - frame < F ? (int)(n_frames - frame) : F;
  constexpr int N = 1 << LOGN;
  FrameJob job;
  job.llr = llr + frame * N;
  job.payload = payload + frame * code.kp;
  job.status = status + frame;
  job.stats = STATS ? stats + frame : nullptr;
  job.D = 0;
  job.L = L;
  scl_frames<LOGN, TR, STATS, L, LW>(code, job, nf, lds + wave * wave_words);
}

template <class TR, bool STATS>
using SclKernel = void (*)(CodeArgs, int, const typename TR::In*, int64_t, uint8_t*, uint8_t*,
                           scs_stats*, int);

template <class TR, bool STATS, int L>
SclKernel<TR, STATS> scl_kernel_for_l(int logn) {
  switch (logn) {
    case 1: return scl_uniform_kernel<1, TR, STATS, L>;
    case 2: return scl_uniform_kernel<2, TR, STATS, L>;
    case 3: return scl_uniform_kernel<3, TR, STATS, L>;
    case 4: return scl_uniform_kernel<4, TR, STATS, L>;
    case 5: return scl_uniform_kernel<5, TR, STATS, L>;
    case 6: return scl_uniform_kernel<6, TR, STATS, L>;
    case 7: return scl_uniform_kernel<7, TR, STATS, L>;
    case 8: return scl_uniform_kernel<8, TR, STATS, L>;
    case 9: return scl_uniform_kernel<9, TR, STATS, L>;
    case 10: return scl_uniform_kernel<10, TR, STATS, L>;
    case 11: return scl_uniform_kernel<11, TR, STATS, L>;
    default: return nullptr;
  }
}

template <class TR, bool STATS>
SclKernel<TR, STATS> scl_kernel_for(int logn, int L) {
  switch (L) {
    case 1: return scl_kernel_for_l<TR, STATS, 1>(logn);
    case 2: return scl_kernel_for_l<TR, STATS, 2>(logn);
    case 4: return scl_kernel_for_l<TR, STATS, 4>(logn);
    case 8: return scl_kernel_for_l<TR, STATS, 8>(logn);
    default: return nullptr;
  }
}

template <class TR>
hipError_t launch_scl_t(const polarscs::SclLaunch& a) {
  const int wave_words = scl_words_per_wave(a.code.N, a.L);
  const int wpb = a.waves_per_block;
  const size_t lds = (size_t)wpb * wave_words * 4;
  const int64_t per_block = (int64_t)wpb * (scl_entries(a.L) / a.L);  // frames
  const int64_t blocks = (a.n_frames + per_block - 1) / per_block;
  (void)hipGetLastError();  // drop an error left by an earlier call of another library
  if (a.stats) {
    auto k = scl_kernel_for<TR, true>(a.code.logn, a.L);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, a.code, a.L,
                       (const typename TR::In*)a.llr, a.n_frames, a.payload, a.status, a.stats,
                       wave_words);
  } else {
    auto k = scl_kernel_for<TR, false>(a.code.logn, a.L);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, a.code, a.L,
                       (const typename TR::In*)a.llr, a.n_frames, a.payload, a.status, a.stats,
                       wave_words);
  }
  return hipGetLastError();
}

}  // namespace

namespace polarscs {

size_t scl_lds_bytes(int N, int L) { return (size_t)scl_words_per_wave(N, L) * 4; }

hipError_t launch_scl(const SclLaunch& a) {
  return a.dtype == SCS_LLR_F32 ? launch_scl_t<TrF32>(a) : launch_scl_t<TrI8>(a);
}

}  // namespace polarscs
