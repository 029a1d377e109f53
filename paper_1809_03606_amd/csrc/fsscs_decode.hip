// Fast simplified stack decoding (FSSCS-RM) of polar codes on gfx950.
//
// Method: Aurora & Gross, Section 4: the SCS search of Section 2.2.5 where one extension
// decodes a whole fast-decoding node (R-0, REP, R-1, SPC; Section 2.2.2) and places every
// candidate of the node's list rule (Section 2.2.4) on the stack, with one alpha tree per
// frame recomputed on a path switch (the reduced-memory scheme of Section 3.3).
//
// Mapping: as the SCS kernel (one wavefront per frame, the banked stack of scs_stack.h
// with one 64-bit key per slot, the decided bits u of slot s in lane-private memory, L
// counters and the alpha tree in LDS).  Per extension:
//   * the alpha tree is computed from the first stale stage down to the node's stage
//     lambda (not to the leaves);
//   * the node's 2^lambda LLRs sit one per lane (up to 64) or in LDS, 64 per row;
//   * the candidates follow the rules of Section 2.2.4, with these readings: least reliable
//     positions in ascending |alpha|, ties to the smaller index; SPC keeps the flip patterns
//     of its four least reliable positions that give even parity, in increasing order of
//     the pattern as a 4-bit number; R-0 and REP metrics add the node sum taken pairwise
//     with halving distance (w[j] += w[j + h], h = 2^lambda / 2, ..., 1);
//   * a candidate's bits are kept in the u domain: u = (hard decisions) re-encoded, and a
//     flip at position m adds the indicator of the subsets of m (the row m of the
//     transform), because the transform is linear and its own inverse;
//   * R-1 / SPC candidates are formed all at once, one flip mask per lane, and pushed in
//     generation order; when the stack is full after the first child, one lane-wise
//     comparison with the worst key drops every candidate that could not enter it (a full
//     stack stays full and its worst key only falls while the node's candidates arrive).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "polarscs.h"
#include "scs_device.h"
#include "scs_launch.h"
#include "scs_stack.h"
#include "scs_tree.h"

namespace {

constexpr int kNodeR0 = 0, kNodeR1 = 1, kNodeRep = 2, kNodeSpc = 3;

// A value the compiler cannot prove wave-uniform (read back from a small array) that is.
__device__ __forceinline__ uint32_t uniform(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}

// Plain sum of two non-negative metric terms (the node sums; no saturation inside a sum).
__device__ __forceinline__ uint32_t term_add(TrF32, uint32_t a, uint32_t b) {
  return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
}
__device__ __forceinline__ uint32_t term_add(TrI8, uint32_t a, uint32_t b) { return a + b; }

// Stages top .. bottom (both >= 6) of the tree for leaf position i, 64 values per
// instruction, as in the SCS kernel's big stages.
template <int LAM, int LOGN, class TR, bool STATS>
__device__ __forceinline__ void big_stages_to(int top, int bottom, int i, uint32_t u,
                                              const typename TR::In* __restrict__ root,
                                              uint32_t* al, int lane, uint32_t& fg) {
  if constexpr (LAM >= 6) {
    if (LAM <= top && LAM >= bottom) {
      constexpr int Lam = 1 << LAM;
      const bool odd = (i >> LAM) & 1;
      const int base = ((i >> LAM) - 1) << LAM;
      uint32_t bx = 0u;
      if (odd) bx = sibling_big<LAM>(u, base, lane);
      uint32_t* dst = al + (Lam - 1);
      const uint32_t* src = al + (2 * Lam - 1);
      if constexpr (LAM + 1 == LOGN) {
        // from the channel LLRs: lane l makes the V consecutive values V l .. V l + V - 1,
        // so each operand is V consecutive LLRs and their partial-sum bits one word
        constexpr int V = Lam / kWave;
        const int e0 = V * lane;
        const uint32_t m = odd ? lane_word(bx, (base >> 5) + (e0 >> 5)) >> (e0 & 31) : 0u;
        uint32_t x[V], y[V];
#pragma unroll
        for (int k = 0; k < V; ++k) x[k] = TR::load(root, e0 + k);
#pragma unroll
        for (int k = 0; k < V; ++k) y[k] = TR::load(root, e0 + Lam + k);
#pragma unroll
        for (int k = 0; k < V; ++k)
          dst[e0 + k] = odd ? TR::g(x[k], y[k], (m >> k) & 1u) : TR::f(x[k], y[k]);
      } else if (!odd) {
#pragma unroll
        for (int r = 0; r < Lam / kWave; ++r) {
          const int e = r * kWave + lane;
          dst[e] = TR::f(src[e], src[e + Lam]);
        }
      } else {
#pragma unroll
        for (int r = 0; r < Lam / kWave; ++r) {
          const int e = r * kWave + lane;
          const int w0 = (base >> 5) + 2 * r;
          const uint32_t mlo = readlane(bx, w0), mhi = readlane(bx, w0 + 1);
          const uint32_t m = lane < 32 ? mlo : mhi;
          const bool ub = (m >> (lane & 31)) & 1u;
          dst[e] = TR::g(src[e], src[e + Lam], ub);
        }
      }
      if constexpr (STATS) fg += (uint32_t)Lam;
      lds_order();
    }
    big_stages_to<LAM - 1, LOGN, TR, STATS>(top, bottom, i, u, root, al, lane, fg);
  }
}

// Register stages LAM .. stop (LAM <= start), each stored for later nodes.
template <int LAM, class TR, bool STATS>
__device__ __forceinline__ void small_chain_to(uint32_t& x, int start, int stop, int i,
                                               uint32_t u, uint32_t* al, uint32_t* dummy,
                                               int lane, uint32_t& fg) {
  if constexpr (LAM >= 0) {
    if (LAM <= start && LAM >= stop) {
      x = reg_stage<LAM, TR>(x, i, u, lane);
      if constexpr (LAM >= 1)
        *(lane < (1 << LAM) ? &al[(1 << LAM) - 1 + lane] : &dummy[lane]) = x;
      if constexpr (STATS) fg += 1u << LAM;
    }
    small_chain_to<LAM - 1, TR, STATS>(x, start, stop, i, u, al, dummy, lane, fg);
  }
}

// Alpha of node (lam, i >> lam) below the root: stages top .. lam (top >= lam).  For
// lam <= 5 the values come back one per lane (lane e = value e); for lam >= 6 they are
// left in LDS at al[2^lam - 1 + e].
template <int LOGN, class TR, bool STATS>
__device__ __forceinline__ uint32_t node_alpha(int top, int lam, int i, uint32_t u,
                                               const typename TR::In* __restrict__ root,
                                               uint32_t* al, uint32_t* dummy, int lane,
                                               uint32_t& fg) {
  constexpr int SM = Layout<LOGN>::SMALL;
  if (top >= 6)
    big_stages_to<LOGN - 1, LOGN, TR, STATS>(top, lam > 6 ? lam : 6, i, u, root, al, lane, fg);
  if (lam >= 6) return 0u;
  const int start = top < SM ? top : SM;
  const int nin = 2 << start;
  const int q = lane < nin ? lane : nin - 1;
  uint32_t x;
  if (start + 1 == LOGN)
    x = TR::load(root, q);
  else
    x = al[nin - 1 + q];
  small_chain_to<SM, TR, STATS>(x, start, lam, i, u, al, dummy, lane, fg);
  lds_order();
  return x;
}

// Lane-wise sum with halving distance over lanes < n (n a power of two <= 64); lane 0
// holds the result.
// Each step's distance is a compile-time constant so the exchange is a DPP or swizzle
// move; n is wave-uniform, so the skipped steps are scalar branches.
template <class TR, int H = 32>
__device__ __forceinline__ uint32_t lane_halving_sum(uint32_t w, int n) {
  if constexpr (H >= 1) {
    if (n > H) w = term_add(TR(), w, xor_lane<H>(w));
    return lane_halving_sum<TR, H / 2>(w, n);
  } else {
    return readlane(w, 0);
  }
}

// Node sums of Section 2.2.4: s0 = sum of HD(alpha)|alpha|, s1 = sum of (1 - HD(alpha))|alpha|,
// each taken pairwise with halving distance.  Up to 64 values: one per lane in x.  More:
// the values are in LDS (`vals`, n words); the first step writes the s0 terms to
// vals[0, n/2) and the s1 terms to vals[n/2, n) (each lane reads both of its inputs before
// writing them), then each half halves in place.
template <class TR>
__device__ __forceinline__ void node_sums(int lam, uint32_t x, uint32_t* vals, int lane,
                                          uint32_t& s0, uint32_t& s1) {
  const int n = 1 << lam;
  auto t0 = [](uint32_t a) -> uint32_t { return TR::hd(a) ? TR::mag(a) : 0u; };
  auto t1 = [](uint32_t a) -> uint32_t { return TR::hd(a) ? 0u : TR::mag(a); };
  if (n <= kWave) {
    s0 = lane_halving_sum<TR>(lane < n ? t0(x) : 0u, n);
    s1 = lane_halving_sum<TR>(lane < n ? t1(x) : 0u, n);
    return;
  }
  const int h0 = n / 2;
  for (int j = lane; j < h0; j += kWave) {
    const uint32_t a = vals[j], b = vals[j + h0];
    vals[j] = term_add(TR(), t0(a), t0(b));
    vals[j + h0] = term_add(TR(), t1(a), t1(b));
  }
  lds_order();
  for (int h = h0 / 2; h >= kWave; h >>= 1) {
    for (int j = lane; j < h; j += kWave) {
      vals[j] = term_add(TR(), vals[j], vals[j + h]);
      vals[h0 + j] = term_add(TR(), vals[h0 + j], vals[h0 + j + h]);
    }
    lds_order();
  }
  s0 = lane_halving_sum<TR>(vals[lane], kWave);
  s1 = lane_halving_sum<TR>(vals[h0 + lane], kWave);
}

// Position of the smallest magnitude among the node's n values (ties: the smaller
// position); `mmin` receives that magnitude.  Up to 64 values: one per lane in `mag`,
// lanes >= n holding ~0.  More: in LDS at vals[0, n).  The chosen position's magnitude is
// then replaced by ~0 so that the next call finds the next one (magnitudes are below 2^31,
// so ~0 is never chosen while a real value is left).
__device__ __forceinline__ int node_argmin_take(int n, uint32_t& mag, uint32_t* vals, int lane,
                                                uint32_t& mmin) {
  if (n <= kWave) {
    const uint32_t mb = wave_min(mag);
    const int e = __builtin_ctzll(ballot(mag == mb));
    if (lane == e) mag = 0xFFFFFFFFu;
    mmin = mb;
    return e;
  }
  uint32_t best = 0xFFFFFFFFu;
  int bidx = 0x7FFFFFFF;
  for (int e = lane; e < n; e += kWave) {
    const uint32_t m = vals[e];
    if (m < best) {
      best = m;
      bidx = e;
    }
  }
  const uint32_t mb = wave_min(best);
  const int e = (int)wave_min(best == mb ? (uint32_t)bidx : 0xFFFFFFFFu);
  lds_order();  // every lane has read its values before one of them is replaced
  if (lane == 0) vals[e] = 0xFFFFFFFFu;
  lds_order();
  mmin = mb;
  return e;
}

// Indicator of the subsets of m within a 32-bit word (row m & 31 of the transform).
__device__ __forceinline__ uint32_t subsets32(int m) {
  uint32_t x = 1u << (m & 31);
#pragma unroll
  for (int s = 0; s < 5; ++s) x ^= (x >> (1 << s)) & kLowMask[s];
  return x;
}

struct NodeBlock {
  // The node's bits in the u domain as lane-per-word values: lane w holds word w of the
  // frame's bit vector for the words the node covers (`in` marks them); a node of fewer
  // than 32 leaves is a bit field of one word, merged with the path's other bits there.
  uint32_t word;
  bool in;
};

template <int LOGN, class TR, bool STATS, int NB>
__device__ __forceinline__ void fsscs_frame(const CodeArgs& code, const FrameJob& job,
                                            uint32_t* lds) {
  using LY = Layout<LOGN>;
  constexpr int N = LY::N;
  constexpr int W = LY::W;
  const int lane = lane_id();
  const int D = job.D, L = job.L;
  const bool use_crc = code.crc != 0;
  const typename TR::In* __restrict__ root = (const typename TR::In*)job.llr;
  constexpr int kRow = 64 * NB;  // the row entry that takes the stores of lanes that must not
  uint32_t prow[kRow + 1];
  uint32_t* cnt32 = lds;
  uint32_t* al = cnt32 + (N + 3) / 4;
  uint32_t* dummy = al + N;

  const uint32_t infow = lane < W ? code.info[lane] : 0u;
  for (int j = lane; j < (N + 3) / 4; j += kWave) cnt32[j] = 0u;
  lds_order();

  PathStack<NB> S;
  S.init(D, make_key(0u, key_lo(N, 0, 0u)));
  uint32_t next_seq = 1;
  uint64_t cand = kNone, lb = 0ull;
  int cand_slot = 0;
  uint64_t maxk = kNone;
  int max_slot = 0;
  // the tree: position of the node it was last computed for, that node's stage, and the
  // bits of the path it follows; children of that extension: sequence numbers [c_lo, c_hi)
  int wl = -1, wlam = 0;
  uint32_t ucur = 0u;
  uint32_t c_lo = 0u, c_hi = 0u;

  uint32_t fb = 0u, out = 0u;
  bool have_fb = false;
  int fails = 0;
  uint32_t st = 0u;
  uint32_t n_it = 0, n_sw = 0, n_cp = 0, n_sc = 0, n_fg = 0, n_ev = 0, n_dr = 0, n_pr = 0;

  uint32_t budget = (uint32_t)L * (uint32_t)N + (uint32_t)L + 1u;
  for (;;) {
    if (budget == 0u) {
      st = 0u;
      break;
    }
    --budget;
    int p;
    uint64_t pk;
    bool cont;
    if (cand < lb) {
      p = cand_slot;
      pk = cand;
      cont = true;
    } else {
      if (S.empty()) {
        st = SCS_STATUS_FALLBACK | SCS_STATUS_EXHAUSTED;
        out = fb;
        break;
      }
      S.best(lane, p, pk, lb);
      cont = pk == cand;
    }
    // the key is wave-uniform; saying so keeps the extension in scalar control flow
    pk = make_key((uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(pk >> 32)),
                  (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)pk));
    // the slot stays live while the path is extended: its first candidate takes it over
    if (max_slot == p) maxk = kNone;
    cand = kNone;
    const uint32_t plo = (uint32_t)pk;
    const int i = N - (int)(plo >> kSeqBits);

    if (i == N) {
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

    // ---- the node at position i ---------------------------------------------------
    // one aligned word through the scalar cache (i is wave-uniform); the table is padded
    const uint32_t nw = reinterpret_cast<const uint32_t*>(code.nodes)[i >> 2];
    const uint32_t nd = (nw >> (8 * (i & 3))) & 0xffu;
    const int lam = (int)(nd & 15u), cls = (int)(nd >> 4);
    const int Lam = 1 << lam;
    if constexpr (STATS) {
      ++n_it;
      const uint32_t seq = plo & kSeqMask;
      if (!(seq >= c_lo && seq < c_hi)) ++n_sw;
      n_sc += (i == 0) ? (uint32_t)(N - Lam) : ((2u << __builtin_ctz((uint32_t)i)) - (uint32_t)Lam);
    }
    const uint32_t old = atomicAdd(lane == 0 ? &cnt32[i >> 2] : &dummy[lane],
                                   lane == 0 ? (1u << (8 * (i & 3))) : 0u);

    int top;
    if (cont) {
      top = __builtin_ctz((uint32_t)i);
    } else {
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
        if (A < wlam) A = wlam;  // stages below the last node's stage were not computed
      }
      const int Bm = (d >= i) ? 0 : msb((uint32_t)(i ^ d)) + 1;
      top = (A > Bm ? A : Bm) - 1;
      ucur = nu;
    }
    if (top < lam) top = lam;
    uint32_t xa = node_alpha<LOGN, TR, STATS>(top, lam, i, ucur, root, al, dummy, lane, n_fg);
    // the node's values: up to 64 one per lane in xa, more in LDS at vals[0, 2^lam); a node
    // that is the whole code holds the channel LLRs, copied into the (free) tree memory
    uint32_t* vals = al + (Lam - 1);
    if (lam == LOGN) {
      if (Lam > kWave) {
        for (int e = lane; e < N; e += kWave) al[e] = TR::load(root, e);
        lds_order();
        vals = al;
      } else {
        xa = TR::load(root, lane < Lam ? lane : Lam - 1);
      }
    } else if (Lam == kWave) {
      xa = vals[lane];
    }
    const bool wide = Lam > 32;  // the node covers whole words
    const uint32_t ppm = (uint32_t)(pk >> 32);

    // ---- hard decisions of the node, re-encoded into the u domain ------------------
    const int wi = i >> 5;
    uint32_t hdw = 0u;   // node of <= 32 leaves: u bits, bit e = position i + e
    uint32_t ublk = 0u;  // wider node: lane-per-word u bits of the node's words
    bool inb = false;    // lane holds one of the node's words
    if (!wide) {
      hdw = (uint32_t)ballot(lane < Lam && TR::hd(xa));
#pragma unroll
      for (int s2 = 0; s2 < 5; ++s2)
        if (s2 < lam) hdw ^= (hdw >> (1 << s2)) & kLowMask[s2];
    } else {
      inb = lane >= wi && lane < wi + (Lam >> 5);
      uint32_t v = 0u;
      for (int r = 0; r < (Lam >> 6); ++r) {
        const uint64_t b = ballot(TR::hd(Lam == kWave ? xa : vals[r * kWave + lane]));
        const int w0 = wi + 2 * r;
        v = lane == w0 ? (uint32_t)b : (lane == w0 + 1 ? (uint32_t)(b >> 32) : v);
      }
#pragma unroll
      for (int s2 = 0; s2 < 5; ++s2) v ^= (v >> (1 << s2)) & kLowMask[s2];
      // word-level steps: word w takes in word w + dw when bit dw of its offset is clear
      auto word_step = [&](auto DW) {
        constexpr int dw = decltype(DW)::value;
        const uint32_t y = xor_lane<dw>(v);
        if (!((lane - wi) & dw)) v ^= y;
      };
      if (lam > 5) word_step(std::integral_constant<int, 1>());
      if (lam > 6) word_step(std::integral_constant<int, 2>());
      if (lam > 7) word_step(std::integral_constant<int, 4>());
      if (lam > 8) word_step(std::integral_constant<int, 8>());
      if (lam > 9) word_step(std::integral_constant<int, 16>());
      if (lam > 10) word_step(std::integral_constant<int, 32>());
      ublk = v;
    }
    // parity of the hard decisions = u_0 of the node (row 0 of the transform is all ones)
    const int parity = wide ? (int)(readlane(ublk, wi) & 1u) : (int)(hdw & 1u);

    // ---- candidates (Section 2.2.4), each pushed onto the stack as it is made -------
    // Order of the node rules: R-0 one candidate; REP all-zero, then all-one; R-1 / SPC
    // every flip mask f over the least reliable positions m[0..nlr) in increasing f (SPC:
    // only masks whose flip count has the parity of the hard decisions).  Candidate c has
    // sequence number seq0 + c; the first one takes the parent's slot.
    const uint32_t seq0 = next_seq;
    const uint32_t lo0 = key_lo(N, i + Lam, seq0);
    const uint32_t fm = wide ? 0u : (Lam == 32 ? 0xFFFFFFFFu : ((1u << Lam) - 1u)) << (i & 31);
    const bool bin = wide ? inb : lane == wi;  // the lane holds a word the node writes
    uint32_t nc = 0u;
    uint64_t k0 = kNone;
    uint32_t w0 = 0u;
    // x: the candidate's u bits of the node (a bit field from bit 0 for a node of <= 32
    // leaves, else lane-per-word); pmc: its metric (wave-uniform)
    // the exact worst live key and its slot, when unknown
    auto find_worst = [&]() { S.worst(lane, max_slot, maxk); };
    // candidate c (generation order) with metric pmc and bits x
    auto push = [&](uint32_t c, uint32_t pmc, uint32_t x) {
      const uint32_t word = wide ? x : ((ucur & ~fm) | (x << (i & 31)));
      const uint64_t kc = make_key(pmc, lo0 + c);
      if (c == 0u) {
        k0 = kc;
        w0 = word;
        prow[bin ? p : kRow] = word;
        S.rekey(p, kc, lane);
        if (kc > maxk) {
          maxk = kc;
          max_slot = p;
        }
      } else {
        int t = -1;
        if (S.count() < D) {
          t = S.first_free();
          if (kc > maxk) {
            maxk = kc;
            max_slot = t;
          }
        } else {
          if (maxk == kNone) find_worst();
          if (kc < maxk) {
            t = max_slot;
            maxk = kNone;
            if constexpr (STATS) ++n_ev;
          } else {
            if constexpr (STATS) ++n_dr;
          }
        }
        if (t >= 0) {
          prow[lane < W ? t : kRow] = bin ? word : ucur;
          S.put(t, kc, lane);
          if (kc < lb) lb = kc;
        }
      }
    };

    if (cls == kNodeR0 || cls == kNodeRep) {
      uint32_t s0 = 0u, s1 = 0u;
      node_sums<TR>(lam, xa, vals, lane, s0, s1);
      push(0u, uniform(TR::pm_add(ppm, s0)), 0u);
      nc = 1u;
      if (cls == kNodeRep) {  // re-encoded all-ones: a single 1 at the node's last position
        push(1u, uniform(TR::pm_add(ppm, s1)),
             wide ? (lane == wi + (Lam >> 5) - 1 ? 0x80000000u : 0u) : 1u << (Lam - 1));
        nc = 2u;
      }
    } else {
      const int nlr = cls == kNodeR1 ? (lam >= 1 ? 2 : 1) : 4;
      uint32_t magr = lane < Lam ? TR::mag(xa) : 0xFFFFFFFFu;
      if (Lam > kWave) {  // magnitudes in place of the values (not needed again)
        for (int e = lane; e < Lam; e += kWave) vals[e] = TR::mag(vals[e]);
        lds_order();
      }
      // mm[k]: magnitude at the k-th least reliable position m; sub[k]: the u-domain
      // change of flipping it (the subsets of m: word offsets within the node that are
      // subsets of m >> 5, bits that are subsets of m & 31)
      uint32_t mm[4] = {0u, 0u, 0u, 0u}, sub[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (k < nlr) {
          const int e = node_argmin_take(Lam, magr, vals, lane, mm[k]);
          sub[k] = subsets32(e);
          if (wide) sub[k] = (((lane - wi) & ~(e >> 5)) == 0) ? sub[k] : 0u;
        }
      }
      const uint32_t xh = wide ? ublk : hdw;
      // every flip mask at once: lane f forms candidate f's metric (the same additions in
      // the same order) and, for a node of <= 32 leaves, its bit field
      uint32_t pmv = ppm, xv = xh;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if ((lane >> k) & 1) {
          pmv = TR::pm_add(pmv, mm[k]);
          xv ^= sub[k];
        }
      }
      const uint64_t fall = ballot(lane < (1 << nlr) &&
                                   (cls != kNodeSpc || (__builtin_popcount((uint32_t)lane) & 1) == parity));
      nc = (uint32_t)__builtin_popcountll(fall);
      auto x_of = [&](int f) -> uint32_t {
        if (!wide) return readlane(xv, f);
        uint32_t x = xh;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (f & (1 << k)) x ^= sub[k];
        return x;
      };
      const int f0 = __builtin_ctzll(fall);
      push(0u, readlane(pmv, f0), x_of(f0));
      uint64_t fset = fall & (fall - 1ull);
      // A full stack stays full while the candidates arrive, and its worst key can only
      // fall; so a candidate whose key is not below the worst key now is dropped whatever
      // comes before it.  One comparison over the lanes settles all of those.
      if (fset != 0ull && S.count() >= D) {
        if (maxk == kNone) find_worst();
        const uint32_t cl = (uint32_t)__builtin_popcountll(fall & ((1ull << lane) - 1ull));
        const uint64_t keep = ballot(make_key(pmv, lo0 + cl) < maxk) & fset;
        if constexpr (STATS) n_dr += (uint32_t)__builtin_popcountll(fset & ~keep);
        fset = keep;
      }
      while (fset) {
        const int f = __builtin_ctzll(fset);
        fset &= fset - 1ull;
        const uint32_t c = (uint32_t)__builtin_popcountll(fall & ((1ull << f) - 1ull));
        push(c, readlane(pmv, f), x_of(f));
      }
    }
    next_seq += nc;
    ucur = bin ? w0 : ucur;
    lds_order();

    if ((int)((readlane(old, 0) >> (8 * (i & 3))) & 0xFFu) + 1 == L) {
      if constexpr (STATS) ++n_pr;
      S.prune(N, i);
      maxk = kNone;
    }
    wl = i;
    wlam = lam;
    c_lo = seq0;
    c_hi = seq0 + nc;
    cand = k0;
    cand_slot = p;
  }

  // systematic encoding: the payload is read from the codeword (the path's bits re-encoded)
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

// The int8 kernel with one stack bank is held to 72 VGPRs (7 wavefronts per SIMD instead of
// 5 at the compiler's 84): 6 % faster on PC(1024,512), D = 32.  The same limit slows the
// binary32 kernels (74 and 77 VGPRs), which keep the compiler's choice.  The four-bank
// kernels are held to 80 VGPRs (6 per SIMD instead of 4 at the compiler's 112, a few words
// spilled): 12 % faster at D = 256.
template <class TR, int NB>
constexpr int fsscs_waves_per_simd() {
  return std::is_same<TR, TrI8>::value && NB == 1 ? 7 : NB == 4 ? 6 : 1;
}

template <int LOGN, class TR, bool STATS, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fsscs_waves_per_simd<TR, NB>())))
void fsscs_uniform_kernel(CodeArgs code, int D, int L,
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
  fsscs_frame<LOGN, TR, STATS, NB>(code, job, lds + wave * wave_words);
}

template <class TR, bool STATS>
using FsscsKernel = void (*)(CodeArgs, int, int, const typename TR::In*, int64_t, uint8_t*,
                             uint8_t*, scs_stats*, int);

template <class TR, bool STATS, int NB>
FsscsKernel<TR, STATS> fsscs_kernel_for_nb(int logn) {
  switch (logn) {
    case 1: return fsscs_uniform_kernel<1, TR, STATS, NB>;
    case 2: return fsscs_uniform_kernel<2, TR, STATS, NB>;
    case 3: return fsscs_uniform_kernel<3, TR, STATS, NB>;
    case 4: return fsscs_uniform_kernel<4, TR, STATS, NB>;
    case 5: return fsscs_uniform_kernel<5, TR, STATS, NB>;
    case 6: return fsscs_uniform_kernel<6, TR, STATS, NB>;
    case 7: return fsscs_uniform_kernel<7, TR, STATS, NB>;
    case 8: return fsscs_uniform_kernel<8, TR, STATS, NB>;
    case 9: return fsscs_uniform_kernel<9, TR, STATS, NB>;
    case 10: return fsscs_uniform_kernel<10, TR, STATS, NB>;
    case 11: return fsscs_uniform_kernel<11, TR, STATS, NB>;
    default: return nullptr;
  }
}

// banks of 64 stack slots: one up to D = 64, two up to 128, kMaxBanks above
template <class TR, bool STATS>
FsscsKernel<TR, STATS> fsscs_kernel_for(int logn, int D) {
  if (D <= 64) return fsscs_kernel_for_nb<TR, STATS, 1>(logn);
  if (D <= 128) return fsscs_kernel_for_nb<TR, STATS, 2>(logn);
  return fsscs_kernel_for_nb<TR, STATS, kMaxBanks>(logn);
}

template <class TR>
hipError_t launch_fsscs_t(const polarscs::FsscsLaunch& a) {
  const int N = a.code.N;
  const int wave_words = lds_words_per_wave(N, a.D);
  const int wpb = a.waves_per_block;
  const size_t lds = (size_t)wpb * wave_words * 4;
  const int64_t blocks = (a.n_frames + wpb - 1) / wpb;
  (void)hipGetLastError();  // drop an error left by an earlier call of another library
  if (a.stats) {
    auto k = fsscs_kernel_for<TR, true>(a.code.logn, a.D);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, a.code, a.D,
                       a.L, (const typename TR::In*)a.llr, a.n_frames, a.payload, a.status,
                       a.stats, wave_words);
  } else {
    auto k = fsscs_kernel_for<TR, false>(a.code.logn, a.D);
    if (!k) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * wpb), lds, a.stream, a.code, a.D,
                       a.L, (const typename TR::In*)a.llr, a.n_frames, a.payload, a.status,
                       a.stats, wave_words);
  }
  return hipGetLastError();
}

}  // namespace

namespace polarscs {

hipError_t launch_fsscs(const FsscsLaunch& a) {
  return a.dtype == SCS_LLR_F32 ? launch_fsscs_t<TrF32>(a) : launch_fsscs_t<TrI8>(a);
}

}  // namespace polarscs
