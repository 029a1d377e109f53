// SCS decoding with several frames per wavefront (G = 16 or 32 lanes per frame).
//
// Same method and results as the one-frame-per-wavefront kernel (Aurora & Gross, Section
// 2.2.5 stack search on the reduced-memory tree of Section 3.3, eq. minsum / llrcalc /
// bitcalc / scest / PMupd), arranged so that the per-frame bookkeeping (keys, CRC
// registers, decisions, counters) runs as vector instructions shared by the 64 / G
// frames of a wavefront instead of scalar instructions per frame.
//
// Layout, per frame ("row" of G lanes, j = lane within the row):
//   * slot s of the stack = lane s mod G, register s / G (S registers per lane);
//   * bit vectors (decided bits, partial sums, outputs): word w = lane w mod G,
//     register w / G (WR registers);
//   * alpha stages in LDS (stage lambda at offset 2^lambda - 1); stages with
//     Lambda <= G also pass through one register per row within an iteration (value e in
//     lane e, partner in lane e xor Lambda); larger stages are computed G values at a time;
//   * a copy of the in-place partial sums in LDS feeds the g operations;
//   * per-frame control values are held redundantly by all lanes of the row.
// Every data-dependent choice is a per-row predicate; a step is issued when any row of
// the wavefront needs it.
#include <hip/hip_runtime.h>

#include "scs_device.h"
#include "scs_launch.h"

namespace {

template <int G>
__device__ __forceinline__ uint32_t row_min(uint32_t v) {
  v = min(v, dpp<0xB1>(v));
  v = min(v, dpp<0x4E>(v));
  v = min(v, dpp<0x141>(v));
  v = min(v, dpp<0x140>(v));
  if constexpr (G == 32) v = min(v, xor_lane<16>(v));
  return v;
}

template <int G>
__device__ __forceinline__ uint32_t row_max(uint32_t v) {
  v = max(v, dpp<0xB1>(v));
  v = max(v, dpp<0x4E>(v));
  v = max(v, dpp<0x141>(v));
  v = max(v, dpp<0x140>(v));
  if constexpr (G == 32) v = max(v, xor_lane<16>(v));
  return v;
}

// Lane j0 (row-relative, may differ between rows) of the caller's row.
template <int G>
__device__ __forceinline__ uint32_t row_read(uint32_t v, int j0) {
  const int src = (lane_id() & ~(G - 1)) | (j0 & (G - 1));
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}

// The caller's row of a wave ballot.
template <int G>
__device__ __forceinline__ uint32_t row_bits(uint64_t m) {
  const uint64_t x = m >> (lane_id() & ~(G - 1));
  return G == 32 ? (uint32_t)x : ((uint32_t)x & 0xFFFFu);
}

// Bits [0, lim) of word w.
__device__ __forceinline__ uint32_t word_mask(int w, int lim) {
  const int lo = w * 32;
  if (lo + 32 <= lim) return 0xFFFFFFFFu;
  if (lo >= lim) return 0u;
  return (1u << (lim - lo)) - 1u;
}

// Word w (per row) of a row-distributed bit vector, delivered to every lane of the row.
template <int G, int WR>
__device__ __forceinline__ uint32_t row_word(const uint32_t (&v)[WR], int w) {
  uint32_t sel = v[0];
#pragma unroll
  for (int k = 1; k < WR; ++k) sel = (w / G == k) ? v[k] : sel;
  return row_read<G>(sel, w & (G - 1));
}

template <int G>
constexpr int log2c() {
  return G == 16 ? 4 : 5;
}

// Cross-word folds of beta_push for levels LAM .. LOGN-1 (half-block of 2^(LAM-5) words).
template <int LAM, int LOGN, int G, int WR>
__device__ __forceinline__ void push_cross(uint32_t (&beta)[WR], int pos, int t, bool pred, int j) {
  if constexpr (LAM < LOGN) {
    const bool go = pred && LAM < t;
    if (__builtin_amdgcn_ballot_w64(go)) {
      constexpr int dw = 1 << (LAM - 5);
      const int a0 = (pos >> (LAM + 1)) << (LAM + 1 - 5);
      if constexpr (dw < G) {
#pragma unroll
        for (int k = 0; k < WR; ++k) {
          const uint32_t y = xor_lane<dw>(beta[k]);
          const int w = k * G + j;
          if (go && w >= a0 && w < a0 + dw) beta[k] ^= y;
        }
      } else {
#pragma unroll
        for (int k = 0; k + dw / G < WR; ++k) {
          const int w = k * G + j;
          if (go && w >= a0 && w < a0 + dw) beta[k] ^= beta[k + dw / G];
        }
      }
    }
    push_cross<LAM + 1, LOGN, G, WR>(beta, pos, t, pred, j);
  }
}

// In-place partial sums: bit `bit` enters position pos (the path had length pos) and every
// block that it completes folds (eq. bitcalc, left half ^= right half).  Rows with
// pred = false keep their vector.
template <int LOGN, int G, int WR>
__device__ __forceinline__ void beta_push_rows(uint32_t (&beta)[WR], int pos, uint32_t bit,
                                               bool pred, int j) {
  const int w = pos >> 5;
  const int t = __builtin_ctz(~(uint32_t)pos);
#pragma unroll
  for (int k = 0; k < WR; ++k) {
    uint32_t x = beta[k];
    x = (x & ~(1u << (pos & 31))) | (bit << (pos & 31));
#pragma unroll
    for (int lam = 0; lam < 5; ++lam) {
      if (lam < t) {
        const int half = 1 << lam;
        const int start = ((pos >> (lam + 1)) << (lam + 1)) & 31;
        x ^= (x >> half) & (((1u << half) - 1u) << start);
      }
    }
    if (pred && k * G + j == w) beta[k] = x;
  }
  if constexpr (LOGN > 5) push_cross<5, LOGN, G, WR>(beta, pos, t, pred, j);
}

template <int S, int LOGN, int G, int WR>
__device__ __forceinline__ void build_cross(uint32_t (&x)[WR], int PL, int j) {
  if constexpr (S < LOGN) {
    constexpr int dw = 1 << (S - 5);
    const int limw = (PL >> (S + 1)) << (S + 1 - 5);
    if constexpr (dw < G) {
#pragma unroll
      for (int k = 0; k < WR; ++k) {
        const uint32_t y = xor_lane<dw>(x[k]);
        const int w = k * G + j;
        if (!(w & dw) && w < limw) x[k] ^= y;
      }
    } else {
#pragma unroll
      for (int k = 0; k + dw / G < WR; ++k) {
        const int w = k * G + j;
        if (!(w & dw) && w < limw) x[k] ^= x[k + dw / G];
      }
    }
    build_cross<S + 1, LOGN, G, WR>(x, PL, j);
  }
}

// In-place partial sums of the first PL bits of u from scratch (butterfly stage s inside
// every complete aligned block of 2^(s+1) positions below PL); written for pred rows.
template <int LOGN, int G, int WR>
__device__ __forceinline__ void beta_build_rows(uint32_t (&beta)[WR], const uint32_t (&u)[WR],
                                                int PL, bool pred, int j) {
  constexpr uint32_t kLow[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu,
                                0x0000FFFFu};
  uint32_t x[WR];
#pragma unroll
  for (int k = 0; k < WR; ++k) x[k] = u[k] & word_mask(k * G + j, PL);
#pragma unroll
  for (int s = 0; s < (LOGN < 5 ? LOGN : 5); ++s) {
    const int lim = (PL >> (s + 1)) << (s + 1);
#pragma unroll
    for (int k = 0; k < WR; ++k) x[k] ^= (x[k] >> (1 << s)) & kLow[s] & word_mask(k * G + j, lim);
  }
  if constexpr (LOGN > 5) build_cross<5, LOGN, G, WR>(x, PL, j);
#pragma unroll
  for (int k = 0; k < WR; ++k)
    if (pred) beta[k] = x[k];
}

// Big stages (Lambda > G), from LAM down to SG + 1, for rows with top >= lambda.
template <int LAM, int SG, int LOGN, int G, class TR>
__device__ __forceinline__ void big_rows(bool ext, int top, int i, const typename TR::In* root,
                                         uint32_t* al, const uint32_t* bl, int j, uint32_t& fg) {
  if constexpr (LAM > SG) {
    const bool need = ext && top >= LAM;
    if (__builtin_amdgcn_ballot_w64(need)) {
      constexpr int Lam = 1 << LAM;
      const bool odd = (i >> LAM) & 1;
      const int base = ((i >> LAM) - 1) << LAM;
      uint32_t* dst = al + (Lam - 1);
      const uint32_t* src = al + (2 * Lam - 1);
      if (need) {
#pragma unroll 4
        for (int r = 0; r < Lam / G; ++r) {
          const int e = r * G + j;
          uint32_t pa, pb;
          if constexpr (LAM + 1 == LOGN) {
            pa = TR::load(root, e);
            pb = TR::load(root, e + Lam);
          } else {
            pa = src[e];
            pb = src[e + Lam];
          }
          uint32_t v;
          if (!odd) {
            v = TR::f(pa, pb);
          } else {
            const int q = base + e;
            v = TR::g(pa, pb, (bl[q >> 5] >> (q & 31)) & 1u);
          }
          dst[e] = v;
        }
        fg += (uint32_t)Lam;
      }
      lds_order();
    }
    big_rows<LAM - 1, SG, LOGN, G, TR>(ext, top, i, root, al, bl, j, fg);
  }
}

// Register chain of the small stages LAM .. 0 (Lambda <= G), rows with lambda <= start.
template <int LAM, class TR>
__device__ __forceinline__ void small_rows(uint32_t& x, bool ext, int start, int i, uint32_t* al,
                                           const uint32_t* bl, int j, uint32_t& fg) {
  if constexpr (LAM >= 0) {
    const bool act = ext && LAM <= start;
    if (__builtin_amdgcn_ballot_w64(act)) {
      constexpr int Lam = 1 << LAM;
      const uint32_t y = xor_lane<Lam>(x);
      const bool odd = (i >> LAM) & 1;
      uint32_t v;
      if (!odd) {
        v = TR::f(x, y);
      } else {
        const int base = ((i >> LAM) - 1) << LAM;
        const uint32_t wd = (act && base >= 0) ? bl[base >> 5] : 0u;
        v = TR::g(x, y, (wd >> (((base & 31) + j) & 31)) & 1u);
      }
      if (act) {
        x = v;
        if (j < Lam) al[Lam - 1 + j] = v;
        fg += (uint32_t)Lam;
      }
    }
    small_rows<LAM - 1, TR>(x, ext, start, i, al, bl, j, fg);
  }
}

// LDS words of one frame: decided-bit rows, L counters, alpha stages, partial sums copy.
__host__ __device__ inline int rows_frame_words(int N, int D) {
  const int W = N >= 32 ? N / 32 : 1;
  return D * W + (N + 3) / 4 + N + W;
}
// Per wave, ahead of the frames: the code's information words and prefix counts.
__host__ __device__ inline int rows_table_words(int N) { return 2 * (N >= 32 ? N / 32 : 1); }

template <int LOGN, int G, int S, class TR>
__global__ __launch_bounds__(256) void scs_rows_kernel(CodeArgs code, int D, int L,
                                                       const typename TR::In* __restrict__ llr,
                                                       int64_t n_frames,
                                                       uint8_t* __restrict__ payload,
                                                       uint8_t* __restrict__ status,
                                                       scs_stats* __restrict__ stats,
                                                       int frame_words) {
  extern __shared__ uint32_t lds[];
  constexpr int N = 1 << LOGN;
  constexpr int W = N >= 32 ? N / 32 : 1;
  constexpr int WR = (W + G - 1) / G;
  constexpr int FR = kWave / G;
  constexpr int LG = log2c<G>();
  constexpr bool PAIRS = LOGN > LG;            // stage LG has a parent of 2G values
  constexpr int SG = PAIRS ? LG : LOGN - 1;    // highest stage handled in registers
  const int lane = lane_id();
  const int j = lane & (G - 1);
  const int wave = threadIdx.x >> 6;
  const int64_t frame = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * FR + (lane / G);
  const bool real = frame < n_frames;
  const int crc_bits = code.crc;

  uint32_t* wl_base = lds + wave * (rows_table_words(N) + FR * frame_words);
  uint32_t* tab_info = wl_base;
  uint32_t* tab_pre = wl_base + W;
  uint32_t* fl = wl_base + rows_table_words(N) + (lane / G) * frame_words;
  uint32_t* rows = fl;
  uint32_t* cnt32 = fl + D * W;
  uint32_t* al = cnt32 + (N + 3) / 4;
  uint32_t* bl = al + N;
  const typename TR::In* root = llr + (real ? frame : 0) * (int64_t)N;

  for (int w = lane; w < W; w += kWave) {
    tab_info[w] = code.info[w];
    tab_pre[w] = code.pre[w];
  }
  for (int q = j; q < (N + 3) / 4; q += G) cnt32[q] = 0u;
  lds_order();

  // stack slots
  uint32_t s_pm[S], s_lo[S], s_crc[S];
  int s_pl[S];
#pragma unroll
  for (int k = 0; k < S; ++k) {
    s_pm[k] = 0u;
    s_lo[k] = key_lo(N, 0, 0u);
    s_crc[k] = 0u;
    s_pl[k] = 0;
  }
  uint32_t vb = (j == 0) ? 1u : 0u;  // slot 0: the empty path

  bool done = !real;
  uint32_t st = 0u;
  int fails = 0;
  bool have_fb = false;
  uint32_t next_seq = 1;
  bool have_cand = false;
  int cand_slot = 0;
  uint32_t cand_hi = 0u, cand_lo = 0u, cand_crc = 0u;
  uint32_t lb_hi = 0u, lb_lo = 0u;
  bool have_max = false;
  int max_slot = 0;
  uint32_t max_hi = 0u, max_lo = 0u;
  int wl = -1;
  uint32_t ucur[WR], beta[WR], fb[WR], out[WR];
#pragma unroll
  for (int k = 0; k < WR; ++k) ucur[k] = beta[k] = fb[k] = out[k] = 0u;
  uint32_t n_it = 0, n_sw = 0, n_cp = 0, n_sc = 0, n_fg = 0, n_ev = 0, n_dr = 0, n_pr = 0;
  const uint32_t cap = (uint32_t)L * (uint32_t)N + (uint32_t)L + 1u;
  uint32_t guard = 0;

  while (__builtin_amdgcn_ballot_w64(!done)) {
    bool act = !done;
    if (act && guard >= cap) {  // unreachable bound (at most L N extensions, L completions)
      done = true;
      st = 0u;
      act = false;
    }
    guard += act ? 1u : 0u;
    // an empty stack ends the frame with its fallback
    const bool any_live = row_bits<G>(__builtin_amdgcn_ballot_w64(vb != 0u)) != 0u;
    if (act && !any_live) {
      st = SCS_STATUS_FALLBACK | SCS_STATUS_EXHAUSTED;
#pragma unroll
      for (int k = 0; k < WR; ++k) out[k] = fb[k];
      done = true;
      act = false;
    }

    // ---- the best path ------------------------------------------------------------
    const bool fast = act && have_cand && key_less(cand_hi, cand_lo, lb_hi, lb_lo);
    const bool need = act && !fast;
    uint32_t w_hi = cand_hi, w_lo = cand_lo, w_crc = cand_crc;
    int w_slot = cand_slot;
    if (__builtin_amdgcn_ballot_w64(need)) {
      uint32_t m = 0xFFFFFFFFu;
#pragma unroll
      for (int k = 0; k < S; ++k)
        if ((vb >> k) & 1u) m = min(m, s_pm[k]);
      const uint32_t mh = row_min<G>(m);
      uint32_t m2 = 0xFFFFFFFFu;
#pragma unroll
      for (int k = 0; k < S; ++k)
        if (((vb >> k) & 1u) && s_pm[k] == mh) m2 = min(m2, s_lo[k]);
      const uint32_t ml = row_min<G>(m2);
      uint32_t pk = 0u;
#pragma unroll
      for (int k = 0; k < S; ++k)
        if (((vb >> k) & 1u) && s_pm[k] == mh && s_lo[k] == ml)
          pk = ((uint32_t)(k * G + j + 1) << 16) | s_crc[k];
      pk = row_max<G>(pk);
      const int ws = (int)(pk >> 16) - 1;
      uint32_t m3 = 0xFFFFFFFFu;
#pragma unroll
      for (int k = 0; k < S; ++k)
        if (((vb >> k) & 1u) && k * G + j != ws) m3 = min(m3, s_pm[k]);
      const uint32_t lbh = row_min<G>(m3);
      if (need) {
        w_hi = mh;
        w_lo = ml;
        w_slot = ws;
        w_crc = pk & 0xFFFFu;
        lb_hi = lbh;
        lb_lo = 0u;
      }
    }
    const int pl = N - (int)(w_lo >> kSeqBits);
    const bool cont = act && have_cand && (w_lo & kSeqMask) == (cand_lo & kSeqMask);
    if (act && j == (w_slot & (G - 1))) vb &= ~(1u << (w_slot / G));
    if (act && have_max && max_slot == w_slot) have_max = false;
    if (act) have_cand = false;

    // ---- complete paths: the CRC decides (Section 2.2.5) --------------------------------
    const bool comp = act && pl == N;
    if (__builtin_amdgcn_ballot_w64(comp)) {
      uint32_t rw[WR];
#pragma unroll
      for (int k = 0; k < WR; ++k) {
        const int w = k * G + j;
        rw[k] = (comp && w < W) ? rows[w_slot * W + w] : 0u;
      }
      if (comp) {
        ++n_cp;
        if (crc_bits == 0 || w_crc == 0u) {
          st = SCS_STATUS_OK;
#pragma unroll
          for (int k = 0; k < WR; ++k) out[k] = rw[k];
          done = true;
        } else {
          if (!have_fb) {
#pragma unroll
            for (int k = 0; k < WR; ++k) fb[k] = rw[k];
            have_fb = true;
          }
          if (++fails >= L) {
            st = SCS_STATUS_FALLBACK;
#pragma unroll
            for (int k = 0; k < WR; ++k) out[k] = fb[k];
            done = true;
          }
        }
      }
    }

    // ---- extend the best path by one leaf -------------------------------------------
    const bool ext = act && !comp;
    if (__builtin_amdgcn_ballot_w64(ext)) {
      const int i = ext ? pl : 0;
      if (ext) {
        ++n_it;
        n_sc += (i == 0) ? (uint32_t)(N - 1) : ((2u << __builtin_ctz((uint32_t)i)) - 1u);
      }
      uint32_t old = 0u;
      if (ext && j == 0) old = atomicAdd(&cnt32[i >> 2], 1u << (8 * (i & 3)));

      // the tree follows path w_slot at leaf i
      const bool sr = ext && !cont;
      uint32_t nu[WR];
#pragma unroll
      for (int k = 0; k < WR; ++k) nu[k] = ucur[k];
      int d = 0, A = LOGN;
      if (__builtin_amdgcn_ballot_w64(sr)) {
#pragma unroll
        for (int k = 0; k < WR; ++k) {
          const int w = k * G + j;
          if (sr && w < W) nu[k] = rows[w_slot * W + w];
        }
        const int lim = wl < 0 ? 0 : (wl < i ? wl : i);
        uint32_t first = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < WR; ++k) {
          const int w = k * G + j;
          const uint32_t x = (ucur[k] ^ nu[k]) & word_mask(w, lim);
          if (x) first = min(first, (uint32_t)(w * 32 + __builtin_ctz(x)));
        }
        first = row_min<G>(first);
        d = first < (uint32_t)lim ? (int)first : lim;
        A = wl < 0 ? LOGN : (wl == i ? 0 : msb((uint32_t)(wl ^ i)) + 1);
      }
      int top;
      if (cont) {
        top = __builtin_ctz((uint32_t)i);
      } else {
        const int Bm = (d >= i) ? 0 : msb((uint32_t)(i ^ d)) + 1;
        top = (A > Bm ? A : Bm) - 1;
      }
      const bool inc = ext && (cont || (wl >= 0 && i == wl + 1 && d >= wl));
      const bool reb = ext && !inc;
      if (__builtin_amdgcn_ballot_w64(inc)) {
        const int pw = wl < 0 ? 0 : wl;
        const uint32_t wu = cont ? row_word<G, WR>(ucur, pw >> 5) : row_word<G, WR>(nu, pw >> 5);
        beta_push_rows<LOGN, G, WR>(beta, pw, (wu >> (pw & 31)) & 1u, inc, j);
      }
      if (__builtin_amdgcn_ballot_w64(reb)) beta_build_rows<LOGN, G, WR>(beta, nu, i, reb, j);
      if (sr) {
        ++n_sw;
#pragma unroll
        for (int k = 0; k < WR; ++k) ucur[k] = nu[k];
      }
#pragma unroll
      for (int k = 0; k < WR; ++k) {
        const int w = k * G + j;
        if (ext && w < W) bl[w] = beta[k];
      }
      lds_order();

      // alpha down to leaf i
      big_rows<LOGN - 1, SG, LOGN, G, TR>(ext, top, i, root, al, bl, j, n_fg);
      const int start = ext ? (top < SG ? top : SG) : -1;
      uint32_t x = 0u;
      if constexpr (PAIRS) {
        const bool r0 = ext && start == SG;
        if (__builtin_amdgcn_ballot_w64(r0)) {
          uint32_t pa = 0u, pb = 0u;
          if (r0) {
            if constexpr (SG + 1 == LOGN) {
              pa = TR::load(root, j);
              pb = TR::load(root, j + G);
            } else {
              pa = al[2 * G - 1 + j];
              pb = al[2 * G - 1 + j + G];
            }
          }
          const bool odd = (i >> SG) & 1;
          const int base = ((i >> SG) - 1) << SG;
          const uint32_t wd = (r0 && odd) ? bl[base >> 5] : 0u;
          const uint32_t v = odd ? TR::g(pa, pb, (wd >> (((base & 31) + j) & 31)) & 1u) : TR::f(pa, pb);
          if (r0) {
            x = v;
            al[G - 1 + j] = v;
            n_fg += (uint32_t)G;
          }
        }
        const bool r1 = ext && start >= 0 && start < SG;
        if (r1 && j < (2 << start)) x = al[(2 << start) - 1 + j];
      } else {
        const bool r1 = ext && start >= 0;
        if (r1 && j < (2 << start))
          x = (start + 1 == LOGN) ? TR::load(root, j) : al[(2 << start) - 1 + j];
      }
      lds_order();
      small_rows<(PAIRS ? SG - 1 : SG), TR>(x, ext, start, i, al, bl, j, n_fg);
      lds_order();
      uint32_t a0 = row_read<G>(x, 0);
      if (ext && start < 0) a0 = al[0];

      // leaf decision and children (eq. scest, eq. PMupd)
      const uint32_t iw = ext ? tab_info[i >> 5] : 0u;
      const bool info = (iw >> (i & 31)) & 1u;
      const bool h = TR::hd(a0);
      const uint32_t mag = TR::mag(a0);
      const uint32_t b0 = info ? (h ? 1u : 0u) : 0u;
      const uint32_t pm0 = (!info && h) ? TR::pm_add(w_hi, mag) : w_hi;
      const uint32_t crc0 = info ? crc_step(w_crc, b0) : w_crc;
      const uint32_t seq0 = next_seq;
      if (ext) next_seq += info ? 2u : 1u;
      const uint32_t lo0 = key_lo(N, i + 1, seq0);
      const int wi = i >> 5;
      const uint32_t bitm = 1u << (i & 31);
#pragma unroll
      for (int k = 0; k < WR; ++k) {
        const int w = k * G + j;
        if (ext && w == wi) {
          ucur[k] = (ucur[k] & ~bitm) | (b0 ? bitm : 0u);
          rows[w_slot * W + w] = ucur[k];
        }
      }
#pragma unroll
      for (int k = 0; k < S; ++k) {
        if (ext && k * G + j == w_slot) {
          s_pm[k] = pm0;
          s_lo[k] = lo0;
          s_pl[k] = i + 1;
          s_crc[k] = crc0;
          vb |= 1u << k;
        }
      }
      if (ext && have_max && key_less(max_hi, max_lo, pm0, lo0)) {
        max_hi = pm0;
        max_lo = lo0;
        max_slot = w_slot;
      }

      const bool c1 = ext && info;
      if (__builtin_amdgcn_ballot_w64(c1)) {
        const uint32_t pm1 = TR::pm_add(w_hi, mag);
        const uint32_t crc1 = crc_step(w_crc, b0 ^ 1u);
        const uint32_t lo1 = key_lo(N, i + 1, seq0 + 1u);
        int live = 0, tfree = -1;
#pragma unroll
        for (int k = S - 1; k >= 0; --k) {
          live += __builtin_popcount(row_bits<G>(__builtin_amdgcn_ballot_w64((vb >> k) & 1u)));
          const uint32_t fm = row_bits<G>(
              __builtin_amdgcn_ballot_w64(!((vb >> k) & 1u) && k * G + j < D));
          if (fm) tfree = k * G + __builtin_ctz(fm);
        }
        const bool full = live >= D;
        const bool needmax = c1 && full && !have_max;
        if (__builtin_amdgcn_ballot_w64(needmax)) {
          uint32_t xh = 0u;
#pragma unroll
          for (int k = 0; k < S; ++k)
            if ((vb >> k) & 1u) xh = max(xh, s_pm[k]);
          const uint32_t Mh = row_max<G>(xh);
          uint32_t xl = 0u;
#pragma unroll
          for (int k = 0; k < S; ++k)
            if (((vb >> k) & 1u) && s_pm[k] == Mh) xl = max(xl, s_lo[k]);
          const uint32_t Ml = row_max<G>(xl);
          uint32_t sk = 0u;
#pragma unroll
          for (int k = 0; k < S; ++k)
            if (((vb >> k) & 1u) && s_pm[k] == Mh && s_lo[k] == Ml) sk = (uint32_t)(k * G + j + 1);
          sk = row_max<G>(sk);
          if (needmax) {
            max_hi = Mh;
            max_lo = Ml;
            max_slot = (int)sk - 1;
            have_max = true;
          }
        }
        int t = -1;
        if (c1) {
          if (!full) {
            t = tfree;
            if (have_max && key_less(max_hi, max_lo, pm1, lo1)) {
              max_hi = pm1;
              max_lo = lo1;
              max_slot = t;
            }
          } else if (key_less(pm1, lo1, max_hi, max_lo)) {
            t = max_slot;
            have_max = false;
            ++n_ev;
          } else {
            ++n_dr;
          }
        }
        const bool ins = c1 && t >= 0;
#pragma unroll
        for (int k = 0; k < WR; ++k) {
          const int w = k * G + j;
          if (ins && w < W) rows[t * W + w] = ucur[k] ^ (w == wi ? bitm : 0u);
        }
#pragma unroll
        for (int k = 0; k < S; ++k) {
          if (ins && k * G + j == t) {
            s_pm[k] = pm1;
            s_lo[k] = lo1;
            s_pl[k] = i + 1;
            s_crc[k] = crc1;
            vb |= 1u << k;
          }
        }
        if (ins && key_less(pm1, lo1, lb_hi, lb_lo)) {
          lb_hi = pm1;
          lb_lo = lo1;
        }
      }
      lds_order();

      // L-counter pruning
      old = row_read<G>(old, 0);
      if (ext && (int)((old >> (8 * (i & 3))) & 0xFFu) + 1 == L) {
        ++n_pr;
#pragma unroll
        for (int k = 0; k < S; ++k)
          if (s_pl[k] <= i) vb &= ~(1u << k);
        have_max = false;
      }
      if (ext) {
        wl = i;
        have_cand = true;
        cand_slot = w_slot;
        cand_hi = pm0;
        cand_lo = lo0;
        cand_crc = crc0;
      }
    }
  }

  // output: payload = the first K - r information bits of the output path
  if (real) {
    const int kp = code.kp;
    uint8_t* dst = payload + frame * kp;
#pragma unroll
    for (int k = 0; k < WR; ++k) {
      const int w = k * G + j;
      if (w < W) {
        uint32_t iw = tab_info[w];
        int q = (int)tab_pre[w];
        const uint32_t xo = out[k];
        while (iw) {
          const int b = __builtin_ctz(iw);
          iw &= iw - 1u;
          if (q < kp) dst[q] = (uint8_t)((st ? (xo >> b) : 0u) & 1u);
          ++q;
        }
      }
    }
    if (j == 0) status[frame] = (uint8_t)st;
    if (stats && j < 8) {
      uint32_t v = n_it;
      v = j == 1 ? n_sw : v;
      v = j == 2 ? n_cp : v;
      v = j == 3 ? n_sc : v;
      v = j == 4 ? n_fg : v;
      v = j == 5 ? n_ev : v;
      v = j == 6 ? n_dr : v;
      v = j == 7 ? n_pr : v;
      reinterpret_cast<uint32_t*>(stats + frame)[j] = v;
    }
  }
}

template <int G, int S, class TR>
using RowsKernel = void (*)(CodeArgs, int, int, const typename TR::In*, int64_t, uint8_t*,
                            uint8_t*, scs_stats*, int);

template <int G, int S, class TR>
RowsKernel<G, S, TR> rows_kernel_for(int logn) {
  switch (logn) {
    case 1: return scs_rows_kernel<1, G, S, TR>;
    case 2: return scs_rows_kernel<2, G, S, TR>;
    case 3: return scs_rows_kernel<3, G, S, TR>;
    case 4: return scs_rows_kernel<4, G, S, TR>;
    case 5: return scs_rows_kernel<5, G, S, TR>;
    case 6: return scs_rows_kernel<6, G, S, TR>;
    case 7: return scs_rows_kernel<7, G, S, TR>;
    case 8: return scs_rows_kernel<8, G, S, TR>;
    case 9: return scs_rows_kernel<9, G, S, TR>;
    case 10: return scs_rows_kernel<10, G, S, TR>;
    case 11: return scs_rows_kernel<11, G, S, TR>;
  }
  return nullptr;
}

template <int G, int S, class TR>
hipError_t launch_t(const polarscs::RowsLaunch& a) {
  auto k = rows_kernel_for<G, S, TR>(a.code.logn);
  if (!k) return hipErrorInvalidValue;
  const int FR = kWave / G;
  const int fw = rows_frame_words(a.code.N, a.D);
  const int wave_words = rows_table_words(a.code.N) + FR * fw;
  const int64_t waves = (a.n_frames + FR - 1) / FR;
  const int64_t blocks = (waves + a.waves_per_block - 1) / a.waves_per_block;
  const size_t lds = (size_t)a.waves_per_block * wave_words * 4;
  (void)hipGetLastError();  // drop an error left by an earlier call of another library
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(64 * a.waves_per_block), lds, a.stream,
                     a.code, a.D, a.L, (const typename TR::In*)a.llr, a.n_frames, a.payload,
                     a.status, a.stats, fw);
  return hipGetLastError();
}

template <int G, class TR>
hipError_t launch_g(const polarscs::RowsLaunch& a) {
  const int S = (a.D + G - 1) / G;
  if (S <= 1) return launch_t<G, 1, TR>(a);
  if (S <= 2) return launch_t<G, 2, TR>(a);
  if constexpr (G == 16) return launch_t<G, 4, TR>(a);
  return hipErrorInvalidValue;
}

}  // namespace

namespace polarscs {

size_t rows_lds_bytes(int N, int D, int G, int waves_per_block) {
  const int FR = kWave / G;
  return (size_t)waves_per_block * (rows_table_words(N) + FR * rows_frame_words(N, D)) * 4;
}

hipError_t launch_rows(const RowsLaunch& a) {
  if (a.G == 16) {
    return a.dtype == SCS_LLR_F32 ? launch_g<16, TrF32>(a) : launch_g<16, TrI8>(a);
  }
  if (a.G == 32) {
    return a.dtype == SCS_LLR_F32 ? launch_g<32, TrF32>(a) : launch_g<32, TrI8>(a);
  }
  return hipErrorInvalidValue;
}

}  // namespace polarscs
