// Host half of the C-ABI: code construction, CRC-16, host encoder.
//
// Section 2.1 of Aurora & Gross defines PC(N, K): message bits at the information set,
// zeros at the frozen set, codeword c = u F^(x)n.  The information set here comes from a
// Bhattacharyya construction (the paper uses the 3GPP sequence, which this library does
// not ship).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "polar_code.h"
#include "polarscs.h"

namespace polarscs {

namespace {

std::atomic<uint64_t> g_next_uid{1};

// Table for CRC-16 with polynomial 0x1021 processed a byte at a time, most significant
// bit first: entry v is the register after shifting the byte v through an all-zero
// register.
struct Crc16Table {
  uint16_t t[256];
  Crc16Table() {
    for (int v = 0; v < 256; ++v) {
      uint32_t r = (uint32_t)v << 8;
      for (int b = 0; b < 8; ++b) r = (r & 0x8000) ? ((r << 1) ^ 0x1021) : (r << 1);
      t[v] = (uint16_t)r;
    }
  }
};
const Crc16Table& crc_table() {
  static const Crc16Table tab;
  return tab;
}

// log of the Bhattacharyya parameter of synthetic channel j: start from the channel
// value and, from the most significant index bit down, apply the f transform
// (z -> 2z - z^2) for a 0 bit and the g transform (z -> z^2) for a 1 bit.
double log_bhattacharyya(int j, int logn, double lz0) {
  double lz = lz0;
  for (int b = logn - 1; b >= 0; --b) {
    if ((j >> b) & 1) {
      lz = 2.0 * lz;
    } else {
      // ln(2z - z^2) = ln z + ln(1 + (1 - z)), with 1 - z = -expm1(ln z)
      lz = lz + std::log1p(-std::expm1(lz));
    }
  }
  return lz;
}

}  // namespace

uint16_t crc16_payload(const uint8_t* bits, int nbits) {
  const Crc16Table& T = crc_table();
  uint16_t reg = 0;
  int k = 0;
  for (; k + 8 <= nbits; k += 8) {
    uint32_t byte = 0;
    for (int b = 0; b < 8; ++b) byte = (byte << 1) | (bits[k + b] & 1u);
    reg = (uint16_t)((reg << 8) ^ T.t[((reg >> 8) ^ byte) & 0xFF]);
  }
  for (; k < nbits; ++k) {
    const uint32_t top = ((reg >> 15) ^ bits[k]) & 1u;
    reg = (uint16_t)(reg << 1);
    if (top) reg ^= 0x1021;
  }
  return reg;
}

}  // namespace polarscs

namespace polarscs {

// Split the leaves [first, first + 2^lambda) into fast-decoding nodes, left to right: a
// block whose leaves are all frozen (R-0), all information (R-1), information only at the
// last leaf (REP, two or more leaves) or frozen only at the first leaf (SPC, four or more
// leaves) is one node; any other block is split in halves.  A leaf is R-0 or R-1.
static void split_nodes(polar_code* c, int first, int lam) {
  const int size = 1 << lam;
  int k = 0;
  for (int j = first; j < first + size; ++j) k += c->info[j];
  int cls = -1;
  if (k == 0) cls = 0;
  else if (k == size) cls = 1;
  else if (size >= 2 && k == 1 && c->info[first + size - 1]) cls = 2;
  else if (size >= 4 && k == size - 1 && !c->info[first]) cls = 3;
  if (cls >= 0) {
    c->nodes[first] = (uint8_t)((cls << 4) | lam);
    return;
  }
  split_nodes(c, first, lam - 1);
  split_nodes(c, first + size / 2, lam - 1);
}

void build_node_table(polar_code* c) {
  c->nodes.assign((size_t)c->N, 0xFF);
  split_nodes(c, 0, c->logn);
}

}  // namespace polarscs

using polarscs::crc16_payload;

extern "C" {

const char* polar_strerror(int code) {
  switch (code) {
    case POLAR_OK: return "ok";
    case POLAR_EINVAL: return "invalid argument";
    case POLAR_ENOMEM: return "out of memory";
    case POLAR_EDEVICE: return "HIP runtime error";
    case POLAR_EUNSUPPORTED: return "unsupported";
    case POLAR_ETOOLARGE: return "request exceeds the fixed scratch capacity";
  }
  return "unknown status";
}

int polar_construct(int32_t N, int32_t K, int32_t crc_bits, double design_ebn0_db,
                    polar_code** out) {
  if (!out) return POLAR_EINVAL;
  *out = nullptr;
  if (N < 2 || N > 2048 || (N & (N - 1)) != 0) return POLAR_EINVAL;
  if (K < 1 || K > N) return POLAR_EINVAL;
  if (crc_bits != 0 && crc_bits != 16) return POLAR_EINVAL;
  if (crc_bits >= K) return POLAR_EINVAL;
  if (!std::isfinite(design_ebn0_db)) return POLAR_EINVAL;

  polar_code* c = new (std::nothrow) polar_code;
  if (!c) return POLAR_ENOMEM;
  c->N = N;
  c->K = K;
  c->crc = crc_bits;
  c->logn = 0;
  while ((1 << c->logn) < N) ++c->logn;
  c->uid = polarscs::g_next_uid.fetch_add(1);

  const double lz0 = -((double)K / N) * std::pow(10.0, design_ebn0_db / 10.0);
  std::vector<double> lz(N);
  for (int j = 0; j < N; ++j) lz[j] = polarscs::log_bhattacharyya(j, c->logn, lz0);
  std::vector<int32_t> order(N);
  std::iota(order.begin(), order.end(), 0);
  // K most reliable: smallest parameter first; equal parameters prefer the larger index.
  std::partial_sort(order.begin(), order.begin() + K, order.end(), [&](int32_t a, int32_t b) {
    return lz[a] < lz[b] || (lz[a] == lz[b] && a > b);
  });
  c->info.assign(N, 0);
  for (int k = 0; k < K; ++k) c->info[order[k]] = 1;
  polarscs::finish_code(c);
  *out = c;
  return POLAR_OK;
}

int polar_construct_set(int32_t N, const uint8_t* info_mask, int32_t crc_bits,
                        polar_code** out) {
  if (!out) return POLAR_EINVAL;
  *out = nullptr;
  if (N < 2 || N > 2048 || (N & (N - 1)) != 0 || !info_mask) return POLAR_EINVAL;
  if (crc_bits != 0 && crc_bits != 16) return POLAR_EINVAL;
  int K = 0;
  for (int j = 0; j < N; ++j) {
    if (info_mask[j] > 1) return POLAR_EINVAL;
    K += info_mask[j];
  }
  if (K < 1 || crc_bits >= K) return POLAR_EINVAL;
  polar_code* c = new (std::nothrow) polar_code;
  if (!c) return POLAR_ENOMEM;
  c->N = N;
  c->K = K;
  c->crc = crc_bits;
  c->logn = 0;
  while ((1 << c->logn) < N) ++c->logn;
  c->uid = polarscs::g_next_uid.fetch_add(1);
  c->info.assign(info_mask, info_mask + N);
  polarscs::finish_code(c);
  *out = c;
  return POLAR_OK;
}

}  // extern "C"

namespace polarscs {

// Everything a code needs once its information set is chosen: positions, bit words, CRC
// tables and the fast simplified schedule.
void finish_code(polar_code* c) {
  const int N = c->N, K = c->K, crc_bits = c->crc;
  for (int j = 0; j < N; ++j)
    if (c->info[j]) c->info_pos.push_back(j);
  int run = 0;
  for (int w = 0; w < 64; ++w) {
    uint32_t word = 0;
    for (int b = 0; b < 32; ++b) {
      const int j = 32 * w + b;
      if (j < N && c->info[j]) word |= 1u << b;
    }
    c->info_words[w] = word;
    c->info_prefix[w] = (uint16_t)run;
    run += __builtin_popcount(word);
  }
  // The CRC has no initial value and no final xor, so it is linear over GF(2): the
  // remainder of a payload is the xor of the remainders of its one-bits.
  const int kp = c->payload_bits();
  c->crc_unit.assign(kp, 0);
  if (crc_bits) {
    std::vector<uint8_t> e(kp, 0);
    for (int p = 0; p < kp; ++p) {
      e[p] = 1;
      c->crc_unit[p] = crc16_payload(e.data(), kp);
      e[p] = 0;
    }
    // syndrome share of information rank r: payload bits contribute their remainder, the
    // CRC bits (most significant first) the register bit they must cancel
    const int nbytes = (N + 7) / 8;
    std::vector<uint16_t> share(N, 0);
    for (int r = 0; r < K; ++r)
      share[c->info_pos[r]] = r < kp ? c->crc_unit[r] : (uint16_t)(1u << (crc_bits - 1 - (r - kp)));
    // Systematic encoding: the message sits in the codeword x = u F^(x)n, where x_j is the
    // xor of u_i over every i whose index contains the bits of j.  So decided bit u_i
    // carries the shares of every information position j inside i (a subset sum).
    if (c->systematic)
      for (int b = 1; b < N; b <<= 1)
        for (int i = 0; i < N; ++i)
          if (i & b) share[i] ^= share[i ^ b];
    c->crc_syn.assign((size_t)nbytes * 256, 0);
    for (int b = 0; b < nbytes; ++b)
      for (int v = 1; v < 256; ++v) {
        const int j = __builtin_ctz((unsigned)v);
        const int pos = 8 * b + j;
        c->crc_syn[(size_t)b * 256 + v] =
            (uint16_t)(c->crc_syn[(size_t)b * 256 + (v & (v - 1))] ^ (pos < N ? share[pos] : 0));
      }
  }
  build_node_table(c);
}

// x = u F^(x)n on bits packed 64 to a word: position j takes j xor (j + d) for every
// distance d with bit d of j clear (a masked shift within a word, then whole words).
void transform_packed(uint64_t* x, int N) {
  static const uint64_t kLow[6] = {0x5555555555555555ull, 0x3333333333333333ull,
                                   0x0F0F0F0F0F0F0F0Full, 0x00FF00FF00FF00FFull,
                                   0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
  const int nw = (N + 63) / 64;
  for (int s = 0; s < 6 && (1 << s) < N; ++s)
    for (int w = 0; w < nw; ++w) x[w] ^= (x[w] >> (1 << s)) & kLow[s];
  for (int dw = 1; dw < nw; dw <<= 1)
    for (int w = 0; w < nw; ++w)
      if ((w & dw) == 0) x[w] ^= x[w + dw];
}

// The information positions, packed 64 to a word.
static void info_packed(const polar_code* c, uint64_t* m) {
  for (int w = 0; w < (c->N + 63) / 64; ++w)
    m[w] = (uint64_t)c->info_words[2 * w] | ((uint64_t)c->info_words[2 * w + 1] << 32);
}

// Systematic encoding of message v (at the information positions): u = v F^(x)n cleared
// at the frozen positions, x = u F^(x)n.
void encode_systematic_packed(const polar_code* c, uint64_t* x) {
  uint64_t m[32];
  info_packed(c, m);
  transform_packed(x, c->N);
  for (int w = 0; w < (c->N + 63) / 64; ++w) x[w] &= m[w];
  transform_packed(x, c->N);
}

// True when the systematic encoder shows every message at the information positions: the
// encoder is linear, so it suffices that each unit message comes back as itself.  Sets
// closed upwards in the bit-subset order (every constructed set) always pass.
bool systematic_shows_message(const polar_code* c) {
  const int nw = (c->N + 63) / 64;
  uint64_t m[32], x[32];
  info_packed(c, m);
  for (int p : c->info_pos) {
    std::fill(x, x + nw, 0ull);
    x[p >> 6] = 1ull << (p & 63);
    encode_systematic_packed(c, x);
    for (int w = 0; w < nw; ++w)
      if ((x[w] & m[w]) != (w == (p >> 6) ? 1ull << (p & 63) : 0ull)) return false;
  }
  return true;
}

}  // namespace polarscs

extern "C" {

int polar_code_systematic(const polar_code* code, polar_code** out) {
  if (!code || !out) return POLAR_EINVAL;
  *out = nullptr;
  if (!polarscs::systematic_shows_message(code)) return POLAR_EUNSUPPORTED;
  polar_code* c = new (std::nothrow) polar_code;
  if (!c) return POLAR_ENOMEM;
  c->N = code->N;
  c->K = code->K;
  c->crc = code->crc;
  c->logn = code->logn;
  c->systematic = 1;
  c->uid = polarscs::g_next_uid.fetch_add(1);
  c->info = code->info;
  polarscs::finish_code(c);
  *out = c;
  return POLAR_OK;
}

int polar_code_is_systematic(const polar_code* code) {
  if (!code) return POLAR_EINVAL;
  return code->systematic ? 1 : 0;
}

int polar_code_query(const polar_code* code, int32_t* N, int32_t* K, int32_t* crc_bits,
                     uint8_t* info_mask_or_null) {
  if (!code) return POLAR_EINVAL;
  if (N) *N = code->N;
  if (K) *K = code->K;
  if (crc_bits) *crc_bits = code->crc;
  if (info_mask_or_null) std::memcpy(info_mask_or_null, code->info.data(), (size_t)code->N);
  return POLAR_OK;
}

void polar_code_free(polar_code* code) { delete code; }

int polar_encode(const polar_code* code, const uint8_t* payload, uint8_t* codeword,
                 int64_t B) {
  if (!code || B < 0) return POLAR_EINVAL;
  if (B == 0) return POLAR_OK;
  if (!payload || !codeword) return POLAR_EINVAL;
  const int N = code->N, kp = code->payload_bits();
  const int nw = (N + 63) / 64;
  std::vector<uint64_t> x(nw);
  std::vector<uint8_t> msg(code->K);
  for (int64_t f = 0; f < B; ++f) {
    const uint8_t* pl = payload + f * kp;
    for (int j = 0; j < kp; ++j) msg[j] = pl[j] & 1;
    if (code->crc) {
      const uint16_t r = crc16_payload(msg.data(), kp);
      for (int j = 0; j < code->crc; ++j) msg[kp + j] = (uint8_t)((r >> (code->crc - 1 - j)) & 1);
    }
    std::fill(x.begin(), x.end(), 0);
    for (int j = 0; j < code->K; ++j)
      if (msg[j]) x[code->info_pos[j] >> 6] |= 1ull << (code->info_pos[j] & 63);
    if (code->systematic)
      polarscs::encode_systematic_packed(code, x.data());
    else
      polarscs::transform_packed(x.data(), N);  // u F^(x)n
    uint8_t* cw = codeword + f * N;
    for (int j = 0; j < N; ++j) cw[j] = (uint8_t)((x[j >> 6] >> (j & 63)) & 1);
  }
  return POLAR_OK;
}

}  // extern "C"
