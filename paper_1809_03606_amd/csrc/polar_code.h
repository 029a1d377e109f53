// Internal definition of the opaque polar_code object, shared by the host encoder and the
// HIP launchers of this library.
#pragma once
#include <stdint.h>

#include <vector>

struct polar_code {
  int32_t N = 0;      // code length, 2^logn
  int32_t K = 0;      // information positions, CRC bits included
  int32_t crc = 0;    // 0 or 16
  int32_t logn = 0;
  int32_t systematic = 0;  // 1: the message sits in the codeword at the information set
  uint64_t uid = 0;   // process-unique id (device table caches key on it)
  std::vector<uint8_t> info;     // N bytes, 1 = information position
  std::vector<int32_t> info_pos; // K positions, ascending
  uint32_t info_words[64] = {};  // info mask, bit j of word w = position 32 w + j
  uint16_t info_prefix[64] = {}; // number of information positions before word w
  std::vector<uint16_t> crc_unit; // CRC remainder of the unit payload vector e_p, p < K - crc
  // CRC check of a decided bit vector by bytes: entry 256 b + v is the xor, over the
  // information bits set in value v of byte b (positions 8b..8b+7), of each bit's share of
  // the CRC syndrome (payload bit: its unit remainder; CRC bit: its place in the register).
  // A vector passes the check when the xor over its bytes is 0.  Empty without a CRC.
  std::vector<uint16_t> crc_syn;
  // Fast simplified schedule (Sections 2.2.2 and 3): nodes[i] = (class << 4) | lambda for
  // the first leaf i of every node, 0xFF elsewhere.  Classes: 0 R-0, 1 R-1, 2 REP, 3 SPC.
  std::vector<uint8_t> nodes;
  int32_t payload_bits() const { return K - crc; }
  int32_t words() const { return N >= 32 ? N / 32 : 1; }
};

namespace polarscs {
uint16_t crc16_payload(const uint8_t* bits, int nbits);
void build_node_table(polar_code* c);
void finish_code(polar_code* c);
void transform_packed(uint64_t* x, int N);
void encode_systematic_packed(const polar_code* c, uint64_t* x);
bool systematic_shows_message(const polar_code* c);
}
