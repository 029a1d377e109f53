// Exercises every entry point of the CPU oracle on small seeded inputs, edge cases
// included (zero, saturating and huge LLRs, D = 1 and 256, L = 1 and 255, no CRC, whole-code
// nodes), for a build with the address / undefined-behaviour sanitizers or with the thread
// sanitizer (`threads` argument: concurrent batch calls on disjoint frames, the way the
// Python wrapper splits a batch).  Test infrastructure: run by tests/test_oracle_sanitize.py.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "polar_oracle.h"

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
double uniform() {  // splitmix64 -> [0, 1)
  uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

int g_fail = 0;
void check(int rc, const char* what, int N) {
  if (rc < 0) {
    std::fprintf(stderr, "%s failed (N=%d, rc=%d)\n", what, N, rc);
    g_fail = 1;
  }
}

// LLR sets for one frame: kind 0 noisy, 1 all zero, 2 saturating / huge, 3 tiny
void make_llr(int kind, int N, std::vector<float>& f, std::vector<double>& d, std::vector<int8_t>& q) {
  f.resize(N);
  d.resize(N);
  q.resize(N);
  for (int j = 0; j < N; ++j) {
    double v = 0.0;
    if (kind == 0) v = 4.0 * (uniform() - 0.3);
    if (kind == 2) v = (uniform() < 0.5 ? -1.0 : 1.0) * 1e30;
    if (kind == 3) v = (uniform() - 0.5) * 1e-30;
    f[j] = (float)v;
    d[j] = v;
    const double r = std::nearbyint(8.0 * v);
    q[j] = (int8_t)(r > 127 ? 127 : (r < -128 ? -128 : r));
  }
}

void one_code(int N, int K, int crc) {
  std::vector<uint8_t> info(N), u(N), cw(N), pay;
  check(orc_construct(N, K, 2.0, info.data()), "construct", N);
  const int kp = K - crc;
  pay.resize((size_t)2 * (kp > 0 ? kp : 1));
  for (auto& b : pay) b = uniform() < 0.5;
  std::vector<uint8_t> cw2((size_t)2 * N);
  check(orc_encode_batch(N, info.data(), crc, pay.data(), 2, cw2.data()), "encode", N);
  check(orc_encode_systematic_batch(N, info.data(), crc, pay.data(), 2, cw2.data()), "encode_sys", N);
  std::vector<int32_t> st(N), lam(N), ty(N);
  const int nodes = orc_fssc_schedule(N, info.data(), ORC_TYPES_ALL, st.data(), lam.data(), ty.data(), N);
  check(nodes, "schedule", N);
  std::vector<float> f;
  std::vector<double> d;
  std::vector<int8_t> q;
  for (int kind = 0; kind < 4; ++kind) {
    make_llr(kind, N, f, d, q);
    const void* in[3] = {f.data(), d.data(), q.data()};
    for (int mode = 0; mode < 3; ++mode) {
      uint8_t status = 0;
      double pm = 0;
      orc_stats s{};
      check(orc_sc_decode(mode, N, info.data(), in[mode], u.data(), nullptr), "sc", N);
      // the deepest stack with the largest L only on the short codes (time)
      const int DL[4][2] = {{1, 1}, {8, 2}, {64, 8}, {256, N <= 64 ? 255 : 16}};
      for (auto& dl : DL) {
        for (int sys = 0; sys < 2; ++sys) {
          check(orc_scs_decode(mode, N, info.data(), crc, dl[0], dl[1], in[mode], u.data(), &status, &pm, &s, sys), "scs", N);
          check(orc_fsscs_decode(mode, N, info.data(), crc, dl[0], dl[1], ORC_TYPES_ALL, in[mode], u.data(), &status, &pm, &s, sys), "fsscs", N);
        }
      }
      uint32_t seq[64];
      int32_t pl[64];
      double pms[64];
      check(orc_scs_trace(mode, N, info.data(), crc, 16, 4, in[mode], u.data(), &status, &pm, &s, seq, pl, pms, 64, 0), "scs_trace", N);
      check(orc_fsscs_trace(mode, N, info.data(), crc, 16, 4, ORC_TYPES_ALL, in[mode], u.data(), &status, &pm, &s, seq, pl, pms, 64, 0), "fsscs_trace", N);
      for (int L : {1, 2, 4, 8})
        check(orc_scl_decode(mode, N, info.data(), crc, L, in[mode], u.data(), &status, &pm, &s, kind & 1), "scl", N);
      (void)orc_leaf_llr(mode, N, in[mode], u.data(), N - 1);
    }
  }
  // node candidates of every class at a few sizes
  std::vector<double> alpha(64);
  std::vector<uint8_t> beta(64 * 16);
  std::vector<double> pmo(16);
  for (int lam = 0; lam <= 6; ++lam) {
    for (int j = 0; j < (1 << lam); ++j) alpha[j] = 4.0 * (uniform() - 0.5);
    for (int type = 0; type < 4; ++type)
      for (int mode = 0; mode < 3; ++mode)
        (void)orc_node_candidates(mode, type, lam, alpha.data(), 1.0, beta.data(), pmo.data(), 16);
  }
}

void batch_threads(int threads) {
  const int N = 256, K = 128, crc = 16, B = 64;
  std::vector<uint8_t> info(N);
  check(orc_construct(N, K, 2.0, info.data()), "construct", N);
  std::vector<float> llr((size_t)B * N);
  for (auto& v : llr) v = (float)(4.0 * (uniform() - 0.3));
  std::vector<uint8_t> pay((size_t)B * (K - crc)), status(B);
  std::vector<orc_stats> st(B);
  std::vector<std::thread> pool;
  const int per = B / threads;
  for (int t = 0; t < threads; ++t) {
    pool.emplace_back([&, t] {
      const int64_t f0 = (int64_t)t * per;
      const float* x = llr.data() + f0 * N;
      orc_scs_decode_batch(ORC_F32, N, info.data(), crc, 32, 8, x, per, pay.data() + f0 * (K - crc), status.data() + f0, st.data() + f0, 0);
      orc_fsscs_decode_batch(ORC_F32, N, info.data(), crc, 32, 8, ORC_TYPES_ALL, x, per, pay.data() + f0 * (K - crc), status.data() + f0, st.data() + f0, 0);
      orc_scl_decode_batch(ORC_F32, N, info.data(), crc, 4, x, per, pay.data() + f0 * (K - crc), status.data() + f0, st.data() + f0, 0);
    });
  }
  for (auto& th : pool) th.join();
}

}  // namespace

int main(int argc, char** argv) {
  const int threads = argc > 1 ? std::atoi(argv[1]) : 0;
  if (threads > 0) {
    batch_threads(threads);
  } else {
    const int codes[][3] = {{2, 1, 0}, {4, 2, 0}, {8, 4, 0}, {8, 8, 0}, {8, 1, 0}, {32, 24, 16},
                            {64, 32, 0}, {64, 40, 16}, {256, 128, 16}, {1024, 512, 16}};
    for (auto& c : codes) one_code(c[0], c[1], c[2]);
    // brute-force ML on a tiny code
    std::vector<uint8_t> info(16), mins(16 * 8);
    check(orc_construct(16, 6, 2.0, info.data()), "construct", 16);
    std::vector<double> llr(16);
    for (auto& v : llr) v = 4.0 * (uniform() - 0.3);
    double dmin = 0;
    int64_t nmin = 0;
    check(orc_ml_decode(16, info.data(), llr.data(), &dmin, &nmin, mins.data(), 8), "ml", 16);
  }
  std::printf("oracle driver done (%s)\n", threads > 0 ? "threads" : "sequential");
  return g_fail;
}
