// polar_oracle.cpp -- plain CPU reference for polar codes and SC / SCS decoding.
//
// TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
// benchmark's CPU-baseline leg to check the HIP decoder.  The product library never
// links or calls this code, and no source is shared between the two.
//
// Built with -O2, no fast-math and -ffp-contract=off, so binary32 arithmetic is plain
// IEEE round-to-nearest-even with denormals, in program order.
//
// Paper: H. Aurora, W. Gross, "Towards Practical Software Stack Decoding of Polar
// Codes".  Section numbers below refer to it.  Where the paper is silent or garbled the
// reading taken is stated at the point of use (R-numbers match the list of readings in
// the design notes).

#include "polar_oracle.h"

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <vector>

namespace {

int log2_exact(int N) {
  if (N < 2 || (N & (N - 1)) != 0) return -1;
  int n = 0;
  while ((1 << n) < N) ++n;
  return n;
}

// ---------------------------------------------------------------------------------
// Arithmetic of the LLR tree.  Section 2.2.1, eq. (minsum) and eq. (scest).
//
//   f(a, b)    = sign(a) sign(b) min(|a|, |b|)           (exact in every mode)
//   g(a, b, u) = b + (-1)^u a                             (R1: the paper prints
//                a + (-1)^u b, but its kernel figure feeds the XOR output into the
//                first input, so the sign applies to the first operand; the literal
//                formula fails noiseless decoding)
//   HD(x)      = 1 iff x < 0                              (R2: -0 and +0 decide 0)
//   PM update  : eq. (PMupd), PM += |alpha| when the decided bit disagrees with HD.
//
// The sign of f is taken from the IEEE sign bits (R3), so f(-0, 1) = -0; no decision
// depends on the sign of a zero.
// ---------------------------------------------------------------------------------
struct ArF32 {
  typedef float T;    // LLR / alpha type
  typedef float PM;   // path metric type
  static T from_f32(float x) { return x; }
  static T f(T a, T b) {
    T m = std::fabs(a) < std::fabs(b) ? std::fabs(a) : std::fabs(b);
    return (std::signbit(a) != std::signbit(b)) ? -m : m;
  }
  static T g(T a, T b, int u) { return u ? b - a : b + a; }
  static int hd(T x) { return x < 0 ? 1 : 0; }
  static PM mag(T x) { return std::fabs(x); }
  static PM pm_add(PM pm, PM m) { return pm + m; }
  static double to_double(T x) { return (double)x; }
};

struct ArF64 {
  typedef double T;
  typedef double PM;
  static T f(T a, T b) {
    T m = std::fabs(a) < std::fabs(b) ? std::fabs(a) : std::fabs(b);
    return (std::signbit(a) != std::signbit(b)) ? -m : m;
  }
  static T g(T a, T b, int u) { return u ? b - a : b + a; }
  static int hd(T x) { return x < 0 ? 1 : 0; }
  static PM mag(T x) { return std::fabs(x); }
  static PM pm_add(PM pm, PM m) { return pm + m; }
  static double to_double(T x) { return x; }
};

// Fixed point (R18): alpha is an integer in [-127, 127]; g saturates to that range;
// the path metric is a non-negative int16 that saturates at 32767.
struct ArFix {
  typedef int T;
  typedef int PM;
  static int sat127(int x) { return x > 127 ? 127 : (x < -127 ? -127 : x); }
  static T f(T a, T b) {
    int m = std::abs(a) < std::abs(b) ? std::abs(a) : std::abs(b);
    return ((a < 0) != (b < 0)) ? -m : m;
  }
  static T g(T a, T b, int u) { return sat127(u ? b - a : b + a); }
  static int hd(T x) { return x < 0 ? 1 : 0; }
  static PM mag(T x) { return std::abs(x); }
  static PM pm_add(PM pm, PM m) { int s = pm + m; return s > 32767 ? 32767 : s; }
  static double to_double(T x) { return (double)x; }
};

template <class A> typename A::T load_llr(const void* p, int j);
template <> float load_llr<ArF32>(const void* p, int j) { return ((const float*)p)[j]; }
template <> double load_llr<ArF64>(const void* p, int j) { return ((const double*)p)[j]; }
template <> int load_llr<ArFix>(const void* p, int j) {
  return ArFix::sat127((int)((const int8_t*)p)[j]);
}

// ---------------------------------------------------------------------------------
// The SC decoding tree with the memory layout of Section 3.1.
//
//   alpha memory: stage lambda holds Lambda = 2^lambda LLRs, enough for one branch;
//                 stage n holds the channel LLRs (eq. llrcalc, first line).
//   beta memory : stage lambda holds 2*Lambda bits, one half per child of the node
//                 above: node (lambda, phi) lives at offset (phi mod 2) * Lambda.
//
// Node (lambda, phi): stage lambda, branch phi in [0, 2^(n-lambda) - 1] (R4: the
// paper's "(n - lambda + 1) branches" contradicts its own figures).
// ---------------------------------------------------------------------------------
template <class A>
struct Tree {
  typedef typename A::T T;
  int n = 0, N = 0;
  std::vector<std::vector<T>> alpha;        // alpha[lambda][0..Lambda-1], alpha[n] = root
  std::vector<std::vector<uint8_t>> beta;   // beta[lambda][0..2*Lambda-1]
  uint64_t f_ops = 0, g_ops = 0;

  void init(int n_, const void* llr) {
    n = n_;
    N = 1 << n;
    alpha.assign(n + 1, std::vector<T>());
    beta.assign(n + 1, std::vector<uint8_t>());
    for (int lam = 0; lam <= n; ++lam) {
      alpha[lam].assign(1u << lam, T(0));
      beta[lam].assign(2u << lam, 0);
    }
    for (int j = 0; j < N; ++j) alpha[n][j] = load_llr<A>(llr, j);
  }

  // beta of node (lambda, phi), as stored in the stage-lambda beta memory.
  uint8_t* beta_of(int lam, int phi) { return beta[lam].data() + (phi & 1) * (1 << lam); }

  // One node of eq. (llrcalc): alpha_v from its parent p = (lambda+1, phi/2) and, for
  // odd phi, the bits of its left sibling u = (lambda, phi-1).
  void node_alpha(int lam, int phi) {
    const int Lam = 1 << lam;
    const T* ap = alpha[lam + 1].data();
    T* av = alpha[lam].data();
    if ((phi & 1) == 0) {
      for (int i = 0; i < Lam; ++i) av[i] = A::f(ap[i], ap[i + Lam]);
      f_ops += Lam;
    } else {
      const uint8_t* bu = beta_of(lam, phi - 1);
      for (int i = 0; i < Lam; ++i) av[i] = A::g(ap[i], ap[i + Lam], bu[i]);
      g_ops += Lam;
    }
  }

  // Algorithm 1, recursively_calc_alpha(lambda, phi): walk up while phi is even
  // (the parent of an even node is stale), then compute the node.
  void calc_alpha(int lam, int phi) {
    if (lam == n) return;
    if ((phi & 1) == 0) calc_alpha(lam + 1, phi >> 1);
    node_alpha(lam, phi);
  }

  // Algorithm 4, the SCS-RM variant: after a path switch every ancestor is stale, so
  // the recursion goes to the root whatever the parity (R5: the listing's loop
  // variable and its psi are taken as i = 0..Lambda-1 and psi = floor(phi/2)).
  void calc_alpha_rm(int lam, int phi, bool switched) {
    if (lam == n) return;
    if ((phi & 1) == 0 || switched) calc_alpha_rm(lam + 1, phi >> 1, switched);
    node_alpha(lam, phi);
  }

  // Algorithm 2, recursively_update_beta(lambda, phi), eq. (bitcalc): once the right
  // child (odd phi) is known, combine it with its left sibling into the parent and
  // continue upwards while the parent is itself a right child.
  void update_beta(int lam, int phi) {
    if ((phi & 1) == 0) return;
    if (lam == n) return;
    const int Lam = 1 << lam;
    const uint8_t* bl = beta_of(lam, phi - 1);
    const uint8_t* br = beta_of(lam, phi);
    uint8_t* bv = beta_of(lam + 1, phi >> 1);
    for (int i = 0; i < Lam; ++i) {
      bv[i] = bl[i] ^ br[i];
      bv[i + Lam] = br[i];
    }
    update_beta(lam + 1, phi >> 1);
  }

  // Leaf bit: beta_(0,i)[0] = u_i (R6: the paper's beta_(0,i)[i] indexes a one-bit
  // node), then propagate.
  void set_leaf(int i, uint8_t u) {
    beta_of(0, i)[0] = u;
    update_beta(0, i);
  }

  // Algorithm 3: populate beta with the first PL decided bits of a path.
  void populate_beta(const uint8_t* u, int PL) {
    for (int i = 0; i < PL; ++i) set_leaf(i, u[i]);
  }

  T leaf() const { return alpha[0][0]; }
};

template <class A>
int sc_decode_t(int n, const uint8_t* info, const void* llr, uint8_t* u_hat, double* leaf_llr) {
  Tree<A> t;
  t.init(n, llr);
  const int N = 1 << n;
  // Section 2.2.1: for i = 0..N-1, alpha at leaf i (Algorithm 1), decide by eq. (scest),
  // propagate the bit (Algorithm 2).
  for (int i = 0; i < N; ++i) {
    t.calc_alpha(0, i);
    typename A::T a = t.leaf();
    if (leaf_llr) leaf_llr[i] = A::to_double(a);
    uint8_t u = info[i] ? (uint8_t)A::hd(a) : 0;
    u_hat[i] = u;
    t.set_leaf(i, u);
  }
  return 0;
}

template <class A>
double leaf_llr_t(int n, const void* llr, const uint8_t* prefix, int i) {
  Tree<A> t;
  t.init(n, llr);
  t.populate_beta(prefix, i);
  t.calc_alpha_rm(0, i, true);
  return A::to_double(t.leaf());
}

// ---------------------------------------------------------------------------------
// CRC-16 (R13): polynomial x^16 + x^12 + x^5 + 1 (0x1021), register starts at 0,
// bits enter most significant first, no reflection, no final xor.
// ---------------------------------------------------------------------------------
uint16_t crc16_bits(const uint8_t* bits, int nbits) {
  uint16_t reg = 0;
  for (int k = 0; k < nbits; ++k) {
    int fb = ((reg >> 15) & 1) ^ (bits[k] & 1);
    reg = (uint16_t)(reg << 1);
    if (fb) reg ^= 0x1021;
  }
  return reg;
}

// ---------------------------------------------------------------------------------
// Successive-cancellation stack decoding, Section 2.2.5 with the reduced-memory
// scheme of Section 3.3.
//
// Readings (R7-R15):
//  - S is the set of live paths, at most D of them, and includes the path being
//    extended: each iteration removes the best path from S and inserts its children.
//  - order: key (PM ascending, PL descending, seq ascending); seq numbers paths in
//    creation order, the hard-decision child before the flipped child, and a child that
//    is discarded still uses up its number.
//  - every leaf estimate is an iteration, frozen positions included.
//  - when S is full a child replaces the worst path only if its key is strictly
//    smaller, otherwise the child is dropped.
//  - the L counter is indexed by the length before the extension, i in [0, N-1]; when
//    L extensions have been made at length i, every path with PL <= i is removed.
//  - with a CRC, a length-N path that fails the check is removed and counted; the first
//    such path is the fallback output; after L failures, or if S empties, decoding
//    stops with the fallback.
// ---------------------------------------------------------------------------------
// Optional record of the paths taken off the stack, in the order they are taken (test
// instrumentation for the hand-worked traces: it changes no result).
struct PopTrace {
  uint32_t* seq = nullptr;
  int32_t* pl = nullptr;
  double* pm = nullptr;
  int cap = 0, n = 0;
  void add(uint32_t s, int l, double m) {
    if (n < cap) {
      seq[n] = s;
      pl[n] = l;
      pm[n] = m;
    }
    ++n;
  }
};

template <class A>
struct Path {
  typename A::PM pm;
  int pl;
  uint32_t seq;
  std::vector<uint8_t> u;
};

template <class A>
bool key_less(const Path<A>& a, const Path<A>& b) {
  if (a.pm < b.pm) return true;
  if (b.pm < a.pm) return false;
  if (a.pl != b.pl) return a.pl > b.pl;
  return a.seq < b.seq;
}

bool crc_passes(int N, const uint8_t* info, int crc_bits, const uint8_t* u) {
  if (crc_bits == 0) return true;
  std::vector<uint8_t> inf;
  for (int j = 0; j < N; ++j)
    if (info[j]) inf.push_back(u[j]);
  const int K = (int)inf.size();
  const int k = K - crc_bits;
  uint16_t c = crc16_bits(inf.data(), k);
  for (int b = 0; b < crc_bits; ++b)
    if (((c >> (crc_bits - 1 - b)) & 1) != inf[k + b]) return false;
  return true;
}

// CRC check of a decided bit vector u.  With systematic encoding (Section 2.2.2, last
// paragraph; Section 4) the message sits in the codeword estimate x = u F^(x)n at the
// information positions, so the check reads x there; otherwise it reads u.
bool path_crc_passes(int N, const uint8_t* info, int crc_bits, const uint8_t* u, bool sys) {
  if (!sys) return crc_passes(N, info, crc_bits, u);
  std::vector<uint8_t> x((size_t)N);
  orc_polar_transform(N, u, x.data());
  return crc_passes(N, info, crc_bits, x.data());
}

template <class A>
int scs_decode_t(int n, const uint8_t* info, int crc_bits, int D, int L, const void* llr,
                 uint8_t* u_hat, uint8_t* status, double* pm_out, orc_stats* st, bool sys,
                 PopTrace* tr = nullptr) {
  const int N = 1 << n;
  Tree<A> t;
  t.init(n, llr);
  orc_stats s;
  std::memset(&s, 0, sizeof s);

  std::vector<Path<A>> S;
  S.push_back(Path<A>{typename A::PM(0), 0, 0u, std::vector<uint8_t>(N, 0)});
  uint32_t next_seq = 1;
  std::vector<int> count(N, 0);  // the L counter per pre-extension length
  int fails = 0;
  bool have_fallback = false;
  Path<A> fallback;
  // Identity of the path whose alpha/beta state is held in the single tree
  // (Section 3.3): the hard-decision child of the last extension.
  bool mem_valid = false;
  uint32_t mem_seq = 0;

  uint8_t stat = 0;
  const Path<A>* out = nullptr;
  Path<A> result;

  for (;;) {
    if (S.empty()) {  // only reachable after CRC failures, so a fallback exists
      stat = ORC_ST_FALLBACK | ORC_ST_EXHAUSTED;
      out = have_fallback ? &fallback : nullptr;
      break;
    }
    // The winner: linear search for the smallest key (Section 3.3).
    size_t w = 0;
    for (size_t q = 1; q < S.size(); ++q)
      if (key_less<A>(S[q], S[w])) w = q;
    Path<A> p = S[w];
    S.erase(S.begin() + (long)w);
    if (tr) tr->add(p.seq, p.pl, (double)p.pm);

    if (p.pl == N) {  // termination / CRC, Section 2.2.5
      ++s.completions;
      if (path_crc_passes(N, info, crc_bits, p.u.data(), sys)) {
        result = p;
        out = &result;
        stat = ORC_ST_OK;
        break;
      }
      if (!have_fallback) {
        fallback = p;
        have_fallback = true;
      }
      if (++fails >= L) {
        stat = ORC_ST_FALLBACK;
        out = &fallback;
        break;
      }
      continue;
    }

    const int i = p.pl;
    ++s.iterations;
    s.sc_elems += (i == 0) ? (uint64_t)(N - 1) : ((2ull << __builtin_ctz((unsigned)i)) - 1);

    // alpha at leaf i for path p.
    if (mem_valid && p.seq == mem_seq) {
      t.calc_alpha(0, i);                 // Algorithm 1: the SC schedule continues
    } else {
      ++s.switches;
      t.populate_beta(p.u.data(), i);     // Algorithm 3
      t.calc_alpha_rm(0, i, true);        // Algorithm 4
    }
    const typename A::T a = t.leaf();
    const int h = A::hd(a);
    const typename A::PM m = A::mag(a);

    // Children (eq. PMupd): an information bit splits, a frozen bit (value 0) does not.
    Path<A> c0 = p;
    c0.pl = i + 1;
    c0.seq = next_seq++;
    std::vector<Path<A>> kids;
    if (info[i]) {
      c0.u[i] = (uint8_t)h;
      Path<A> c1 = p;
      c1.pl = i + 1;
      c1.u[i] = (uint8_t)(1 - h);
      c1.pm = A::pm_add(p.pm, m);
      c1.seq = next_seq++;
      kids.push_back(c0);
      kids.push_back(c1);
    } else {
      c0.u[i] = 0;
      if (h) c0.pm = A::pm_add(p.pm, m);
      kids.push_back(c0);
    }
    // The tree now follows the first child: propagate its bit (Algorithm 2).
    t.set_leaf(i, kids[0].u[i]);
    mem_valid = true;
    mem_seq = kids[0].seq;

    // Insert, replacing the worst path of a full stack only by a better one.
    for (auto& c : kids) {
      if ((int)S.size() < D) {
        S.push_back(c);
        continue;
      }
      size_t wq = 0;
      for (size_t q = 1; q < S.size(); ++q)
        if (key_less<A>(S[wq], S[q])) wq = q;
      if (key_less<A>(c, S[wq])) {
        S[wq] = c;
        ++s.evictions;
      } else {
        ++s.drops;
      }
    }

    // L-counter pruning.
    if (++count[i] == L) {
      ++s.prunes;
      std::vector<Path<A>> keep;
      for (auto& q : S)
        if (q.pl > i) keep.push_back(q);
      S.swap(keep);
    }
  }

  s.f_ops = t.f_ops;
  s.g_ops = t.g_ops;
  if (out) {
    std::memcpy(u_hat, out->u.data(), (size_t)N);
    if (pm_out) *pm_out = (double)out->pm;
  } else {
    std::memset(u_hat, 0, (size_t)N);
    if (pm_out) *pm_out = 0.0;
  }
  *status = stat;
  if (st) *st = s;
  return 0;
}

// ---------------------------------------------------------------------------------
// Fast simplified decoding: FSSC nodes (Section 2.2.2), their FSSCL candidate rules
// (Section 2.2.4), the FSSC schedule made once per code (Section 3, FSSC schedule
// figure) and the stack decoder built on them, FSSCS-RM (Section 4).
//
// Readings:
//  - node classes, tested in this order on the leaves of a node of Lambda = 2^lambda
//    leaves: all frozen -> R-0; all information -> R-1; only the last leaf information
//    (Lambda >= 2) -> REP; only the first leaf frozen (Lambda >= 4) -> SPC; otherwise the
//    node is split into its two children.  A leaf is always R-0 or R-1.  `types` limits
//    the classes used above the leaves (bit t = class t allowed).
//  - candidates of a node, numbered in the order written in Section 2.2.4: R-0: one;
//    REP: all-0 then all-1; R-1 (Chase-II on the two least reliable positions m1, m2):
//    HD, flip m1, flip m2, flip both (a one-leaf R-1 node has only HD and flip m1); SPC
//    (equations not given in the paper): the flip patterns of the four least reliable
//    positions m1..m4 that make the node's parity even, taken in increasing order of the
//    pattern read as a 4-bit number (bit k = flip m_(k+1)), which are 8 of the 16.
//  - least reliable positions: ascending |alpha|, ties to the smaller index.
//  - metrics: each flipped position adds its |alpha| to the path metric, in increasing
//    k; R-0 and REP add the node sums of Section 2.2.4, summed pairwise with halving
//    distance (w[j] += w[j + h] for h = Lambda/2, ..., 1), then one addition to PM.
//  - a path stores its N-bit in-place beta array (Section 4): a node's estimates are
//    written at [PL, PL + Lambda) and the beta operation XORs a completed right child
//    into its left sibling in place, upwards while the parent is itself a right child.
//    At PL = N the array holds the codeword estimate; u is its re-encoding (the
//    transform is its own inverse), and the CRC and the payload are read from u.
//  - an iteration is one node extension; the L counter is indexed by the node's first
//    leaf, the path length before the extension; stack rules as for SCS.
//  - the single alpha memory (Section 3.3) is valid for every child of the last
//    extended path, whose beta arrays hold what the next node's g operations read; any
//    other winner is a path switch and alpha is recomputed from the root.
// ---------------------------------------------------------------------------------
enum { NODE_R0 = 0, NODE_R1 = 1, NODE_REP = 2, NODE_SPC = 3 };

struct FNode {
  int start, lam, type;
};

void fssc_nodes(int lam, int phi, const uint8_t* info, int types, std::vector<FNode>& out) {
  const int Lam = 1 << lam, start = phi * Lam;
  int k = 0;
  for (int j = 0; j < Lam; ++j) k += info[start + j] ? 1 : 0;
  int type = -1;
  if (lam == 0) {
    type = k ? NODE_R1 : NODE_R0;
  } else if (k == 0 && (types & (1 << NODE_R0))) {
    type = NODE_R0;
  } else if (k == Lam && (types & (1 << NODE_R1))) {
    type = NODE_R1;
  } else if (k == 1 && info[start + Lam - 1] && (types & (1 << NODE_REP))) {
    type = NODE_REP;
  } else if (Lam >= 4 && k == Lam - 1 && !info[start] && (types & (1 << NODE_SPC))) {
    type = NODE_SPC;
  }
  if (type >= 0) {
    out.push_back(FNode{start, lam, type});
    return;
  }
  fssc_nodes(lam - 1, 2 * phi, info, types, out);
  fssc_nodes(lam - 1, 2 * phi + 1, info, types, out);
}

// Sum with halving distance: w[j] += w[j + h], h = Lambda/2, ..., 1.
template <class A>
typename A::PM node_sum(std::vector<typename A::PM> w) {
  for (size_t h = w.size() / 2; h >= 1; h /= 2)
    for (size_t j = 0; j < h; ++j) w[j] = w[j] + w[j + h];
  return w[0];
}

// Least reliable positions of alpha_v: the first `cnt` indices in ascending |alpha|,
// ties to the smaller index.
template <class A>
std::vector<int> least_reliable(const std::vector<typename A::T>& a, int cnt) {
  std::vector<int> idx(a.size());
  for (size_t j = 0; j < a.size(); ++j) idx[j] = (int)j;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int x, int y) { return A::mag(a[x]) < A::mag(a[y]); });
  idx.resize((size_t)cnt);
  return idx;
}

template <class A>
struct Cand {
  std::vector<uint8_t> beta;
  typename A::PM pm;
};

// FSSCL candidate rules (Section 2.2.4) for one node.
template <class A>
std::vector<Cand<A>> node_candidates(int type, const std::vector<typename A::T>& a,
                                     typename A::PM pm) {
  typedef typename A::PM PM;
  const int Lam = (int)a.size();
  std::vector<uint8_t> hd(Lam);
  for (int j = 0; j < Lam; ++j) hd[j] = (uint8_t)A::hd(a[j]);
  std::vector<Cand<A>> out;
  if (type == NODE_R0 || type == NODE_REP) {
    std::vector<PM> w0(Lam), w1(Lam);
    for (int j = 0; j < Lam; ++j) {
      w0[j] = hd[j] ? A::mag(a[j]) : PM(0);   // HD(alpha) |alpha|
      w1[j] = hd[j] ? PM(0) : A::mag(a[j]);   // (1 - HD(alpha)) |alpha|
    }
    out.push_back(Cand<A>{std::vector<uint8_t>(Lam, 0), A::pm_add(pm, node_sum<A>(w0))});
    if (type == NODE_REP)
      out.push_back(Cand<A>{std::vector<uint8_t>(Lam, 1), A::pm_add(pm, node_sum<A>(w1))});
    return out;
  }
  const int nlr = type == NODE_R1 ? (Lam >= 2 ? 2 : 1) : 4;
  const std::vector<int> m = least_reliable<A>(a, nlr);
  int parity = 0;
  for (int j = 0; j < Lam; ++j) parity ^= hd[j];
  for (int mask = 0; mask < (1 << nlr); ++mask) {
    if (type == NODE_SPC && (__builtin_popcount((unsigned)mask) & 1) != parity) continue;
    Cand<A> c{hd, pm};
    for (int k = 0; k < nlr; ++k)
      if (mask & (1 << k)) {
        c.beta[m[k]] ^= 1;
        c.pm = A::pm_add(c.pm, A::mag(a[m[k]]));
      }
    out.push_back(c);
  }
  return out;
}

// Alpha memory of Section 3.1 for the fast schedule: the g operations read the left
// sibling's estimates from the path's in-place beta array.
template <class A>
struct FTree {
  typedef typename A::T T;
  int n = 0;
  std::vector<std::vector<T>> alpha;
  uint64_t f_ops = 0, g_ops = 0;

  void init(int n_, const void* llr) {
    n = n_;
    alpha.assign(n + 1, std::vector<T>());
    for (int lam = 0; lam <= n; ++lam) alpha[lam].assign(1u << lam, T(0));
    for (int j = 0; j < (1 << n); ++j) alpha[n][j] = load_llr<A>(llr, j);
  }

  // eq. (llrcalc) for node (lambda, phi); beta: the path's N-bit array.
  void node_alpha(int lam, int phi, const uint8_t* beta) {
    const int Lam = 1 << lam;
    const T* ap = alpha[lam + 1].data();
    T* av = alpha[lam].data();
    if ((phi & 1) == 0) {
      for (int i = 0; i < Lam; ++i) av[i] = A::f(ap[i], ap[i + Lam]);
      f_ops += Lam;
    } else {
      const uint8_t* bu = beta + (size_t)(phi - 1) * Lam;  // left sibling, in place
      for (int i = 0; i < Lam; ++i) av[i] = A::g(ap[i], ap[i + Lam], bu[i]);
      g_ops += Lam;
    }
  }

  // Algorithm 1 from node (lambda, phi); with `switched`, Algorithm 4 (from the root).
  void calc_alpha(int lam, int phi, bool switched, const uint8_t* beta) {
    if (lam == n) return;
    if ((phi & 1) == 0 || switched) calc_alpha(lam + 1, phi >> 1, switched, beta);
    node_alpha(lam, phi, beta);
  }
};

// The beta operation in place (Section 4): a completed right child is XORed into its left
// sibling, which turns the pair into the parent's estimates; repeat upwards.
void beta_in_place(uint8_t* beta, int n, int lam, int phi) {
  while (lam < n && (phi & 1)) {
    const int Lam = 1 << lam;
    uint8_t* left = beta + (size_t)(phi - 1) * Lam;
    const uint8_t* right = beta + (size_t)phi * Lam;
    for (int i = 0; i < Lam; ++i) left[i] ^= right[i];
    ++lam;
    phi >>= 1;
  }
}

template <class A>
struct FPath {
  typename A::PM pm;
  int pl;
  uint32_t seq;
  std::vector<uint8_t> beta;  // N bits, in place
};

template <class A>
bool fkey_less(const FPath<A>& a, const FPath<A>& b) {
  if (a.pm < b.pm) return true;
  if (b.pm < a.pm) return false;
  if (a.pl != b.pl) return a.pl > b.pl;
  return a.seq < b.seq;
}

template <class A>
int fsscs_decode_t(int n, const uint8_t* info, int crc_bits, int D, int L, int types,
                   const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                   orc_stats* st, bool sys, PopTrace* tr = nullptr) {
  const int N = 1 << n;
  std::vector<FNode> sched;
  fssc_nodes(n, 0, info, types, sched);
  std::vector<int> node_at(N, -1);  // the schedule position of a path of length PL
  for (size_t q = 0; q < sched.size(); ++q) node_at[sched[q].start] = (int)q;

  FTree<A> t;
  t.init(n, llr);
  orc_stats s;
  std::memset(&s, 0, sizeof s);
  std::vector<FPath<A>> S;
  S.push_back(FPath<A>{typename A::PM(0), 0, 0u, std::vector<uint8_t>(N, 0)});
  uint32_t next_seq = 1;
  std::vector<int> count(N, 0);
  int fails = 0;
  bool have_fallback = false;
  FPath<A> fallback, result;
  const FPath<A>* out = nullptr;
  uint8_t stat = 0;
  // children of the last extension (the paths the alpha memory is valid for)
  bool mem_valid = false;
  uint32_t mem_lo = 0, mem_hi = 0;
  int mem_pl = -1;

  for (;;) {
    if (S.empty()) {
      stat = ORC_ST_FALLBACK | ORC_ST_EXHAUSTED;
      out = have_fallback ? &fallback : nullptr;
      break;
    }
    size_t w = 0;
    for (size_t q = 1; q < S.size(); ++q)
      if (fkey_less<A>(S[q], S[w])) w = q;
    FPath<A> p = S[w];
    S.erase(S.begin() + (long)w);
    if (tr) tr->add(p.seq, p.pl, (double)p.pm);

    if (p.pl == N) {
      ++s.completions;
      std::vector<uint8_t> u(N);
      // systematic: the message is read from the codeword estimate (beta) itself;
      // otherwise from its re-encoding u
      orc_polar_transform(N, p.beta.data(), u.data());
      if (crc_passes(N, info, crc_bits, sys ? p.beta.data() : u.data())) {
        result = p;
        out = &result;
        stat = ORC_ST_OK;
        break;
      }
      if (!have_fallback) {
        fallback = p;
        have_fallback = true;
      }
      if (++fails >= L) {
        stat = ORC_ST_FALLBACK;
        out = &fallback;
        break;
      }
      continue;
    }

    const int i = p.pl;
    const FNode& v = sched[(size_t)node_at[i]];
    const int Lam = 1 << v.lam, phi = i >> v.lam;
    ++s.iterations;
    s.sc_elems += (i == 0) ? (uint64_t)(N - Lam)
                           : ((2ull << __builtin_ctz((unsigned)i)) - (uint64_t)Lam);

    const bool cont = mem_valid && p.pl == mem_pl && p.seq >= mem_lo && p.seq <= mem_hi;
    if (!cont) ++s.switches;
    t.calc_alpha(v.lam, phi, !cont, p.beta.data());
    const std::vector<typename A::T> a(t.alpha[v.lam].begin(), t.alpha[v.lam].end());

    std::vector<FPath<A>> kids;
    for (const Cand<A>& c : node_candidates<A>(v.type, a, p.pm)) {
      FPath<A> k = p;
      k.pl = i + Lam;
      k.pm = c.pm;
      k.seq = next_seq++;
      std::copy(c.beta.begin(), c.beta.end(), k.beta.begin() + i);
      beta_in_place(k.beta.data(), n, v.lam, phi);
      kids.push_back(k);
    }
    mem_valid = true;
    mem_lo = kids.front().seq;
    mem_hi = kids.back().seq;
    mem_pl = i + Lam;

    for (auto& c : kids) {
      if ((int)S.size() < D) {
        S.push_back(c);
        continue;
      }
      size_t wq = 0;
      for (size_t q = 1; q < S.size(); ++q)
        if (fkey_less<A>(S[wq], S[q])) wq = q;
      if (fkey_less<A>(c, S[wq])) {
        S[wq] = c;
        ++s.evictions;
      } else {
        ++s.drops;
      }
    }
    if (++count[i] == L) {
      ++s.prunes;
      std::vector<FPath<A>> keep;
      for (auto& q : S)
        if (q.pl > i) keep.push_back(q);
      S.swap(keep);
    }
  }

  s.f_ops = t.f_ops;
  s.g_ops = t.g_ops;
  if (out) {
    orc_polar_transform(N, out->beta.data(), u_hat);
    if (pm_out) *pm_out = (double)out->pm;
  } else {
    std::memset(u_hat, 0, (size_t)N);
    if (pm_out) *pm_out = 0.0;
  }
  *status = stat;
  if (st) *st = s;
  return 0;
}

// ---------------------------------------------------------------------------------
// Successive-cancellation list decoding with CRC selection (CA-SCL), Section 2.2.3, with
// one alpha/beta tree per list entry (Section 3.2 keeps L trees; lazy copying is an
// optimisation of the same computation and is not reproduced here: a surviving child
// simply copies its parent's tree).
//
// Readings:
//  - the list starts with one path of metric 0; at a frozen leaf every path takes u = 0
//    and its metric grows by |alpha| when HD(alpha) = 1 (eq. PMupd); at an information
//    leaf every path l (in list order) offers two candidates, u = 0 then u = 1, each with
//    the metric of eq. (PMupd); the min(2 n, L) candidates with the smallest key (metric,
//    then candidate number 2 l + u) survive and form the new list in ascending key order.
//  - selection (the CRC aid of Section 2.2.3): the paths are taken in ascending (metric,
//    list position); the first whose information bits pass the CRC is the output (status
//    OK); if none passes (or there is no CRC) the first path is the output, with status
//    FALLBACK when a CRC was checked and failed for every path.
//  - statistics: iterations = leaf estimates (paths x leaves), completions = CRC checks.
// ---------------------------------------------------------------------------------
template <class A>
struct ListPath {
  typename A::PM pm;
  Tree<A> tree;
  std::vector<uint8_t> u;
};

template <class A>
int scl_decode_t(int n, const uint8_t* info, int crc_bits, int L, const void* llr,
                 uint8_t* u_hat, uint8_t* status, double* pm_out, orc_stats* st,
                 bool sys) {
  typedef typename A::PM PM;
  const int N = 1 << n;
  orc_stats s;
  std::memset(&s, 0, sizeof s);
  std::vector<ListPath<A>> list(1);
  list[0].pm = PM(0);
  list[0].tree.init(n, llr);
  list[0].u.assign(N, 0);
  for (int i = 0; i < N; ++i) {
    std::vector<typename A::T> a(list.size());
    for (size_t l = 0; l < list.size(); ++l) {
      list[l].tree.calc_alpha(0, i);  // Algorithm 1 on the path's own tree
      a[l] = list[l].tree.leaf();
      ++s.iterations;
    }
    if (!info[i]) {
      for (size_t l = 0; l < list.size(); ++l) {
        if (A::hd(a[l])) list[l].pm = A::pm_add(list[l].pm, A::mag(a[l]));
        list[l].u[i] = 0;
        list[l].tree.set_leaf(i, 0);
      }
      continue;
    }
    // candidates 2 l + u, metric of eq. (PMupd)
    struct C {
      PM pm;
      int idx;
    };
    std::vector<C> cand;
    for (size_t l = 0; l < list.size(); ++l)
      for (int u = 0; u < 2; ++u) {
        PM m = list[l].pm;
        if (u != A::hd(a[l])) m = A::pm_add(m, A::mag(a[l]));
        cand.push_back(C{m, (int)(2 * l + u)});
      }
    std::stable_sort(cand.begin(), cand.end(), [](const C& x, const C& y) {
      return x.pm < y.pm || (!(y.pm < x.pm) && x.idx < y.idx);
    });
    const size_t keep = std::min(cand.size(), (size_t)L);
    std::vector<ListPath<A>> next;
    for (size_t k = 0; k < keep; ++k) {
      const int l = cand[k].idx >> 1, u = cand[k].idx & 1;
      ListPath<A> c = list[(size_t)l];  // the parent's tree, copied
      c.pm = cand[k].pm;
      c.u[i] = (uint8_t)u;
      c.tree.set_leaf(i, (uint8_t)u);
      next.push_back(std::move(c));
    }
    list.swap(next);
  }
  std::vector<size_t> order(list.size());
  for (size_t l = 0; l < order.size(); ++l) order[l] = l;
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return list[x].pm < list[y].pm; });
  size_t out = order[0];
  uint8_t stat = ORC_ST_OK;
  if (crc_bits) {
    stat = ORC_ST_FALLBACK;
    for (size_t q : order) {
      ++s.completions;
      if (path_crc_passes(N, info, crc_bits, list[q].u.data(), sys)) {
        out = q;
        stat = ORC_ST_OK;
        break;
      }
    }
  }
  for (auto& p : list) {
    s.f_ops += p.tree.f_ops;
    s.g_ops += p.tree.g_ops;
  }
  std::memcpy(u_hat, list[out].u.data(), (size_t)N);
  if (pm_out) *pm_out = (double)list[out].pm;
  *status = stat;
  if (st) *st = s;
  return 0;
}

// Bhattacharyya parameters in the log domain (R17): z0 = exp(-R * Eb/N0) for BPSK on
// AWGN; the "minus" (f) child of z is 2z - z^2 and the "plus" (g) child is z^2.
// Indices: the children of index j are 2j (minus) and 2j+1 (plus), so the first split
// is the most significant bit of the leaf index, as in the tree of eq. (llrcalc).
void bhatta_log(int n, double rate, double design_db, double* lz) {
  const int N = 1 << n;
  std::vector<double> cur(1, -rate * std::pow(10.0, design_db / 10.0));
  for (int level = 0; level < n; ++level) {
    std::vector<double> nxt(cur.size() * 2);
    for (size_t j = 0; j < cur.size(); ++j) {
      const double l = cur[j];
      // ln(2z - z^2) = ln z + ln(2 - z), and 2 - z = 1 - (z - 1) = 1 - expm1(ln z).
      nxt[2 * j] = l + std::log1p(-std::expm1(l));
      nxt[2 * j + 1] = 2.0 * l;                    // ln(z^2)
    }
    cur.swap(nxt);
  }
  for (int j = 0; j < N; ++j) lz[j] = cur[j];
}

}  // namespace

extern "C" {

int orc_bhattacharyya_log(int N, double rate, double design_ebn0_db, double* lz) {
  const int n = log2_exact(N);
  if (n < 0 || !lz) return -1;
  bhatta_log(n, rate, design_ebn0_db, lz);
  return 0;
}

int orc_construct(int N, int K, double design_ebn0_db, uint8_t* info_mask) {
  const int n = log2_exact(N);
  if (n < 0 || K < 0 || K > N || !info_mask) return -1;
  std::vector<double> lz(N);
  bhatta_log(n, (double)K / N, design_ebn0_db, lz.data());
  std::vector<int> idx(N);
  for (int j = 0; j < N; ++j) idx[j] = j;
  // Most reliable first: smaller parameter, then larger index.
  std::sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (lz[a] != lz[b]) return lz[a] < lz[b];
    return a > b;
  });
  std::memset(info_mask, 0, (size_t)N);
  for (int k = 0; k < K; ++k) info_mask[idx[k]] = 1;
  return 0;
}

uint16_t orc_crc16_bits(const uint8_t* bits, int nbits) { return crc16_bits(bits, nbits); }

int orc_polar_transform(int N, const uint8_t* u, uint8_t* c) {
  // Section 2.1: c = u F^{(x)n}, drawn as the n-stage XOR tree of the encoder figure:
  // at stage s (distance 2^s) every upper wire j takes the XOR of wire j + 2^s.
  if (log2_exact(N) < 0) return -1;
  std::vector<uint8_t> x(u, u + N);
  for (int s = 1; s < N; s <<= 1)
    for (int j = 0; j < N; ++j)
      if ((j & s) == 0) x[j] ^= x[j + s];
  std::memcpy(c, x.data(), (size_t)N);
  return 0;
}

int orc_encode_batch(int N, const uint8_t* info_mask, int crc_bits, const uint8_t* payload,
                     int64_t B, uint8_t* codeword) {
  if (log2_exact(N) < 0 || (crc_bits != 0 && crc_bits != 16)) return -1;
  std::vector<int> pos;
  for (int j = 0; j < N; ++j)
    if (info_mask[j]) pos.push_back(j);
  const int K = (int)pos.size();
  const int k = K - crc_bits;
  if (k < 0) return -1;
  std::vector<uint8_t> u(N), msg(K);
  for (int64_t b = 0; b < B; ++b) {
    const uint8_t* pl = payload + b * k;
    for (int j = 0; j < k; ++j) msg[j] = pl[j] & 1;
    if (crc_bits) {
      uint16_t c = crc16_bits(msg.data(), k);
      for (int j = 0; j < crc_bits; ++j) msg[k + j] = (uint8_t)((c >> (crc_bits - 1 - j)) & 1);
    }
    // Section 2.1: message bits at the indices of A, zeros elsewhere.
    std::fill(u.begin(), u.end(), 0);
    for (int j = 0; j < K; ++j) u[pos[j]] = msg[j];
    orc_polar_transform(N, u.data(), codeword + b * N);
  }
  return 0;
}

int orc_encode_systematic_batch(int N, const uint8_t* info_mask, int crc_bits,
                                const uint8_t* payload, int64_t B, uint8_t* codeword) {
  // Systematic encoding (Section 2.2.2, last paragraph; Section 4): the codeword carries the
  // message itself at the information positions.  Two passes of the transform: put the
  // message at the information positions of v, take u = v F^(x)n, clear u at the frozen
  // positions, and send x = u F^(x)n.  x is a codeword of the code (u is zero where frozen)
  // and shows the message at the information positions when the set is closed under the
  // binary-domination order, as the constructed sets are.
  if (log2_exact(N) < 0 || (crc_bits != 0 && crc_bits != 16)) return -1;
  std::vector<int> pos;
  for (int j = 0; j < N; ++j)
    if (info_mask[j]) pos.push_back(j);
  const int K = (int)pos.size();
  const int k = K - crc_bits;
  if (k < 0) return -1;
  std::vector<uint8_t> msg((size_t)K), v((size_t)N), u((size_t)N);
  for (int64_t b = 0; b < B; ++b) {
    // the message: payload, then its CRC remainder (most significant bit first)
    for (int j = 0; j < k; ++j) msg[j] = payload[b * k + j] & 1;
    if (crc_bits) {
      const uint16_t c = crc16_bits(msg.data(), k);
      for (int j = 0; j < crc_bits; ++j) msg[k + j] = (uint8_t)((c >> (crc_bits - 1 - j)) & 1);
    }
    std::fill(v.begin(), v.end(), 0);
    for (int j = 0; j < K; ++j) v[pos[j]] = msg[j];
    orc_polar_transform(N, v.data(), u.data());
    for (int j = 0; j < N; ++j)
      if (!info_mask[j]) u[j] = 0;
    orc_polar_transform(N, u.data(), codeword + b * N);
  }
  return 0;
}

int orc_sc_decode(int mode, int N, const uint8_t* info_mask, const void* llr, uint8_t* u_hat,
                  double* leaf_llr) {
  const int n = log2_exact(N);
  if (n < 0) return -1;
  switch (mode) {
    case ORC_F32: return sc_decode_t<ArF32>(n, info_mask, llr, u_hat, leaf_llr);
    case ORC_F64: return sc_decode_t<ArF64>(n, info_mask, llr, u_hat, leaf_llr);
    case ORC_FIX: return sc_decode_t<ArFix>(n, info_mask, llr, u_hat, leaf_llr);
  }
  return -1;
}

double orc_leaf_llr(int mode, int N, const void* llr, const uint8_t* prefix, int i) {
  const int n = log2_exact(N);
  if (n < 0 || i < 0 || i >= N) return NAN;
  switch (mode) {
    case ORC_F32: return leaf_llr_t<ArF32>(n, llr, prefix, i);
    case ORC_F64: return leaf_llr_t<ArF64>(n, llr, prefix, i);
    case ORC_FIX: return leaf_llr_t<ArFix>(n, llr, prefix, i);
  }
  return NAN;
}

int orc_scs_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                   const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                   orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0 || D < 1 || L < 1 || (crc_bits != 0 && crc_bits != 16)) return -1;
  const bool sys = systematic != 0;
  switch (mode) {
    case ORC_F32: return scs_decode_t<ArF32>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, sys);
    case ORC_F64: return scs_decode_t<ArF64>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, sys);
    case ORC_FIX: return scs_decode_t<ArFix>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, sys);
  }
  return -1;
}

int orc_scs_trace(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                  const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                  orc_stats* st, uint32_t* seq, int32_t* pl, double* pm, int cap,
                  int systematic) {
  const int n = log2_exact(N);
  if (n < 0 || D < 1 || L < 1 || (crc_bits != 0 && crc_bits != 16) || cap < 0) return -1;
  PopTrace tr;
  tr.seq = seq;
  tr.pl = pl;
  tr.pm = pm;
  tr.cap = cap;
  int rc = -1;
  switch (mode) {
    case ORC_F32: rc = scs_decode_t<ArF32>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
    case ORC_F64: rc = scs_decode_t<ArF64>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
    case ORC_FIX: rc = scs_decode_t<ArFix>(n, info_mask, crc_bits, D, L, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
  }
  return rc < 0 ? rc : tr.n;
}

int orc_fsscs_trace(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                    int types, const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                    orc_stats* st, uint32_t* seq, int32_t* pl, double* pm, int cap,
                    int systematic) {
  const int n = log2_exact(N);
  if (n < 0 || D < 1 || L < 1 || (crc_bits != 0 && crc_bits != 16) || cap < 0) return -1;
  PopTrace tr;
  tr.seq = seq;
  tr.pl = pl;
  tr.pm = pm;
  tr.cap = cap;
  int rc = -1;
  switch (mode) {
    case ORC_F32: rc = fsscs_decode_t<ArF32>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
    case ORC_F64: rc = fsscs_decode_t<ArF64>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
    case ORC_FIX: rc = fsscs_decode_t<ArFix>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, systematic != 0, &tr); break;
  }
  return rc < 0 ? rc : tr.n;
}

int orc_scs_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                         const void* llr, int64_t B, uint8_t* payload, uint8_t* status,
                         orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0) return -1;
  const size_t esz = mode == ORC_F32 ? 4 : (mode == ORC_F64 ? 8 : 1);
  int K = 0;
  for (int j = 0; j < N; ++j) K += info_mask[j] ? 1 : 0;
  const int k = K - crc_bits;
  std::vector<uint8_t> u(N);
  for (int64_t b = 0; b < B; ++b) {
    int rc = orc_scs_decode(mode, N, info_mask, crc_bits, D, L,
                            (const uint8_t*)llr + (size_t)b * N * esz, u.data(), status + b,
                            nullptr, st ? st + b : nullptr, systematic);
    if (rc) return rc;
    // the payload: the first K - crc information bits of u, or with systematic encoding of
    // the codeword estimate u F^(x)n
    if (systematic) {
      std::vector<uint8_t> x(u);
      orc_polar_transform(N, x.data(), u.data());
    }
    int q = 0;
    for (int j = 0; j < N && q < k; ++j)
      if (info_mask[j]) payload[b * k + q++] = u[j];
  }
  return 0;
}

int orc_ml_decode(int N, const uint8_t* info_mask, const double* llr, double* disc_min,
                  int64_t* n_min, uint8_t* minimisers, int64_t max_out) {
  if (log2_exact(N) < 0) return -1;
  std::vector<int> pos;
  for (int j = 0; j < N; ++j)
    if (info_mask[j]) pos.push_back(j);
  const int K = (int)pos.size();
  if (K > 20) return -1;
  std::vector<uint8_t> u(N), c(N);
  double best = INFINITY;
  int64_t cnt = 0;
  for (uint64_t m = 0; m < (1ull << K); ++m) {
    std::fill(u.begin(), u.end(), 0);
    for (int j = 0; j < K; ++j) u[pos[j]] = (uint8_t)((m >> j) & 1);
    orc_polar_transform(N, u.data(), c.data());
    double d = 0.0;
    for (int j = 0; j < N; ++j)
      if (c[j] != (llr[j] < 0 ? 1 : 0)) d += std::fabs(llr[j]);
    if (d < best) {
      best = d;
      cnt = 0;
    }
    if (d == best) {
      if (cnt < max_out && minimisers) std::memcpy(minimisers + cnt * N, u.data(), (size_t)N);
      ++cnt;
    }
  }
  *disc_min = best;
  *n_min = cnt;
  return 0;
}

int orc_fssc_schedule(int N, const uint8_t* info_mask, int types, int32_t* start, int32_t* lam,
                      int32_t* type, int max_nodes) {
  const int n = log2_exact(N);
  if (n < 0) return -1;
  std::vector<FNode> sched;
  fssc_nodes(n, 0, info_mask, types, sched);
  for (size_t q = 0; q < sched.size() && (int)q < max_nodes; ++q) {
    start[q] = sched[q].start;
    lam[q] = sched[q].lam;
    type[q] = sched[q].type;
  }
  return (int)sched.size();
}

int orc_node_candidates(int mode, int type, int lam, const double* alpha, double pm,
                        uint8_t* beta_out, double* pm_out, int max_out) {
  const int Lam = 1 << lam;
  if (type < 0 || type > 3 || lam < 0 || lam > 11) return -1;
  if ((type == NODE_SPC && Lam < 4) || (type == NODE_REP && Lam < 2)) return -1;
  int cnt = 0;
  auto emit = [&](const std::vector<uint8_t>& b, double m) {
    if (cnt < max_out) {
      std::memcpy(beta_out + (size_t)cnt * Lam, b.data(), (size_t)Lam);
      pm_out[cnt] = m;
    }
    ++cnt;
  };
  if (mode == ORC_F64) {
    std::vector<double> a(alpha, alpha + Lam);
    for (auto& c : node_candidates<ArF64>(type, a, pm)) emit(c.beta, c.pm);
  } else if (mode == ORC_F32) {
    std::vector<float> a(Lam);
    for (int j = 0; j < Lam; ++j) a[j] = (float)alpha[j];
    for (auto& c : node_candidates<ArF32>(type, a, (float)pm)) emit(c.beta, (double)c.pm);
  } else {
    std::vector<int> a(Lam);
    for (int j = 0; j < Lam; ++j) a[j] = (int)alpha[j];
    for (auto& c : node_candidates<ArFix>(type, a, (int)pm)) emit(c.beta, (double)c.pm);
  }
  return cnt;
}

int orc_fsscs_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int D, int L,
                     int types, const void* llr, uint8_t* u_hat, uint8_t* status,
                     double* pm_out, orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0 || D < 1 || L < 1 || (crc_bits != 0 && crc_bits != 16)) return -1;
  const bool sys = systematic != 0;
  switch (mode) {
    case ORC_F32: return fsscs_decode_t<ArF32>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, sys);
    case ORC_F64: return fsscs_decode_t<ArF64>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, sys);
    case ORC_FIX: return fsscs_decode_t<ArFix>(n, info_mask, crc_bits, D, L, types, llr, u_hat, status, pm_out, st, sys);
  }
  return -1;
}

int orc_fsscs_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int D,
                           int L, int types, const void* llr, int64_t B, uint8_t* payload,
                           uint8_t* status, orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0) return -1;
  const size_t esz = mode == ORC_F32 ? 4 : (mode == ORC_F64 ? 8 : 1);
  int K = 0;
  for (int j = 0; j < N; ++j) K += info_mask[j] ? 1 : 0;
  const int k = K - crc_bits;
  std::vector<uint8_t> u(N);
  for (int64_t b = 0; b < B; ++b) {
    int rc = orc_fsscs_decode(mode, N, info_mask, crc_bits, D, L, types,
                              (const uint8_t*)llr + (size_t)b * N * esz, u.data(), status + b,
                              nullptr, st ? st + b : nullptr, systematic);
    if (rc) return rc;
    // the payload: the first K - crc information bits of u, or with systematic encoding of
    // the codeword estimate u F^(x)n
    if (systematic) {
      std::vector<uint8_t> x(u);
      orc_polar_transform(N, x.data(), u.data());
    }
    int q = 0;
    for (int j = 0; j < N && q < k; ++j)
      if (info_mask[j]) payload[b * k + q++] = u[j];
  }
  return 0;
}

int orc_scl_decode(int mode, int N, const uint8_t* info_mask, int crc_bits, int L,
                   const void* llr, uint8_t* u_hat, uint8_t* status, double* pm_out,
                   orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0 || L < 1 || (crc_bits != 0 && crc_bits != 16)) return -1;
  const bool sys = systematic != 0;
  switch (mode) {
    case ORC_F32: return scl_decode_t<ArF32>(n, info_mask, crc_bits, L, llr, u_hat, status, pm_out, st, sys);
    case ORC_F64: return scl_decode_t<ArF64>(n, info_mask, crc_bits, L, llr, u_hat, status, pm_out, st, sys);
    case ORC_FIX: return scl_decode_t<ArFix>(n, info_mask, crc_bits, L, llr, u_hat, status, pm_out, st, sys);
  }
  return -1;
}

int orc_scl_decode_batch(int mode, int N, const uint8_t* info_mask, int crc_bits, int L,
                         const void* llr, int64_t B, uint8_t* payload, uint8_t* status,
                         orc_stats* st, int systematic) {
  const int n = log2_exact(N);
  if (n < 0) return -1;
  const size_t esz = mode == ORC_F32 ? 4 : (mode == ORC_F64 ? 8 : 1);
  int K = 0;
  for (int j = 0; j < N; ++j) K += info_mask[j] ? 1 : 0;
  const int k = K - crc_bits;
  std::vector<uint8_t> u(N);
  for (int64_t b = 0; b < B; ++b) {
    int rc = orc_scl_decode(mode, N, info_mask, crc_bits, L,
                            (const uint8_t*)llr + (size_t)b * N * esz, u.data(), status + b,
                            nullptr, st ? st + b : nullptr, systematic);
    if (rc) return rc;
    // the payload: the first K - crc information bits of u, or with systematic encoding of
    // the codeword estimate u F^(x)n
    if (systematic) {
      std::vector<uint8_t> x(u);
      orc_polar_transform(N, x.data(), u.data());
    }
    int q = 0;
    for (int j = 0; j < N && q < k; ++j)
      if (info_mask[j]) payload[b * k + q++] = u[j];
  }
  return 0;
}

}  // extern "C"
