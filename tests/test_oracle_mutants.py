"""The hand-worked pins are sharp: each plausible slip in the oracle's stack rules, node
sums, fixed-point metric or systematic encoding, planted in a copy of the oracle source and
built on the CPU, makes the golden tests (test_oracle_golden_search.py,
test_oracle_systematic.py) fail.  The copies are loaded in
child processes (POLAR_ORACLE_LIB), never in this one."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "polar_oracle.cpp")
GOLDEN_TESTS = [os.path.join(ROOT, "tests", f) for f in
                ("test_oracle_golden_search.py", "test_oracle_systematic.py")]

# name -> (text in the oracle source, replacement); the first occurrence is replaced
MUTANTS = {
    # reading R11: order of equal metrics
    "shorter_path_first": ("if (a.pl != b.pl) return a.pl > b.pl;",
                           "if (a.pl != b.pl) return a.pl < b.pl;"),
    "newest_path_first": ("return a.seq < b.seq;", "return a.seq > b.seq;"),
    "flipped_child_numbered_first": ("c1.seq = next_seq++;",
                                     "c1.seq = c0.seq; c0.seq = next_seq++;"),
    "metric_only_slot_order": ("if (key_less<A>(S[q], S[w])) w = q;",
                               "if (S[q].pm < S[w].pm) w = q;"),
    # reading R12: full stack
    "worst_by_metric_only": ("if (key_less<A>(S[wq], S[q])) wq = q;",
                             "if (S[wq].pm < S[q].pm) wq = q;"),
    "full_stack_never_replaces": ("if (key_less<A>(c, S[wq])) {", "if (false) {"),
    # reading R15: output after L CRC failures
    "fallback_last_failed_path": ("if (!have_fallback) {", "if (true) {"),
    # reading R10: L-counter prune keeps paths of the counted length
    "prune_shorter_only": ("if (q.pl > i) keep.push_back(q);",
                           "if (q.pl >= i) keep.push_back(q);"),
    # reading F5: node sums left to right
    "node_sum_left_to_right": (
        "for (size_t j = 0; j < h; ++j) w[j] = w[j] + w[j + h];",
        "if (h == 1) { for (size_t j = 1; j < w.size(); ++j) w[0] = w[0] + w[j]; "
        "for (size_t j = 1; j < w.size(); ++j) w[j] = 0; }"),
    # reading F5: flips summed before they join the metric
    "flips_summed_first": (
        "c.pm = A::pm_add(c.pm, A::mag(a[m[k]]));",
        "c.pm = (k == 0) ? A::mag(a[m[k]]) : A::pm_add(c.pm, A::mag(a[m[k]])); "
        "if (k == nlr - 1 || !(mask >> (k + 1))) c.pm = A::pm_add(pm, c.pm);"),
    # reading F3: bit k of the mask flips m_(4-k) instead of m_(k+1)
    "spc_mask_bits_reversed": ("if (mask & (1 << k)) {", "if (mask & (1 << (nlr - 1 - k))) {"),
    # reading F4: ties of |alpha| to the larger index
    "lrp_ties_to_larger_index": ("idx[j] = (int)j;", "idx[j] = (int)(a.size() - 1 - j);"),
    # reading R18: int16 metric saturation
    "metric_without_saturation": ("return s > 32767 ? 32767 : s;", "return s;"),
    "metric_wraps_int16": ("return s > 32767 ? 32767 : s;", "return (int)(int16_t)s;"),
    # systematic encoding: CRC read from u, frozen positions kept, payload read from u
    "systematic_crc_reads_u": ("if (!sys) return crc_passes(N, info, crc_bits, u);",
                               "return crc_passes(N, info, crc_bits, u);"),
    "systematic_encoder_keeps_frozen": (
        "      if (!info_mask[j]) u[j] = 0;\n    orc_polar_transform(N, u.data(), codeword + b * N);",
        "      if (false) u[j] = 0;\n    orc_polar_transform(N, u.data(), codeword + b * N);"),
    "systematic_payload_from_u": ("    if (systematic) {", "    if (false) {"),
}


def _build(name, tmp):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert old in text, name
    src = os.path.join(tmp, name + ".cpp")
    with open(src, "w") as f:
        f.write(text.replace(old, new, 1))
    lib = os.path.join(tmp, name + ".so")
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-fno-fast-math", "-ffp-contract=off",
                           "-fPIC", "-shared", "-I" + os.path.join(ROOT, "oracle"), "-o", lib,
                           src])
    return lib


def _run_golden(lib):
    env = dict(os.environ, POLAR_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"]
                       + GOLDEN_TESTS, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_results():
    with tempfile.TemporaryDirectory() as tmp:
        names = sorted(MUTANTS)
        with ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
            libs = list(ex.map(lambda n: _build(n, tmp), names))
            runs = list(ex.map(_run_golden, libs))
        yield dict(zip(names, runs))


def test_unmodified_oracle_passes_the_golden_tests():
    rc, out = _run_golden(os.path.join(ROOT, "oracle", "liboracle.so"))
    assert rc == 0, out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_golden_tests_catch_the_mutant(mutant_results, name):
    rc, out = mutant_results[name]
    assert rc == 1, "mutant %s passed the golden tests:\n%s" % (name, out)
