"""The oracle against what the paper and the mathematics fix (CPU only)."""

import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from . import pins
from .invariants import check_graph


def test_reverse_complement_example(oracle_lib):
    pins.pin_reverse_complement()


def test_fig2_worked_example(oracle_lib):
    pins.pin_fig2()


def test_spurious_edge_example(oracle_lib):
    pins.pin_spurious_edge()


def test_special_cases(oracle_lib):
    pins.pin_special_cases()


def test_exhaustive_against_definition(oracle_lib):
    pins.pin_exhaustive()


def test_single_kmers(oracle_lib):
    pins.pin_single_kmers()


def test_random_sets_against_definition(oracle_lib):
    pins.pin_random_sets()


def test_numpy_unique_pin_k31(oracle_lib):
    rs = synth.plain_small().subset(np.arange(1500))
    g = pins.pin_numpy_unique(rs, 31)
    check_graph(g, 31, rs.bases, rs.offsets)


def test_numpy_unique_pin_k63(oracle_lib):
    rs = synth.plain_large(scale=2e-5)
    rs = rs.subset(np.arange(min(rs.n_reads, 600)))
    g = pins.pin_numpy_unique(rs, 63)
    check_graph(g, 63, rs.bases, rs.offsets)


@pytest.mark.parametrize("k", [1, 3, 15, 33])
def test_numpy_unique_pin_small_k(oracle_lib, k):
    rng = np.random.default_rng(k)
    g = synth.random_genome(rng, 3000)
    rs = synth.sample_reads(rng, g, 200, 80, 0.02)
    pins.pin_numpy_unique(rs, k)


def test_thread_count_does_not_change_result(oracle_lib):
    rs = synth.plain_small().subset(np.arange(800))
    a = oracle.build_graph(rs.bases, rs.offsets, 31, threads=1)
    b = oracle.build_graph(rs.bases, rs.offsets, 31, threads=5)
    for f in ("node_key", "node_count", "edge_u", "edge_v", "edge_orient", "edge_mult", "edge_z"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def _probe_against_build(bases, offsets, k, step_n=37, step_e=41, threads=3):
    g = oracle.build_graph(bases, offsets, k, strings=True)
    sel_n = list(range(0, len(g.node_str), step_n))
    sel_e = list(range(0, len(g.edge_str), step_e))
    absent_n = ["A" * k, "C" * (k - 1) + "A"]
    node_probes = [g.node_str[i] for i in sel_n] + absent_n
    edge_probes = [(g.edge_str[i][0], g.edge_str[i][1], int(g.edge_orient[i])) for i in sel_e]
    # a present edge with its orientation changed is (almost surely) absent
    absent_e = [(e[0], e[1], e[2] ^ 1) for e in edge_probes[:5]]
    nc, ec = oracle.probe_counts(bases, offsets, k, node_probes, edge_probes + absent_e,
                                 threads=threads)
    assert np.array_equal(nc[:len(sel_n)], g.node_count[sel_n])
    assert np.array_equal(ec[:len(sel_e)], g.edge_mult[sel_e])
    mult = {(u, v, int(o)): int(m)
            for (u, v, _, _), o, m in zip(g.edge_str, g.edge_orient, g.edge_mult)}
    for e, c in zip(absent_e, ec[len(sel_e):]):
        assert c == mult.get(e, 0)
    count = {s: int(c) for s, c in zip(g.node_str, g.node_count)}
    for p, c in zip(absent_n, nc[len(sel_n):]):
        assert c == count.get(p, 0)


def test_probe_counts_match_full_build(oracle_lib):
    rs = synth.plain_small().subset(np.arange(500))
    _probe_against_build(rs.bases, rs.offsets, 31)


def test_probe_counts_match_full_build_k63(oracle_lib):
    rs = synth.plain_large(scale=2e-5)
    rs = rs.subset(np.arange(min(rs.n_reads, 400)))
    _probe_against_build(rs.bases, rs.offsets, 63, step_n=11, step_e=13)


def test_probe_counts_palindromes_and_homopolymers(oracle_lib):
    # every probe of small k: palindromic (k+1)-mers, homopolymers, period-2 reads
    reads = ["ACGT", "AAAAAA", "TTTTT", "ACACAC", "TGTGTG", "GGGCCC", "ATAT", "CGCGCG",
             "AATTAATT", "GCATGCAT"]
    bases = "".join(reads).encode()
    offsets = np.zeros(len(reads) + 1, np.uint64)
    np.cumsum([len(r) for r in reads], out=offsets[1:])
    for k in (1, 3, 5):
        _probe_against_build(bases, offsets, k, step_n=1, step_e=1, threads=2)


# ---------------------------------------------------------------------------
# Mutation check: plausible mistakes planted in a copy of the oracle's source
# must each fail at least one pin: in the edge of Sec. 2 (the reading along the
# other strand, the strand bits, which reading names the edge, the tie reading),
# in the canonical form, the enumeration, the packing and the output order.

MUTANTS = {
    "reversal_heads_not_flipped": (r"const Edge against = \{cy, cx, flip\(sy\), flip\(sx\)\};",
                                   "const Edge against = {cy, cx, sy, sx};"),
    "reversal_heads_not_swapped": (r"const Edge against = \{cy, cx, flip\(sy\), flip\(sx\)\};",
                                   "const Edge against = {cy, cx, flip(sx), flip(sy)};"),
    "strand_bit_inverted": (r"const int sx = \(x == cx\) \? PLUS : MINUS;",
                            "const int sx = (x == cx) ? MINUS : PLUS;"),
    "larger_molecule_first": (r"if \(cx < cy\) return along;", "if (cx < cy) return against;"),
    "no_tie_break": (r"return along_first \? along : against;", "return along;"),
    "canonical_is_max": (r"return std::min\(s, reverse_complement\(s\)\);",
                         "return std::max(s, reverse_complement(s));"),
    "complement_not_reversed": (r"std::string r\(s.rbegin\(\), s.rend\(\)\);",
                                "std::string r(s.begin(), s.end());"),
    "drop_last_kmer": (r"for \(uint64_t j = 0; j \+ k <= len; \+\+j\) out->nodes",
                       "for (uint64_t j = 0; j + k < len; ++j) out->nodes"),
    "edge_x_y_swapped": (r"const std::string x = z.substr\(0, k\);",
                         "const std::string x = z.substr(1, k);"),
    "orient_bits_swapped": (r"\(row.e.o1 << 1\) \| row.e.o2", "(row.e.o2 << 1) | row.e.o1"),
    "pack_wrong_code": (r"case 'G': code = 2; break;", "case 'G': code = 3; break;"),
    "edge_order_by_record": (r"return a.z < b.z;", "return a.e < b.e;"),
}


def _run_pins(lib_path):
    rs = synth.plain_small().subset(np.arange(300))
    checks = list(pins.ALL_PINS) + [lambda lib_path=None: pins.pin_numpy_unique(rs, 31, lib_path)]
    for pin in checks:
        try:
            pin(lib_path=lib_path)
        except (AssertionError, RuntimeError, ValueError):
            return False
    return True


def test_pins_pass_on_oracle(oracle_lib):
    assert _run_pins(None)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(oracle_lib, tmp_path, name):
    pattern, repl = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "dbg_oracle.cpp")).read()
    mutated, n = re.subn(pattern, repl, src, count=1)
    assert n == 1, f"mutation {name} did not apply"
    cpp = tmp_path / "mutant.cpp"
    cpp.write_text(mutated)
    so = tmp_path / "mutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-pthread", "-o", str(so),
                    str(cpp)], check=True)
    assert not _run_pins(str(so)), f"planted mistake {name} passed every pin"
