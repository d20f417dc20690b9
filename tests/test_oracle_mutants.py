"""The oracle's pins catch plausible mistakes (CPU only).

Each mutant is a copy of ``oracle/oracle.cpp`` with one deliberate slip -- a
dropped term, a wrong index or bound, a swapped operand, a skipped step --
compiled (with OpenMP, as the oracle itself is) into a scratch library and
loaded (through ``ORACLE_LIB_PATH``) by the pin suite
``tests/test_oracle_pins.py`` in a process of its own; that suite runs every
pin with the sequential and with the threaded evaluation.  Every
mutant must fail at least one pin; the unmutated source, compiled the same
way, must pass them all (so a broken harness cannot pass as "detected").
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")

# (name, exact text in oracle.cpp, replacement)
MUTANTS = [
    ("delta_for_every_recursive_atom",
     "src.push_back(i == j ? &delta[rel] : &P->rels[rel].full);",
     "src.push_back(in[rel] ? &delta[rel] : &P->rels[rel].full);"),
    ("delta_version_of_first_atom_only",
     "        for (size_t j = 0; j < r->body.size(); ++j) {\n          if (!in[r->body[j].rel]) continue;",
     "        for (size_t j = 0; j < 1; ++j) {\n          if (!in[r->body[j].rel]) continue;"),
    ("probe_upper_bound_excludes_equal",
     "if (cmp_row_key(mid) <= 0) lo2 = mid + 1; else hi2 = mid;",
     "if (cmp_row_key(mid) < 0) lo2 = mid + 1; else hi2 = mid;"),
    ("strict_less_taken_as_less_equal",
     "case LT: return a < b;",
     "case LT: return a <= b;"),
    ("greater_not_swapped",
     "c.a = swap ? rhs : lhs;\n        c.b = swap ? lhs : rhs;",
     "c.a = lhs;\n        c.b = rhs;"),
    ("repeated_variable_not_checked",
     "else if (val[f.var] != row[f.j]) return false;",
     "else if (false) return false;"),
    ("duplicates_kept",
     "if (!out.empty() && std::equal(row, row + arity, out.end() - arity)) continue;",
     "if (false) continue;"),
    ("strata_in_reverse_order",
     "  for (auto& comp : comps) {",
     "  std::reverse(comps.begin(), comps.end());\n  for (auto& comp : comps) {"),
    ("empty_first_delta",
     "delta[x] = P->rels[x].full;  // delta_0: loaded facts and exit results",
     "delta[x] = TupleSet{P->rels[x].arity, {}};"),
    ("final_empty_round_not_counted",
     "      ++P->rounds;\n      if (!any) break;",
     "      if (!any) break;\n      ++P->rounds;"),
    ("comparisons_ignored",
     "if (!cmp_holds(cm.op, term_val(cm.a), term_val(cm.b))) return false;",
     "if (false) return false;"),
    ("head_columns_reversed",
     "for (auto& t : r.head.t) out->push_back(term_val(t));",
     "for (auto it = r.head.t.rbegin(); it != r.head.t.rend(); ++it) out->push_back(term_val(*it));"),
    ("exit_results_dropped",
     "rel.full.rows = set_union(rel.arity, rel.full.rows, kv.second);",
     "(void)kv;"),
    ("negated_atoms_ignored",
     "if (!negs_absent()) return;",
     "(void)0;"),
    ("negation_not_a_dependency",
     "    for (auto& a : r.negs) dep[r.head.rel].push_back(a.rel);\n",
     ""),
    # Slips in the threaded mode (only the pins run with several threads
    # reach them): a thread block that stops one row early, the buffers of
    # the other threads dropped, an early deduplication with the wrong arity.
    ("thread_block_drops_last_row",
     "e = lo + std::min<u64>(n, per * (tid + 1));",
     "e = lo + std::min<u64>(n, per * (tid + 1) - (tid + 1 < nt ? 1 : 0));"),
    ("first_thread_buffer_only",
     "for (auto& b : bufs) out.insert(out.end(), b.begin(), b.end());",
     "out.insert(out.end(), bufs[0].begin(), bufs[0].end());"),
    ("early_dedup_wrong_arity",
     "sort_unique((u32)ha, bufs[tid]);",
     "sort_unique(1, bufs[tid]);"),
    ("difference_matches_first_column_only",
     "if (j < nb && std::equal(ra, ra + arity, b.data() + j * arity)) continue;",
     "if (j < nb && std::equal(ra, ra + 1, b.data() + j * arity)) continue;"),
]


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    """Compile the control and every mutant in parallel."""
    src = open(SRC).read()
    d = tmp_path_factory.mktemp("oracle_mutants")
    procs, libs = {}, {}
    for name, old, new in [("control", "", "")] + MUTANTS:
        if name == "control":
            text = src
        else:
            assert src.count(old) == 1, name
            text = src.replace(old, new)
        cpp = d / f"{name}.cpp"
        cpp.write_text(text)
        libs[name] = str(d / f"lib{name}.so")
        procs[name] = subprocess.Popen(["g++", "-std=c++17", "-O1", "-fopenmp", "-shared", "-fPIC", "-o",
                                        libs[name], str(cpp)], stderr=subprocess.PIPE)
    for name, p in procs.items():
        _, err = p.communicate()
        assert p.returncode == 0, (name, err.decode()[-2000:])
    return libs


def run_pins(lib):
    env = dict(os.environ, ORACLE_LIB_PATH=lib)
    try:
        r = subprocess.run([sys.executable, "-m", "pytest", "tests/test_oracle_pins.py", "-x", "-q",
                            "-p", "no:cacheprovider"], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=120)
    except subprocess.TimeoutExpired:
        return None, "timed out"
    return r.returncode, r.stdout[-1500:]


def test_control_passes_every_pin(builds):
    rc, out = run_pins(builds["control"])
    assert rc == 0, out


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_fails_a_pin(builds, name):
    rc, out = run_pins(builds[name])
    assert rc not in (0, None), (name, out)
