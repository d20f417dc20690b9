// Reference evaluator for positive Datalog -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously correct CPU implementation of what the GPU engine
// computes.  Only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark may load it; the engine itself never links, calls or falls
// back to it.  It shares no code, header, table or helper with the engine.
//
// What it computes (paper Sec. 2, "Datalog"): the least model of a Horn-clause
// program over the loaded facts, i.e. the smallest set of facts that contains
// the inputs and is closed under every rule.  Shared variables in a rule body
// act as equality constraints; comparisons are unsigned 32-bit.  A body atom
// written `!rel(...)` is negated (stratified negation, which the paper lists
// among SRDatalog's features): its relation must lie in a strictly lower
// stratum, every variable in it must occur in a positive body atom, and a
// derivation survives only if that tuple is absent from the (complete)
// relation -- the perfect model of a stratified program.
//
// How (paper Sec. 2):
//   * relations are grouped into strongly connected components of the
//     head->body dependency graph and evaluated stratum by stratum, lower
//     strata first; a finished stratum is read-only afterwards;
//   * a recursive stratum is evaluated semi-naively: each round, every
//     recursive rule is evaluated once per same-stratum body atom with that
//     atom bound to the previous round's delta and every other same-stratum
//     atom bound to the full relation; the new delta is the deduplicated
//     result minus the full relation, then merged into it; the loop stops
//     when every delta of the stratum is empty;
//   * each rule body is evaluated as a left-deep pipeline of nested-loop
//     binary joins in the written atom order: for each atom, an index probe
//     (a sorted copy keyed by the columns already bound) yields the matching
//     tuples, tuple at a time, so nothing intermediate is stored.  Comparisons
//     are applied as soon as both operands are bound.
//
// Round bookkeeping (the reading used for per-round parity): delta 0 of a
// recursive stratum is the stratum's loaded facts together with the results of
// its exit rules (rules with no same-stratum body atom).  Round i evaluates
// the recursive rules over (full_i, delta_i) and yields delta_{i+1}.  The
// recorded sizes are |delta_0|, |delta_1|, ..., ending with the empty delta
// that stopped the loop; "rounds" counts the recursive rounds executed,
// including that last one.
//
// Parity pins (in the test suite): closed forms for paths, cycles and
// complete graphs, BFS reachability and distance layers, matrix-product
// triangle and 4-cycle counts, brute-force enumeration on tiny domains
// (stratum by stratum, negation included), a naive per-round evaluator, and
// an independent points-to worklist solver; mutated copies of this file must
// each fail one of them.

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using u32 = uint32_t;
using u64 = uint64_t;

// ----------------------------------------------------------------------------
// Program representation
// ----------------------------------------------------------------------------

struct Term {
  bool is_var = false;
  u32 v = 0;  // variable id or constant value
};

struct Atom {
  int rel = -1;
  std::vector<Term> t;
};

enum CmpOp { LT = 0, LE = 1, NE = 2 };

struct Cmp {
  int op = LT;  // a op b
  Term a, b;
};

struct Rule {
  Atom head;
  std::vector<Atom> body;
  std::vector<Atom> negs;  // negated atoms: filters over lower strata
  std::vector<Cmp> cmps;
  u32 nvars = 0;
};

// A set of tuples: row-major, rows sorted lexicographically, no duplicates.
struct TupleSet {
  u32 arity = 0;
  std::vector<u32> rows;
  u64 size() const { return arity ? rows.size() / arity : 0; }
};

struct Relation {
  std::string name;
  u32 arity = 0;
  TupleSet full;
  std::vector<u64> delta_sizes;  // per round of its stratum (recursive only)
};

// Sort rows lexicographically and drop duplicates.
void sort_unique(u32 arity, std::vector<u32>& rows) {
  const u64 n = arity ? rows.size() / arity : 0;
  if (n == 0) return;
  std::vector<u64> idx(n);
  for (u64 i = 0; i < n; ++i) idx[i] = i;
  const u32* r = rows.data();
  auto less = [&](u64 a, u64 b) {
    return std::lexicographical_compare(r + a * arity, r + a * arity + arity,
                                        r + b * arity, r + b * arity + arity);
  };
  std::sort(idx.begin(), idx.end(), less);
  std::vector<u32> out;
  out.reserve(rows.size());
  for (u64 k = 0; k < n; ++k) {
    const u32* row = r + idx[k] * arity;
    if (!out.empty() && std::equal(row, row + arity, out.end() - arity)) continue;
    out.insert(out.end(), row, row + arity);
  }
  rows.swap(out);
}

// rows(a) minus rows(b); both sorted and unique.
std::vector<u32> set_minus(u32 arity, const std::vector<u32>& a, const std::vector<u32>& b) {
  std::vector<u32> out;
  u64 na = a.size() / arity, nb = b.size() / arity, j = 0;
  for (u64 i = 0; i < na; ++i) {
    const u32* ra = a.data() + i * arity;
    while (j < nb && std::lexicographical_compare(b.data() + j * arity, b.data() + j * arity + arity, ra, ra + arity)) ++j;
    if (j < nb && std::equal(ra, ra + arity, b.data() + j * arity)) continue;
    out.insert(out.end(), ra, ra + arity);
  }
  return out;
}

// Union of two sorted unique sets.
std::vector<u32> set_union(u32 arity, const std::vector<u32>& a, const std::vector<u32>& b) {
  std::vector<u32> out(a);
  out.insert(out.end(), b.begin(), b.end());
  sort_unique(arity, out);
  return out;
}

// ----------------------------------------------------------------------------
// Parser for the textual rule syntax:
//   head(x, z) :- body1(x, y), body2(y, z), x < z.
// Identifiers in term position are variables ("_" is a fresh anonymous one);
// decimal numbers are constants; comparisons: < <= > >= !=.
// '%' or '//' starts a comment that runs to the end of the line.
// A clause without a body must be ground and adds a fact.
// ----------------------------------------------------------------------------

struct Parser {
  const std::string& s;
  size_t i = 0;
  std::string err;
  explicit Parser(const std::string& src) : s(src) {}

  void skip() {
    for (;;) {
      while (i < s.size() && isspace((unsigned char)s[i])) ++i;
      if (i < s.size() && s[i] == '%') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else if (i + 1 < s.size() && s[i] == '/' && s[i + 1] == '/') {
        while (i < s.size() && s[i] != '\n') ++i;
      } else {
        return;
      }
    }
  }
  bool eof() { skip(); return i >= s.size(); }
  bool peek(const char* t) { skip(); return s.compare(i, strlen(t), t) == 0; }
  bool take(const char* t) {
    if (peek(t)) { i += strlen(t); return true; }
    return false;
  }
  bool ident(std::string& out) {
    skip();
    if (i < s.size() && (isalpha((unsigned char)s[i]) || s[i] == '_')) {
      size_t j = i;
      while (j < s.size() && (isalnum((unsigned char)s[j]) || s[j] == '_')) ++j;
      out = s.substr(i, j - i);
      i = j;
      return true;
    }
    return false;
  }
  bool number(u32& out) {
    skip();
    if (i < s.size() && isdigit((unsigned char)s[i])) {
      u64 v = 0;
      while (i < s.size() && isdigit((unsigned char)s[i])) {
        v = v * 10 + (s[i] - '0');
        if (v > 0xffffffffull) { err = "constant exceeds 32 bits"; return false; }
        ++i;
      }
      out = (u32)v;
      return true;
    }
    return false;
  }
};

}  // namespace

struct oracle_prog {
  std::vector<Relation> rels;
  std::map<std::string, int> rel_ids;
  std::vector<Rule> rules;
  std::vector<std::vector<u32>> pending_facts;  // per relation, row-major
  std::string err;
  u64 rounds = 0;
  double seconds = 0.0;
  bool ran = false;
};

namespace {

bool parse_term(Parser& p, std::map<std::string, u32>& vars, u32& nvars, Term& t) {
  u32 c;
  std::string id;
  if (p.number(c)) { t.is_var = false; t.v = c; return true; }
  if (!p.err.empty()) return false;
  if (p.ident(id)) {
    t.is_var = true;
    if (id == "_") { t.v = nvars++; return true; }
    auto it = vars.find(id);
    if (it == vars.end()) it = vars.emplace(id, nvars++).first;
    t.v = it->second;
    return true;
  }
  p.err = "expected a variable or constant";
  return false;
}

bool parse_atom_args(Parser& p, std::map<std::string, u32>& vars, u32& nvars, Atom& a) {
  if (!p.take("(")) { p.err = "expected '('"; return false; }
  if (!p.take(")")) {
    for (;;) {
      Term t;
      if (!parse_term(p, vars, nvars, t)) return false;
      a.t.push_back(t);
      if (p.take(")")) break;
      if (!p.take(",")) { p.err = "expected ',' or ')'"; return false; }
    }
  }
  return true;
}

int parse_program(oracle_prog* P, const std::string& src) {
  Parser p(src);
  while (!p.eof()) {
    Rule r;
    std::map<std::string, u32> vars;
    std::string name;
    if (!p.ident(name)) { P->err = "expected a relation name"; return -10; }
    auto it = P->rel_ids.find(name);
    if (it == P->rel_ids.end()) { P->err = "unknown relation " + name; return -3; }
    r.head.rel = it->second;
    if (!parse_atom_args(p, vars, r.nvars, r.head)) { P->err = p.err; return -10; }
    if (r.head.t.size() != P->rels[r.head.rel].arity) { P->err = "arity mismatch in " + name; return -2; }
    if (p.take(".")) {  // fact
      std::vector<u32> row;
      for (auto& t : r.head.t) {
        if (t.is_var) { P->err = "a fact must be ground"; return -4; }
        row.push_back(t.v);
      }
      auto& pf = P->pending_facts[r.head.rel];
      pf.insert(pf.end(), row.begin(), row.end());
      continue;
    }
    if (!p.take(":-")) { P->err = "expected ':-' or '.'"; return -10; }
    for (;;) {
      // A negated atom  !name(...)
      if (p.take("!")) {
        std::string nid;
        if (!p.ident(nid) || !p.peek("(")) { P->err = "expected an atom after '!'"; return -10; }
        auto jt = P->rel_ids.find(nid);
        if (jt == P->rel_ids.end()) { P->err = "unknown relation " + nid; return -3; }
        Atom a;
        a.rel = jt->second;
        if (!parse_atom_args(p, vars, r.nvars, a)) { P->err = p.err; return -10; }
        if (a.t.size() != P->rels[a.rel].arity) { P->err = "arity mismatch in " + nid; return -2; }
        r.negs.push_back(a);
        if (p.take(".")) break;
        if (!p.take(",")) { P->err = "expected ',' or '.'"; return -10; }
        continue;
      }
      // Either an atom  name(...)  or a comparison  term op term.
      size_t save = p.i;
      std::string id;
      bool is_atom = false;
      if (p.ident(id)) {
        if (p.peek("(")) is_atom = true;
      }
      if (is_atom) {
        auto jt = P->rel_ids.find(id);
        if (jt == P->rel_ids.end()) { P->err = "unknown relation " + id; return -3; }
        Atom a;
        a.rel = jt->second;
        if (!parse_atom_args(p, vars, r.nvars, a)) { P->err = p.err; return -10; }
        if (a.t.size() != P->rels[a.rel].arity) { P->err = "arity mismatch in " + id; return -2; }
        r.body.push_back(a);
      } else {
        p.i = save;
        Cmp c;
        Term lhs, rhs;
        if (!parse_term(p, vars, r.nvars, lhs)) { P->err = p.err; return -10; }
        int op;
        bool swap = false;
        if (p.take("<=")) op = LE;
        else if (p.take(">=")) { op = LE; swap = true; }
        else if (p.take("!=")) op = NE;
        else if (p.take("<")) op = LT;
        else if (p.take(">")) { op = LT; swap = true; }
        else { P->err = "expected a comparison operator"; return -10; }
        if (!parse_term(p, vars, r.nvars, rhs)) { P->err = p.err; return -10; }
        c.op = op;
        c.a = swap ? rhs : lhs;
        c.b = swap ? lhs : rhs;
        r.cmps.push_back(c);
      }
      if (p.take(".")) break;
      if (!p.take(",")) { P->err = "expected ',' or '.'"; return -10; }
    }
    if (r.body.empty()) { P->err = "a rule needs at least one body atom"; return -4; }
    // Safety: every head and comparison variable occurs in a body atom.
    std::vector<bool> bound(r.nvars, false);
    for (auto& a : r.body)
      for (auto& t : a.t)
        if (t.is_var) bound[t.v] = true;
    for (auto& t : r.head.t)
      if (t.is_var && !bound[t.v]) { P->err = "unsafe rule: unbound head variable"; return -4; }
    for (auto& c : r.cmps)
      if ((c.a.is_var && !bound[c.a.v]) || (c.b.is_var && !bound[c.b.v])) {
        P->err = "unsafe rule: unbound comparison variable";
        return -4;
      }
    for (auto& a : r.negs)
      for (auto& t : a.t)
        if (t.is_var && !bound[t.v]) {
          P->err = "unsafe rule: variable only in a negated atom";
          return -4;
        }
    P->rules.push_back(r);
  }
  return 0;
}

// ----------------------------------------------------------------------------
// Rule evaluation by pipelined nested-loop joins with index probes.
// ----------------------------------------------------------------------------

// A sorted copy of a tuple set with its columns permuted so that the columns
// bound before the atom is reached come first; probed with equal_range.
struct Index {
  u32 arity = 0;
  u32 nbound = 0;
  std::vector<u32> perm;  // perm[j] = original column of permuted column j
  std::vector<u32> rows;  // permuted, sorted, row-major
};

Index build_index(const TupleSet& ts, const std::vector<u32>& perm, u32 nbound) {
  Index ix;
  ix.arity = ts.arity;
  ix.nbound = nbound;
  ix.perm = perm;
  const u64 n = ts.size();
  ix.rows.resize(ts.rows.size());
  for (u64 i = 0; i < n; ++i)
    for (u32 j = 0; j < ts.arity; ++j) ix.rows[i * ts.arity + j] = ts.rows[i * ts.arity + perm[j]];
  sort_unique(ts.arity, ix.rows);
  return ix;
}

// Row range [lo, hi) of an index whose first nbound columns equal key.
std::pair<u64, u64> probe(const Index& ix, const u32* key) {
  const u32 k = ix.arity, nb = ix.nbound;
  const u64 n = k ? ix.rows.size() / k : 0;
  auto cmp_row_key = [&](u64 row) -> int {  // compare row prefix with key
    const u32* r = ix.rows.data() + row * k;
    for (u32 j = 0; j < nb; ++j) {
      if (r[j] < key[j]) return -1;
      if (r[j] > key[j]) return 1;
    }
    return 0;
  };
  u64 lo = 0, hi = n;
  while (lo < hi) {  // first row with prefix >= key
    u64 mid = lo + (hi - lo) / 2;
    if (cmp_row_key(mid) < 0) lo = mid + 1; else hi = mid;
  }
  u64 lo2 = lo, hi2 = n;
  while (lo2 < hi2) {  // first row with prefix > key
    u64 mid = lo2 + (hi2 - lo2) / 2;
    if (cmp_row_key(mid) <= 0) lo2 = mid + 1; else hi2 = mid;
  }
  return {lo, lo2};
}

// Is `key` (arity values) a row of the sorted, unique tuple set?
bool has_row(const TupleSet& ts, const u32* key) {
  const u32 k = ts.arity;
  u64 lo = 0, hi = ts.size();
  while (lo < hi) {
    const u64 mid = lo + (hi - lo) / 2;
    const u32* r = ts.rows.data() + mid * k;
    if (std::lexicographical_compare(r, r + k, key, key + k)) lo = mid + 1; else hi = mid;
  }
  return lo < ts.size() && std::equal(key, key + k, ts.rows.data() + lo * k);
}

bool cmp_holds(int op, u32 a, u32 b) {
  switch (op) {
    case LT: return a < b;
    case LE: return a <= b;
    default: return a != b;
  }
}

struct RulePlan {
  const Rule* rule;
  std::vector<Index> ix;                      // per body atom
  std::vector<std::vector<u32>> key_terms;    // per atom: original columns that are bound on entry
  std::vector<std::vector<int>> cmps_after;   // per atom: comparisons checkable after it
  std::vector<int> cmps_first;                // comparisons over constants only
};

// Rows a thread buffers before deduplicating them early.  A test hook lowers
// it so that small inputs exercise the early deduplication.
u64 g_flush_rows = 1ull << 24;

// Evaluate one rule with body atom i reading sources[i] and negated atom k
// reading negsrc[k]; append head rows.  The body is joined in written order;
// `threads` > 1 splits the first atom's matches across OpenMP threads
// (per-thread buffers joined in thread order).
void eval_rule(const Rule& r, const std::vector<const TupleSet*>& sources,
               const std::vector<const TupleSet*>& negsrc, std::vector<u32>& out, int threads) {
  const size_t na = r.body.size();
  RulePlan pl;
  pl.rule = &r;
  pl.ix.resize(na);
  pl.key_terms.resize(na);
  pl.cmps_after.resize(na);
  std::vector<bool> bound(r.nvars, false);
  for (size_t i = 0; i < na; ++i) {
    const Atom& a = r.body[i];
    std::vector<u32> perm, rest;
    std::vector<bool> local = bound;
    for (u32 j = 0; j < a.t.size(); ++j) {
      const Term& t = a.t[j];
      if (!t.is_var || bound[t.v]) perm.push_back(j); else rest.push_back(j);
    }
    u32 nb = (u32)perm.size();
    pl.key_terms[i] = perm;
    perm.insert(perm.end(), rest.begin(), rest.end());
    pl.ix[i] = build_index(*sources[i], perm, nb);
    for (auto& t : a.t)
      if (t.is_var) bound[t.v] = true;
  }
  // Place each comparison after the first atom that binds all its variables.
  std::vector<bool> b2(r.nvars, false);
  std::vector<bool> placed(r.cmps.size(), false);
  for (size_t c = 0; c < r.cmps.size(); ++c) {
    const Cmp& cm = r.cmps[c];
    if (!cm.a.is_var && !cm.b.is_var) { pl.cmps_first.push_back((int)c); placed[c] = true; }
  }
  for (size_t i = 0; i < na; ++i) {
    for (auto& t : r.body[i].t)
      if (t.is_var) b2[t.v] = true;
    for (size_t c = 0; c < r.cmps.size(); ++c) {
      if (placed[c]) continue;
      const Cmp& cm = r.cmps[c];
      if ((!cm.a.is_var || b2[cm.a.v]) && (!cm.b.is_var || b2[cm.b.v])) {
        pl.cmps_after[i].push_back((int)c);
        placed[c] = true;
      }
    }
  }
  for (int c : pl.cmps_first) {
    const Cmp& cm = r.cmps[c];
    if (!cmp_holds(cm.op, cm.a.v, cm.b.v)) return;
  }

  // For each atom, its free columns (in index order) with the variable they
  // bind and whether that is the variable's first occurrence in the atom
  // (a repeated variable must then agree with the first occurrence).
  struct FreeCol { u32 j; u32 var; bool first; };
  std::vector<std::vector<FreeCol>> freecols(na);
  for (size_t i = 0; i < na; ++i) {
    const Index& ix = pl.ix[i];
    std::vector<bool> seen(r.nvars, false);
    for (u32 j = ix.nbound; j < ix.arity; ++j) {
      const Term& t = r.body[i].t[ix.perm[j]];
      freecols[i].push_back({j, t.v, !seen[t.v]});
      seen[t.v] = true;
    }
  }

  // Depth-first nested loops over the atoms.  Which variables are bound at
  // each atom is fixed by the written order, so values are simply
  // overwritten on the way down.
  struct Walker {
    const Rule& r;
    const RulePlan& pl;
    const std::vector<std::vector<FreeCol>>& fc;
    std::vector<u32> val;
    std::vector<u32>* out;
    const std::vector<const TupleSet*>& neg;
    u32 term_val(const Term& t) const { return t.is_var ? val[t.v] : t.v; }
    // A derivation survives when no negated atom's tuple is present.
    bool negs_absent() const {
      u32 key[64];
      for (size_t k = 0; k < r.negs.size(); ++k) {
        for (size_t j = 0; j < r.negs[k].t.size(); ++j) key[j] = term_val(r.negs[k].t[j]);
        if (has_row(*neg[k], key)) return false;
      }
      return true;
    }
    bool bind(size_t i, const u32* row) {
      for (const FreeCol& f : fc[i]) {
        if (f.first) val[f.var] = row[f.j];
        else if (val[f.var] != row[f.j]) return false;
      }
      return true;
    }
    bool cmps_ok(size_t i) const {
      for (int c : pl.cmps_after[i]) {
        const Cmp& cm = r.cmps[c];
        if (!cmp_holds(cm.op, term_val(cm.a), term_val(cm.b))) return false;
      }
      return true;
    }
    void emit() {
      if (!negs_absent()) return;
      for (auto& t : r.head.t) out->push_back(term_val(t));
    }
    void walk(size_t i) {
      if (i == r.body.size()) { emit(); return; }
      const Index& ix = pl.ix[i];
      u32 key[64];
      u32 nk = 0;
      for (u32 j : pl.key_terms[i]) key[nk++] = term_val(r.body[i].t[j]);
      auto rg = probe(ix, key);
      for (u64 k = rg.first; k < rg.second; ++k) {
        if (bind(i, ix.rows.data() + k * ix.arity) && cmps_ok(i)) walk(i + 1);
      }
    }
  };

  // Outermost atom: enumerate its matches (no variable is bound yet).
  const Index& ix0 = pl.ix[0];
  std::vector<u32> key0;
  for (u32 j : pl.key_terms[0]) key0.push_back(r.body[0].t[j].v);
  auto rg0 = probe(ix0, key0.data());
  const u64 lo = rg0.first, hi = rg0.second;
  int nt = threads > 0 ? threads : 1;
  std::vector<std::vector<u32>> bufs(nt);
#pragma omp parallel num_threads(nt) if (nt > 1)
  {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    Walker w{r, pl, freecols, std::vector<u32>(r.nvars, 0), &bufs[tid], negsrc};
    // Static contiguous split: thread t takes a contiguous block of rows, so
    // joining the buffers in thread order reproduces the sequential order.
    u64 n = hi - lo, per = (n + nt - 1) / nt;
    u64 b = lo + std::min<u64>(n, per * tid), e = lo + std::min<u64>(n, per * (tid + 1));
    const u64 ha = r.head.t.size();
    u64 limit = g_flush_rows;
    for (u64 k = b; k < e; ++k) {
      if (w.bind(0, ix0.rows.data() + k * ix0.arity) && w.cmps_ok(0)) w.walk(1);
      // Keep per-thread candidate buffers bounded: deduplicating early does
      // not change the set that is produced.  The next flush waits until the
      // buffer has doubled past its deduplicated size.
      if (ha && bufs[tid].size() / ha > limit) {
        sort_unique((u32)ha, bufs[tid]);
        limit = std::max<u64>(g_flush_rows, 2 * (bufs[tid].size() / ha));
      }
    }
  }
  for (auto& b : bufs) out.insert(out.end(), b.begin(), b.end());
}

// ----------------------------------------------------------------------------
// Stratification: strongly connected components of the dependency graph
// (head relation depends on each body relation), emitted dependencies first.
// ----------------------------------------------------------------------------

std::vector<std::vector<int>> strata(const oracle_prog* P) {
  const int n = (int)P->rels.size();
  std::vector<std::vector<int>> dep(n);
  for (auto& r : P->rules) {
    for (auto& a : r.body) dep[r.head.rel].push_back(a.rel);
    for (auto& a : r.negs) dep[r.head.rel].push_back(a.rel);
  }
  // Tarjan's algorithm (iterative bookkeeping kept simple with recursion;
  // programs here have few relations).
  std::vector<int> index(n, -1), low(n, 0), stack;
  std::vector<bool> on(n, false);
  std::vector<std::vector<int>> out;
  int counter = 0;
  struct Frame { int v; size_t e; };
  for (int s = 0; s < n; ++s) {
    if (index[s] >= 0) continue;
    std::vector<Frame> call{{s, 0}};
    index[s] = low[s] = counter++;
    stack.push_back(s);
    on[s] = true;
    while (!call.empty()) {
      Frame& f = call.back();
      if (f.e < dep[f.v].size()) {
        int w = dep[f.v][f.e++];
        if (index[w] < 0) {
          index[w] = low[w] = counter++;
          stack.push_back(w);
          on[w] = true;
          call.push_back({w, 0});
        } else if (on[w]) {
          low[f.v] = std::min(low[f.v], index[w]);
        }
      } else {
        int v = f.v;
        call.pop_back();
        if (!call.empty()) low[call.back().v] = std::min(low[call.back().v], low[v]);
        if (low[v] == index[v]) {
          std::vector<int> comp;
          for (;;) {
            int w = stack.back();
            stack.pop_back();
            on[w] = false;
            comp.push_back(w);
            if (w == v) break;
          }
          std::sort(comp.begin(), comp.end());
          out.push_back(comp);  // every component it depends on is already out
        }
      }
    }
  }
  return out;
}

int run_program(oracle_prog* P, int threads) {
  // Stratification: a negated relation must be finished before the rule's
  // head is computed, i.e. lie in another (hence lower) component.
  {
    auto cs = strata(P);
    std::vector<size_t> comp_of(P->rels.size(), 0);
    for (size_t ci = 0; ci < cs.size(); ++ci)
      for (int x : cs[ci]) comp_of[x] = ci;
    for (auto& r : P->rules)
      for (auto& a : r.negs)
        if (comp_of[a.rel] == comp_of[r.head.rel]) {
          P->err = "program not stratifiable: negation inside a recursive component";
          return -5;
        }
  }
  for (size_t r = 0; r < P->rels.size(); ++r) {
    auto& rel = P->rels[r];
    auto& pf = P->pending_facts[r];
    rel.full.arity = rel.arity;
    rel.full.rows.insert(rel.full.rows.end(), pf.begin(), pf.end());
    pf.clear();
    sort_unique(rel.arity, rel.full.rows);
    rel.delta_sizes.clear();
  }
  P->rounds = 0;
  auto comps = strata(P);
  for (auto& comp : comps) {
    std::vector<bool> in(P->rels.size(), false);
    for (int x : comp) in[x] = true;
    std::vector<const Rule*> exit_rules, rec_rules;
    for (auto& r : P->rules) {
      if (!in[r.head.rel]) continue;
      bool rec = false;
      for (auto& a : r.body)
        if (in[a.rel]) rec = true;
      (rec ? rec_rules : exit_rules).push_back(&r);
    }
    // Exit rules read only finished relations.
    std::map<int, std::vector<u32>> fresh;
    for (const Rule* r : exit_rules) {
      std::vector<const TupleSet*> src, nsrc;
      for (auto& a : r->body) src.push_back(&P->rels[a.rel].full);
      for (auto& a : r->negs) nsrc.push_back(&P->rels[a.rel].full);
      eval_rule(*r, src, nsrc, fresh[r->head.rel], threads);
    }
    for (auto& kv : fresh) {
      auto& rel = P->rels[kv.first];
      sort_unique(rel.arity, kv.second);
      rel.full.rows = set_union(rel.arity, rel.full.rows, kv.second);
    }
    if (rec_rules.empty()) continue;
    // Semi-naive rounds.
    std::map<int, TupleSet> delta;
    for (int x : comp) {
      delta[x] = P->rels[x].full;  // delta_0: loaded facts and exit results
      P->rels[x].delta_sizes.push_back(delta[x].size());
    }
    for (;;) {
      std::map<int, std::vector<u32>> cand;
      for (const Rule* r : rec_rules) {
        for (size_t j = 0; j < r->body.size(); ++j) {
          if (!in[r->body[j].rel]) continue;
          std::vector<const TupleSet*> src;
          for (size_t i = 0; i < r->body.size(); ++i) {
            int rel = r->body[i].rel;
            src.push_back(i == j ? &delta[rel] : &P->rels[rel].full);
          }
          std::vector<const TupleSet*> nsrc;
          for (auto& a : r->negs) nsrc.push_back(&P->rels[a.rel].full);
          eval_rule(*r, src, nsrc, cand[r->head.rel], threads);
        }
      }
      bool any = false;
      std::map<int, TupleSet> next;
      for (int x : comp) {
        auto& rel = P->rels[x];
        std::vector<u32> c = std::move(cand[x]);
        sort_unique(rel.arity, c);
        TupleSet d;
        d.arity = rel.arity;
        d.rows = set_minus(rel.arity, c, rel.full.rows);
        if (d.size()) any = true;
        next[x] = std::move(d);
      }
      for (int x : comp) {
        auto& rel = P->rels[x];
        rel.full.rows = set_union(rel.arity, rel.full.rows, next[x].rows);
        rel.delta_sizes.push_back(next[x].size());
      }
      delta = std::move(next);
      ++P->rounds;
      if (!any) break;
    }
  }
  return 0;
}

}  // namespace

// ----------------------------------------------------------------------------
// C entry points (used from Python through ctypes by the tests and the
// CPU-baseline leg of the benchmark).
// ----------------------------------------------------------------------------

extern "C" {

oracle_prog* oracle_create(void) { return new oracle_prog(); }

void oracle_destroy(oracle_prog* P) { delete P; }

const char* oracle_error(const oracle_prog* P) { return P ? P->err.c_str() : "null program"; }

int oracle_declare(oracle_prog* P, const char* name, uint32_t arity) {
  if (!P || !name || arity == 0) return -1;
  if (P->rel_ids.count(name)) { P->err = "relation declared twice"; return -1; }
  Relation r;
  r.name = name;
  r.arity = arity;
  r.full.arity = arity;
  P->rel_ids[name] = (int)P->rels.size();
  P->rels.push_back(r);
  P->pending_facts.emplace_back();
  return 0;
}

int oracle_add_rules(oracle_prog* P, const char* text) {
  if (!P || !text) return -1;
  return parse_program(P, text);
}

// rows: row-major n x arity.
int oracle_load(oracle_prog* P, const char* name, const uint32_t* rows, uint64_t n) {
  if (!P || !name) return -1;
  auto it = P->rel_ids.find(name);
  if (it == P->rel_ids.end()) { P->err = "unknown relation"; return -3; }
  auto& pf = P->pending_facts[it->second];
  pf.insert(pf.end(), rows, rows + n * P->rels[it->second].arity);
  return 0;
}

int oracle_run(oracle_prog* P, int threads, double* seconds) {
  if (!P) return -1;
  auto t0 = std::chrono::steady_clock::now();
  int rc = run_program(P, threads);
  auto t1 = std::chrono::steady_clock::now();
  P->seconds = std::chrono::duration<double>(t1 - t0).count();
  if (seconds) *seconds = P->seconds;
  P->ran = true;
  return rc;
}

uint64_t oracle_size(const oracle_prog* P, const char* name) {
  auto it = P->rel_ids.find(name);
  if (it == P->rel_ids.end()) return 0;
  return P->rels[it->second].full.size();
}

int oracle_read(const oracle_prog* P, const char* name, uint32_t* out) {
  auto it = P->rel_ids.find(name);
  if (it == P->rel_ids.end()) return -3;
  const auto& rows = P->rels[it->second].full.rows;
  std::memcpy(out, rows.data(), rows.size() * sizeof(u32));
  return 0;
}

uint64_t oracle_rounds(const oracle_prog* P) { return P->rounds; }

// Test hook: per-thread rows buffered before an early deduplication (0 restores
// the default of 2^24).
void oracle_set_flush_rows(uint64_t rows) { g_flush_rows = rows ? rows : (1ull << 24); }

// Writes up to cap delta sizes of the relation; returns how many exist.
uint64_t oracle_delta_sizes(const oracle_prog* P, const char* name, uint64_t* out, uint64_t cap) {
  auto it = P->rel_ids.find(name);
  if (it == P->rel_ids.end()) return 0;
  const auto& d = P->rels[it->second].delta_sizes;
  for (uint64_t i = 0; i < d.size() && i < cap; ++i) out[i] = d[i];
  return d.size();
}

}  // extern "C"
