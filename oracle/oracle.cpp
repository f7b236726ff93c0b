// Oracle: a plain, slow, obviously correct CPU evaluation of basic graph
// patterns (BGPs) over an RDF triple set.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the benchmark's CPU
// baseline leg use it.  It shares no code, header or table with the GPU
// library.
//
// What it computes (paper Sec. 3.1, Sec. 6 "procedure of SM-based BGP query
// evaluation", Sec. 6.1 last paragraphs):
//   * The dataset D is a SET of (s, p, o) triples (Sec. 3.1), so duplicates in
//     the input are removed first.
//   * Each triple pattern (TP) t_i is initialised as the relation R_i of the
//     variable bindings it matches on its own (Sec. 6, step "Initializing").
//   * Relations are joined pairwise on their common variables, the schema of a
//     join being the distinct union of the two schemas (Sec. 6, step
//     "Joining"); the join keeps every matching pair (no accumulation of a
//     value column: the boolean reading of the sparse-matrix product in
//     Sec. 6.1).
//   * The final relation over all variables is returned (step "Returning"),
//     here as rows in variable-number order, sorted lexicographically.
//
// Join order: query order repaired for connectivity (start with TP 0, then
// repeatedly the lowest-numbered remaining TP that shares a variable with the
// bound set, else the lowest-numbered remaining TP).  This deliberately
// ignores the paper's statistics-based plan; the result does not depend on
// the order.  Each join is a hash join keyed on the shared variables, or a
// nested-loop Cartesian product when none is shared.
//
// Pattern encoding: endpoint >= 0 is a vertex constant; endpoint < 0 is the
// variable -(x+1).  The predicate is always a constant (Sec. 6.3 assumes a
// known predicate).
//
// A second evaluation of the same definition runs on every host core
// (OpenMP), for the benchmark's CPU baseline: the same join order, each
// pattern's relation gathered by a parallel scan of D, each later relation
// keyed on its shared variables once (pairs of key and row, sorted in
// parallel, probed by binary search), the first relation's rows split into
// one contiguous range per thread, each range carried through all later
// joins, and a parallel sort of the rows.  Its output equals the
// single-threaded evaluation's (tested).
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <memory>
#include <parallel/algorithm>
#include <unordered_map>
#include <vector>

namespace {

struct Triple {
  int32_t s, p, o;
  bool operator<(const Triple& b) const {
    if (s != b.s) return s < b.s;
    if (p != b.p) return p < b.p;
    return o < b.o;
  }
  bool operator==(const Triple& b) const { return s == b.s && p == b.p && o == b.o; }
};

// A relation: schema (variable numbers) and row-major values.
struct Relation {
  std::vector<int32_t> vars;
  std::vector<int32_t> vals;
  int64_t rows = 0;
};

std::vector<Triple> dedupe(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n) {
  std::vector<Triple> d(n);
  for (int64_t i = 0; i < n; ++i) d[i] = Triple{s[i], p[i], o[i]};
  std::sort(d.begin(), d.end());
  d.erase(std::unique(d.begin(), d.end()), d.end());
  return d;
}

// R_i: the bindings of the TP's variables for which the instantiated TP is in D.
Relation tp_relation(const std::vector<Triple>& D, int32_t ts, int32_t tp, int32_t to) {
  Relation r;
  bool sv = ts < 0, ov = to < 0;
  int32_t xs = sv ? -ts - 1 : -1, xo = ov ? -to - 1 : -1;
  if (sv) r.vars.push_back(xs);
  if (ov && !(sv && xo == xs)) r.vars.push_back(xo);
  for (const Triple& t : D) {
    if (t.p != tp) continue;
    if (!sv && t.s != ts) continue;
    if (!ov && t.o != to) continue;
    if (sv && ov && xs == xo && t.s != t.o) continue;
    if (sv) r.vals.push_back(t.s);
    if (ov && !(sv && xo == xs)) r.vals.push_back(t.o);
    ++r.rows;
  }
  return r;
}

uint64_t pack_key(const int32_t* row, const std::vector<int>& cols) {
  uint64_t k = 0;
  for (int c : cols) k = (k << 32) | (uint32_t)row[c];
  return k;
}

// Natural join of a (current) and b (a TP relation with at most 2 variables).
// Stops (returning rows = cap + 1) once more than cap rows exist, cap >= 0.
Relation join(const Relation& a, const Relation& b, int64_t cap) {
  std::vector<int> a_shared, b_shared, b_new;
  for (size_t j = 0; j < b.vars.size(); ++j) {
    auto it = std::find(a.vars.begin(), a.vars.end(), b.vars[j]);
    if (it != a.vars.end()) {
      a_shared.push_back((int)(it - a.vars.begin()));
      b_shared.push_back((int)j);
    } else {
      b_new.push_back((int)j);
    }
  }
  Relation out;
  out.vars = a.vars;
  for (int j : b_new) out.vars.push_back(b.vars[j]);
  const size_t wa = a.vars.size(), wb = b.vars.size();
  if (b_shared.empty()) {  // Cartesian product
    for (int64_t i = 0; i < a.rows; ++i)
      for (int64_t j = 0; j < b.rows; ++j) {
        for (size_t c = 0; c < wa; ++c) out.vals.push_back(a.vals[i * wa + c]);
        for (int c : b_new) out.vals.push_back(b.vals[j * wb + c]);
        if (++out.rows > cap && cap >= 0) return out;
      }
    return out;
  }
  std::unordered_multimap<uint64_t, int64_t> h;
  h.reserve((size_t)b.rows * 2 + 1);
  for (int64_t j = 0; j < b.rows; ++j) h.emplace(pack_key(&b.vals[j * wb], b_shared), j);
  for (int64_t i = 0; i < a.rows; ++i) {
    auto range = h.equal_range(pack_key(&a.vals[i * wa], a_shared));
    for (auto it = range.first; it != range.second; ++it) {
      int64_t j = it->second;
      for (size_t c = 0; c < wa; ++c) out.vals.push_back(a.vals[i * wa + c]);
      for (int c : b_new) out.vals.push_back(b.vals[j * wb + c]);
      if (++out.rows > cap && cap >= 0) return out;
    }
  }
  return out;
}

std::vector<int> join_order(const int32_t* tps, int32_t ntp, int32_t nvars) {
  std::vector<int> order;
  std::vector<char> used(ntp, 0), bound(nvars > 0 ? nvars : 1, 0);
  for (int step = 0; step < ntp; ++step) {
    int pick = -1;
    for (int t = 0; t < ntp && pick < 0; ++t) {
      if (used[t]) continue;
      int32_t s = tps[3 * t], o = tps[3 * t + 2];
      if ((s < 0 && bound[-s - 1]) || (o < 0 && bound[-o - 1])) pick = t;
    }
    for (int t = 0; t < ntp && pick < 0; ++t)
      if (!used[t]) pick = t;
    used[pick] = 1;
    order.push_back(pick);
    if (tps[3 * pick] < 0) bound[-tps[3 * pick] - 1] = 1;
    if (tps[3 * pick + 2] < 0) bound[-tps[3 * pick + 2] - 1] = 1;
  }
  return order;
}

struct Result {
  int32_t nvars = 0;
  int64_t rows = 0;
  std::vector<int32_t> vals;  // sorted, row-major, variable order
};

inline uint64_t mix64(uint64_t z) {
  z ^= z >> 30; z *= 0xbf58476d1ce4e5b9ULL;
  z ^= z >> 27; z *= 0x94d049bb133111ebULL;
  z ^= z >> 31;
  return z;
}

// R_i gathered by a parallel scan of D: threads take contiguous ranges of D
// and their rows are concatenated in range order, so the relation equals
// tp_relation's.
Relation tp_relation_par(const std::vector<Triple>& D, int32_t ts, int32_t tp, int32_t to,
                         int threads) {
  Relation r;
  const bool sv = ts < 0, ov = to < 0;
  const int32_t xs = sv ? -ts - 1 : -1, xo = ov ? -to - 1 : -1;
  const bool two = ov && !(sv && xo == xs);
  if (sv) r.vars.push_back(xs);
  if (two) r.vars.push_back(xo);
  const int64_t n = (int64_t)D.size();
  std::vector<std::vector<int32_t>> part(threads);
#pragma omp parallel num_threads(threads)
  {
    const int t = omp_get_thread_num();
    const int64_t a = n * t / threads, b = n * (t + 1) / threads;
    std::vector<int32_t>& v = part[t];
    for (int64_t i = a; i < b; ++i) {
      const Triple& x = D[i];
      if (x.p != tp) continue;
      if (!sv && x.s != ts) continue;
      if (!ov && x.o != to) continue;
      if (sv && ov && xs == xo && x.s != x.o) continue;
      if (sv) v.push_back(x.s);
      if (two) v.push_back(x.o);
    }
  }
  const size_t w = r.vars.size();
  for (auto& v : part) {
    r.vals.insert(r.vals.end(), v.begin(), v.end());
    r.rows += w ? (int64_t)(v.size() / w) : 0;
  }
  if (w == 0) {  // all-constant pattern: one empty row per matching triple
    int64_t m = 0;
    for (const Triple& x : D) m += x.p == tp && x.s == ts && x.o == to;
    r.rows = m;
  }
  return r;
}

}  // namespace

extern "C" {

// Sorted distinct triples of the input; returns their number.  Output arrays
// (may be null to query the count) must hold n entries.
int64_t oracle_dedupe(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                      int32_t* s_out, int32_t* p_out, int32_t* o_out) {
  std::vector<Triple> d = dedupe(s, p, o, n);
  if (s_out)
    for (size_t i = 0; i < d.size(); ++i) { s_out[i] = d[i].s; p_out[i] = d[i].p; o_out[i] = d[i].o; }
  return (int64_t)d.size();
}

// The h-index sparse matrix of predicate `pred` (Sec. 5.3) in compressed form:
// orient 0 groups the (s, o) pairs by subject (rows = subjects, members =
// objects), orient 1 by object.  keys: distinct row ids ascending (the "Row"
// array of Sec. 6.3), ptr: nr+1 offsets (the "Rpos" array, 0-based; "Num" is
// the difference), nbr: members ascending within each row.  Returns nnz; with
// null outputs, only nnz and *nr are computed.
int64_t oracle_csr(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n, int32_t pred,
                   int32_t orient, int64_t* nr, int32_t* keys, int32_t* ptr, int32_t* nbr) {
  std::vector<Triple> d = dedupe(s, p, o, n);
  std::vector<std::pair<int32_t, int32_t>> pairs;
  for (const Triple& t : d)
    if (t.p == pred) pairs.emplace_back(orient == 0 ? t.s : t.o, orient == 0 ? t.o : t.s);
  std::sort(pairs.begin(), pairs.end());
  int64_t r = 0;
  for (size_t i = 0; i < pairs.size(); ++i) {
    bool head = i == 0 || pairs[i].first != pairs[i - 1].first;
    if (head) {
      if (keys) { keys[r] = pairs[i].first; ptr[r] = (int32_t)i; }
      ++r;
    }
    if (nbr) nbr[i] = pairs[i].second;
  }
  if (ptr) ptr[r] = (int32_t)pairs.size();
  *nr = r;
  return (int64_t)pairs.size();
}

// A dataset handle: the deduplicated triple set, built once and reused by
// oracle_join_dataset (so repeated queries do not pay the set construction).
void* oracle_dataset_new(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n) {
  return new std::vector<Triple>(dedupe(s, p, o, n));
}
void oracle_dataset_free(void* ds) { delete static_cast<std::vector<Triple>*>(ds); }

static void* join_impl(const std::vector<Triple>& D, const int32_t* tps, int32_t ntp,
                       int32_t nvars, int64_t cap_rows);

// Evaluates the BGP.  Returns an opaque result handle (null on invalid input).
// Rows beyond cap_rows (if cap_rows >= 0) make the call return null.
void* oracle_join(const int32_t* s, const int32_t* p, const int32_t* o, int64_t n,
                  const int32_t* tps, int32_t ntp, int32_t nvars, int64_t cap_rows) {
  if (ntp < 0 || nvars < 0) return nullptr;
  std::vector<Triple> D = dedupe(s, p, o, n);
  return join_impl(D, tps, ntp, nvars, cap_rows);
}

void* oracle_join_dataset(void* ds, const int32_t* tps, int32_t ntp, int32_t nvars,
                          int64_t cap_rows) {
  if (!ds || ntp < 0 || nvars < 0) return nullptr;
  return join_impl(*static_cast<std::vector<Triple>*>(ds), tps, ntp, nvars, cap_rows);
}

// The same evaluation on `threads` host threads (see the file comment).
void* oracle_join_dataset_omp(void* ds, const int32_t* tps, int32_t ntp, int32_t nvars,
                              int64_t cap_rows, int32_t threads) {
  if (!ds || ntp <= 0 || nvars < 0 || threads < 1) return nullptr;
  const std::vector<Triple>& D = *static_cast<std::vector<Triple>*>(ds);
  std::vector<int> order = join_order(tps, ntp, nvars);
  std::vector<Relation> rel(ntp);
  for (int j = 0; j < ntp; ++j) {
    const int t = order[j];
    rel[j] = tp_relation_par(D, tps[3 * t], tps[3 * t + 1], tps[3 * t + 2], threads);
  }
  // the schema after each join, and per later relation its shared and new
  // columns and a hash table on the shared ones
  std::vector<std::vector<int>> a_shared(ntp), b_shared(ntp), b_new(ntp);
  std::vector<int32_t> vars = rel[0].vars;
  // per later relation: (key of its shared columns, row), sorted in parallel
  std::vector<std::vector<std::pair<uint64_t, int64_t>>> keyed(ntp);
  for (int j = 1; j < ntp; ++j) {
    const Relation& b = rel[j];
    for (size_t c = 0; c < b.vars.size(); ++c) {
      auto it = std::find(vars.begin(), vars.end(), b.vars[c]);
      if (it != vars.end()) {
        a_shared[j].push_back((int)(it - vars.begin()));
        b_shared[j].push_back((int)c);
      } else {
        b_new[j].push_back((int)c);
      }
    }
    for (int c : b_new[j]) vars.push_back(b.vars[c]);
    if (!b_shared[j].empty()) {
      const size_t wb = b.vars.size();
      std::vector<std::pair<uint64_t, int64_t>>& kv = keyed[j];
      kv.resize((size_t)b.rows);
#pragma omp parallel for num_threads(threads)
      for (int64_t r = 0; r < b.rows; ++r) kv[r] = {pack_key(&b.vals[r * wb], b_shared[j]), r};
      __gnu_parallel::sort(kv.begin(), kv.end());
    }
  }
  if ((int32_t)vars.size() != nvars) return nullptr;
  // the first relation's rows in one contiguous range per thread, each
  // carried through every later join
  const int64_t n0 = rel[0].rows;
  if (cap_rows >= 0 && n0 > cap_rows) return nullptr;
  const size_t w0 = rel[0].vars.size();
  std::vector<Relation> out(threads);
  std::atomic<int64_t> total{0};
  std::atomic<bool> over{false};
  // rows after each join, summed over the threads (an intermediate above the
  // cap stops the evaluation, as in the single-threaded one)
  std::unique_ptr<std::atomic<int64_t>[]> step_rows(new std::atomic<int64_t>[ntp]);
  for (int j = 0; j < ntp; ++j) step_rows[j] = 0;
#pragma omp parallel num_threads(threads)
  {
    const int t = omp_get_thread_num();
    Relation cur;
    cur.vars = rel[0].vars;
    const int64_t a = n0 * t / threads, b = n0 * (t + 1) / threads;
    cur.rows = b - a;
    if (w0) cur.vals.assign(rel[0].vals.begin() + a * w0, rel[0].vals.begin() + b * w0);
    for (int j = 1; j < ntp && !over.load(); ++j) {
      const Relation& r = rel[j];
      const size_t wa = cur.vars.size(), wb = r.vars.size();
      Relation nx;
      nx.vars = cur.vars;
      for (int c : b_new[j]) nx.vars.push_back(r.vars[c]);
      int64_t counted = 0;  // rows of this step already added to step_rows[j]
      for (int64_t i = 0; i < cur.rows && !over.load(); ++i) {
        auto emit = [&](int64_t k) {
          for (size_t c = 0; c < wa; ++c) nx.vals.push_back(cur.vals[i * wa + c]);
          for (int c : b_new[j]) nx.vals.push_back(r.vals[k * wb + c]);
          ++nx.rows;
        };
        if (b_shared[j].empty()) {
          for (int64_t k = 0; k < r.rows; ++k) emit(k);
        } else {
          const uint64_t key = pack_key(&cur.vals[i * wa], a_shared[j]);
          const auto& kv = keyed[j];
          auto it = std::lower_bound(kv.begin(), kv.end(), std::make_pair(key, (int64_t)INT64_MIN));
          for (; it != kv.end() && it->first == key; ++it) emit(it->second);
        }
        if (cap_rows >= 0 && nx.rows - counted >= 65536) {  // the threads' running total
          if ((step_rows[j] += nx.rows - counted) > cap_rows) over.store(true);
          counted = nx.rows;
        }
      }
      if (cap_rows >= 0 && (step_rows[j] += nx.rows - counted) > cap_rows) over.store(true);
      cur = std::move(nx);
    }
    total += cur.rows;
    out[t] = std::move(cur);
  }
  const int64_t rows = total.load();
  if (over.load() || (cap_rows >= 0 && rows > cap_rows)) return nullptr;
  Result* res = new Result;
  res->nvars = nvars;
  res->rows = rows;
  std::vector<int> col_of(nvars);
  for (int c = 0; c < nvars; ++c) col_of[vars[c]] = c;
  std::vector<int32_t> perm((size_t)rows * nvars);
  int64_t at = 0;
  for (const Relation& r : out) {
    for (int64_t i = 0; i < r.rows; ++i, ++at)
      for (int x = 0; x < nvars; ++x) perm[at * nvars + x] = r.vals[i * nvars + col_of[x]];
  }
  std::vector<int64_t> idx(rows);
  for (int64_t i = 0; i < rows; ++i) idx[i] = i;
  __gnu_parallel::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(&perm[a * nvars], &perm[a * nvars] + nvars,
                                        &perm[b * nvars], &perm[b * nvars] + nvars);
  });
  res->vals.resize((size_t)rows * nvars);
#pragma omp parallel for num_threads(threads)
  for (int64_t i = 0; i < rows; ++i)
    for (int x = 0; x < nvars; ++x) res->vals[i * nvars + x] = perm[idx[i] * nvars + x];
  return res;
}

static void* join_impl(const std::vector<Triple>& D, const int32_t* tps, int32_t ntp,
                       int32_t nvars, int64_t cap_rows) {
  std::vector<int> order = join_order(tps, ntp, nvars);
  Relation cur;  // the unit relation: one row, no columns
  cur.rows = 1;
  for (int t : order) {
    Relation r = tp_relation(D, tps[3 * t], tps[3 * t + 1], tps[3 * t + 2]);
    cur = join(cur, r, cap_rows);
    if (cap_rows >= 0 && cur.rows > cap_rows) return nullptr;
  }
  // variables that appear in no TP cannot be bound: the BGP defines them only
  // through its patterns, so such inputs are rejected
  if ((int32_t)cur.vars.size() != nvars) return nullptr;
  Result* res = new Result;
  res->nvars = nvars;
  res->rows = cur.rows;
  std::vector<int> col_of(nvars);
  for (int c = 0; c < nvars; ++c) col_of[cur.vars[c]] = c;
  std::vector<int32_t> perm((size_t)cur.rows * nvars);
  for (int64_t i = 0; i < cur.rows; ++i)
    for (int x = 0; x < nvars; ++x) perm[i * nvars + x] = cur.vals[i * nvars + col_of[x]];
  std::vector<int64_t> idx(cur.rows);
  for (int64_t i = 0; i < cur.rows; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return std::lexicographical_compare(&perm[a * nvars], &perm[a * nvars] + nvars,
                                        &perm[b * nvars], &perm[b * nvars] + nvars);
  });
  res->vals.resize((size_t)cur.rows * nvars);
  for (int64_t i = 0; i < cur.rows; ++i)
    for (int x = 0; x < nvars; ++x) res->vals[i * nvars + x] = perm[idx[i] * nvars + x];
  return res;
}

int64_t oracle_result_rows(void* h) { return static_cast<Result*>(h)->rows; }
int32_t oracle_result_nvars(void* h) { return static_cast<Result*>(h)->nvars; }

void oracle_result_copy(void* h, int32_t* out) {
  Result* r = static_cast<Result*>(h);
  if (!r->vals.empty()) std::memcpy(out, r->vals.data(), r->vals.size() * sizeof(int32_t));
}

// Order-independent fingerprint of a row multiset: (rows, sum of h1, sum of
// h2) modulo 2^64, with h_k a chain of the SplitMix64 finaliser over the
// row's values in variable order started from seed k.  Rows are row-major
// [n][nvars].
static uint64_t row_h1(const int32_t* row, int32_t nvars) {
  uint64_t x = 0x1234567ULL;
  for (int c = 0; c < nvars; ++c) x = mix64(x ^ (uint32_t)row[c]);
  return x;
}

void oracle_fingerprint_rows(const int32_t* rows, int64_t n, int32_t nvars, uint64_t* out3) {
  uint64_t a = 0, b = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t y = 0x89abcdefULL;
    for (int c = 0; c < nvars; ++c) y = mix64(y ^ (uint32_t)rows[i * nvars + c]);
    a += row_h1(rows + i * nvars, nvars);
    b += y;
  }
  out3[0] = (uint64_t)n;
  out3[1] = a;
  out3[2] = b;
}

void oracle_result_fingerprint(void* h, uint64_t* out3) {
  Result* r = static_cast<Result*>(h);
  oracle_fingerprint_rows(r->vals.data(), r->rows, r->nvars, out3);
}

// The SplitMix64 finaliser itself (pinned by the tests to the generator's
// published output sequence).
uint64_t oracle_mix64(uint64_t z) { return mix64(z); }

// Hash partition of the sorted rows: those with h1(row) mod `mod` ==
// `residue`, in sorted order, copied to out (may be null to count).
// Returns their number.
int64_t oracle_result_partition(void* h, int32_t mod, int32_t residue, int32_t* out) {
  Result* r = static_cast<Result*>(h);
  int64_t k = 0;
  for (int64_t i = 0; i < r->rows; ++i) {
    const int32_t* row = r->vals.data() + i * r->nvars;
    if ((int64_t)(row_h1(row, r->nvars) % (uint64_t)mod) != residue) continue;
    if (out) std::memcpy(out + k * r->nvars, row, sizeof(int32_t) * r->nvars);
    ++k;
  }
  return k;
}

void oracle_result_free(void* h) { delete static_cast<Result*>(h); }

}  // extern "C"
