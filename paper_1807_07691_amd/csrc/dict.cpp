// Dictionary encoding of text triples and a minimal BGP parser (paper
// Sec. 5.2: the bijections h_p over predicates and h_so over subjects and
// objects, assigned by order of occurrence; Sec. 6.3: results are decoded
// back to the original strings; Sec. 3.2 / Sec. 4: a query is parsed into
// its triple patterns).
//
// Codes are 0-based here (the paper numbers from 1): the first term seen gets
// 0.  Subjects and objects share one code space, predicates have their own.
//
// Accepted term syntax (N-Triples-like, one triple per statement, statements
// ended by '.' or a line break): <iri>, "literal" with optional @lang or
// ^^<datatype> (backslash escapes kept verbatim), _:blank, and any other
// token without white space (e.g. :likes or A).  A term's code is keyed on
// its exact text.  '#' starts a comment outside IRIs and literals.
#include <cctype>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"

using namespace gsmat;

struct gsmat_dict {
  std::unordered_map<std::string, int32_t> so_code, p_code;
  std::vector<std::string> so_term, p_term;
  std::vector<int32_t> s, p, o;  // codes of the last loaded text, in order
};

namespace {

struct Lexer {
  const char* a;
  size_t n, i = 0;
  int line = 1;

  Lexer(const char* t, size_t len) : a(t), n(len) {}

  [[noreturn]] void fail(const std::string& what) const {
    throw StatusFail{GSMAT_EINVAL, "line " + std::to_string(line) + ": " + what};
  }

  // Skips blanks and comments; stops at a line break when `stop_nl`.
  void skip(bool stop_nl) {
    while (i < n) {
      const char c = a[i];
      if (c == '\n') {
        if (stop_nl) return;
        ++line;
        ++i;
      } else if (c == ' ' || c == '\t' || c == '\r') {
        ++i;
      } else if (c == '#') {
        while (i < n && a[i] != '\n') ++i;
      } else {
        return;
      }
    }
  }

  bool at_end() const { return i >= n; }
  char peek() const { return i < n ? a[i] : '\0'; }

  // One term (or a single-character punctuation token: . { } ).
  std::string token() {
    const size_t b = i;
    const char c = a[i];
    if (c == '.' || c == '{' || c == '}') {
      ++i;
      return std::string(1, c);
    }
    if (c == '<') {
      while (i < n && a[i] != '>' && a[i] != '\n') ++i;
      if (i >= n || a[i] != '>') fail("unterminated IRI");
      ++i;
      return std::string(a + b, i - b);
    }
    if (c == '"') {
      ++i;
      while (i < n && a[i] != '"') {
        if (a[i] == '\n') fail("line break inside a literal");
        if (a[i] == '\\') ++i;
        ++i;
      }
      if (i >= n) fail("unterminated literal");
      ++i;  // closing quote
      if (i < n && a[i] == '@') {
        while (i < n && !is_space(a[i]) && a[i] != '.') ++i;
      } else if (i + 1 < n && a[i] == '^' && a[i + 1] == '^') {
        i += 2;
        if (i >= n || a[i] != '<') fail("datatype must be an IRI");
        while (i < n && a[i] != '>') ++i;
        if (i >= n) fail("unterminated datatype IRI");
        ++i;
      }
      return std::string(a + b, i - b);
    }
    while (i < n && !is_space(a[i]) && a[i] != '{' && a[i] != '}' && a[i] != '#') {
      // a '.' ends a bare token when followed by white space or the end
      if (a[i] == '.' && (i + 1 >= n || is_space(a[i + 1]))) break;
      ++i;
    }
    return std::string(a + b, i - b);
  }

  static bool is_space(char c) { return c == ' ' || c == '\t' || c == '\r' || c == '\n'; }
};

int32_t intern(std::unordered_map<std::string, int32_t>& code, std::vector<std::string>& term,
               const std::string& t) {
  auto it = code.find(t);
  if (it != code.end()) return it->second;
  if (term.size() >= (size_t)INT32_MAX) throw StatusFail{GSMAT_EUNSUPPORTED, "too many terms"};
  const int32_t c = (int32_t)term.size();
  code.emplace(t, c);
  term.push_back(t);
  return c;
}

bool is_var_token(const std::string& t) { return t.size() > 1 && (t[0] == '?' || t[0] == '$'); }

bool keyword(const std::string& t, const char* k) {
  if (t.size() != std::strlen(k)) return false;
  for (size_t j = 0; j < t.size(); ++j)
    if (std::toupper((unsigned char)t[j]) != k[j]) return false;
  return true;
}

}  // namespace

extern "C" gsmat_status gsmat_dict_new(gsmat_dict** out) {
  return guarded([&]() -> gsmat_status {
    if (!out) throw StatusFail{GSMAT_EINVAL, "out is NULL"};
    *out = new gsmat_dict;
    return GSMAT_OK;
  });
}

extern "C" void gsmat_dict_free(gsmat_dict* d) { delete d; }

extern "C" gsmat_status gsmat_dict_load_text(gsmat_dict* d, const char* text, size_t len,
                                             int64_t* n_triples) {
  return guarded([&]() -> gsmat_status {
    if (!d) throw StatusFail{GSMAT_EINVAL, "dictionary is NULL"};
    if (!text && len) throw StatusFail{GSMAT_EINVAL, "text is NULL"};
    d->s.clear();
    d->p.clear();
    d->o.clear();
    // parse fully before encoding, so a syntax error leaves the codes unchanged
    std::vector<std::string> toks;
    Lexer lx(text ? text : "", len);
    for (;;) {
      lx.skip(false);
      if (lx.at_end()) break;
      std::string t[3];
      for (int k = 0; k < 3; ++k) {
        lx.skip(true);
        if (lx.at_end() || lx.peek() == '\n') lx.fail("a triple needs three terms");
        t[k] = lx.token();
        if (t[k] == "." || t[k] == "{" || t[k] == "}") lx.fail("unexpected '" + t[k] + "'");
        if (is_var_token(t[k])) lx.fail("a variable in data: " + t[k]);
      }
      lx.skip(true);
      if (!lx.at_end() && lx.peek() == '.') lx.token();
      lx.skip(true);
      if (!lx.at_end() && lx.peek() != '\n') lx.fail("more than three terms in a triple");
      for (auto& x : t) toks.push_back(std::move(x));
    }
    for (size_t j = 0; j < toks.size(); j += 3) {
      // order of occurrence: subject, predicate, object of each triple in turn
      d->s.push_back(intern(d->so_code, d->so_term, toks[j]));
      d->p.push_back(intern(d->p_code, d->p_term, toks[j + 1]));
      d->o.push_back(intern(d->so_code, d->so_term, toks[j + 2]));
    }
    if (n_triples) *n_triples = (int64_t)d->s.size();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_dict_triples(const gsmat_dict* d, int32_t* s, int32_t* p,
                                           int32_t* o) {
  return guarded([&]() -> gsmat_status {
    if (!d) throw StatusFail{GSMAT_EINVAL, "dictionary is NULL"};
    const size_t n = d->s.size();
    if (n && (!s || !p || !o)) throw StatusFail{GSMAT_EINVAL, "output array is NULL"};
    if (n) {
      std::memcpy(s, d->s.data(), sizeof(int32_t) * n);
      std::memcpy(p, d->p.data(), sizeof(int32_t) * n);
      std::memcpy(o, d->o.data(), sizeof(int32_t) * n);
    }
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_dict_sizes(const gsmat_dict* d, int32_t* n_terms,
                                         int32_t* n_predicates) {
  return guarded([&]() -> gsmat_status {
    if (!d) throw StatusFail{GSMAT_EINVAL, "dictionary is NULL"};
    if (n_terms) *n_terms = (int32_t)d->so_term.size();
    if (n_predicates) *n_predicates = (int32_t)d->p_term.size();
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_dict_lookup(const gsmat_dict* d, const char* term, size_t len,
                                          int32_t is_predicate, int32_t* code) {
  return guarded([&]() -> gsmat_status {
    if (!d || !code || (!term && len)) throw StatusFail{GSMAT_EINVAL, "NULL argument"};
    const auto& m = is_predicate ? d->p_code : d->so_code;
    auto it = m.find(std::string(term ? term : "", len));
    *code = it == m.end() ? -1 : it->second;
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_dict_term(const gsmat_dict* d, int32_t code, int32_t is_predicate,
                                        char* buf, size_t cap, size_t* len) {
  return guarded([&]() -> gsmat_status {
    if (!d) throw StatusFail{GSMAT_EINVAL, "dictionary is NULL"};
    const auto& v = is_predicate ? d->p_term : d->so_term;
    if (code < 0 || (size_t)code >= v.size())
      throw StatusFail{GSMAT_EINVAL, "code " + std::to_string(code) + " is not in the dictionary"};
    const std::string& t = v[code];
    if (len) *len = t.size();
    if (buf && cap) {
      const size_t c = std::min(cap - 1, t.size());
      std::memcpy(buf, t.data(), c);
      buf[c] = '\0';
      if (c < t.size()) throw StatusFail{GSMAT_ETOOBIG, "buffer too small"};
    }
    return GSMAT_OK;
  });
}

extern "C" gsmat_status gsmat_parse_bgp(const gsmat_dict* d, const char* text, size_t len,
                                        gsmat_pattern* pats, int32_t cap, int32_t* n_pats,
                                        int32_t* n_vars, char* var_names, size_t names_cap) {
  return guarded([&]() -> gsmat_status {
    if (!d || !n_pats || (!text && len)) throw StatusFail{GSMAT_EINVAL, "NULL argument"};
    Lexer lx(text ? text : "", len);
    std::vector<std::string> toks;
    for (;;) {
      lx.skip(false);
      if (lx.at_end()) break;
      toks.push_back(lx.token());
    }
    // optional SELECT <vars or *> WHERE { ... }: the patterns between the
    // braces (every variable is returned; the projection list is not used)
    size_t b = 0, e = toks.size();
    if (!toks.empty() && keyword(toks[0], "SELECT")) {
      size_t open = 0;
      while (open < toks.size() && toks[open] != "{") ++open;
      size_t close = toks.size();
      while (close > open + 1 && toks[close - 1] != "}") --close;
      if (open == toks.size() || close <= open + 1 || toks[close - 1] != "}")
        throw StatusFail{GSMAT_EINVAL, "SELECT needs a WHERE { ... } block"};
      b = open + 1;
      e = close - 1;
    }
    std::unordered_map<std::string, int32_t> var;
    std::vector<std::string> names;
    std::vector<gsmat_pattern> out;
    auto term = [&](const std::string& t, bool pred) -> int32_t {
      if (is_var_token(t)) {
        if (pred) throw StatusFail{GSMAT_EUNSUPPORTED, "variable predicate " + t};
        const std::string nm = t.substr(1);
        auto it = var.find(nm);
        if (it != var.end()) return -(it->second + 1);
        const int32_t v = (int32_t)names.size();
        var.emplace(nm, v);
        names.push_back(nm);
        return -(v + 1);
      }
      // a constant the data never had matches nothing: one past the last code
      const auto& m = pred ? d->p_code : d->so_code;
      auto it = m.find(t);
      if (it != m.end()) return it->second;
      return (int32_t)(pred ? d->p_term.size() : d->so_term.size());
    };
    size_t j = b;
    while (j < e) {
      if (toks[j] == ".") {
        ++j;
        continue;
      }
      if (j + 3 > e) throw StatusFail{GSMAT_EINVAL, "a triple pattern needs three terms"};
      for (int k = 0; k < 3; ++k)
        if (toks[j + k] == "." || toks[j + k] == "{" || toks[j + k] == "}")
          throw StatusFail{GSMAT_EINVAL, "a triple pattern needs three terms"};
      gsmat_pattern q;
      q.s = term(toks[j], false);
      q.p = term(toks[j + 1], true);
      q.o = term(toks[j + 2], false);
      out.push_back(q);
      j += 3;
    }
    *n_pats = (int32_t)out.size();
    if (n_vars) *n_vars = (int32_t)names.size();
    if ((int32_t)out.size() > cap) throw StatusFail{GSMAT_ETOOBIG, "more patterns than cap"};
    if (!out.empty() && !pats) throw StatusFail{GSMAT_EINVAL, "pats is NULL"};
    std::copy(out.begin(), out.end(), pats);
    if (var_names && names_cap) {
      size_t at = 0;
      for (const std::string& nm : names) {
        if (at + nm.size() + 1 > names_cap) throw StatusFail{GSMAT_ETOOBIG, "names buffer too small"};
        std::memcpy(var_names + at, nm.data(), nm.size());
        at += nm.size();
        var_names[at++] = '\0';
      }
    }
    return GSMAT_OK;
  });
}
