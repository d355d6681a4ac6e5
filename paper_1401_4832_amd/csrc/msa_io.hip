// msa_io.hip -- alignment ingestion (sec. 4): FASTA or Stockholm text to the
// symbol codes the other entry points take.  Host code only.
//
// PFAM alignments mark insert residues (not aligned to the model) in
// lowercase, and the matching positions of the other sequences with ".";
// both are removed before DCA.  Codes: the 20 standard residues
// A C D E F G H I K L M N P Q R S T V W Y are 0..19, "-" is 20 (q = 21); the
// non-standard uppercase letters B J O U X Z count as gaps; "*" is skipped;
// any other character is an error, and so are sequences of different
// aligned lengths.
#include <string.h>

#include <string>
#include <unordered_map>
#include <vector>

#include "plm.h"

namespace {

constexpr uint8_t kGap = 20;

// code of an aligned character: 0..20, 254 = skip (insert or terminator), 255 = invalid
uint8_t code_of(char ch) {
  static const char* kAlphabet = "ACDEFGHIKLMNPQRSTVWY";
  if ((ch >= 'a' && ch <= 'z') || ch == '.' || ch == '*') return 254;
  if (ch == '-') return kGap;
  if (ch >= 'A' && ch <= 'Z') {
    const char* p = strchr(kAlphabet, ch);
    return p ? (uint8_t)(p - kAlphabet) : kGap;  // B J O U X Z
  }
  return 255;
}

struct Parsed {
  std::vector<std::string> seqs;
  std::string err;
};

bool is_space(char c) { return c == ' ' || c == '\t' || c == '\r' || c == '\n' || c == '\v' || c == '\f'; }

std::vector<std::string> split_lines(const char* t, size_t n) {
  std::vector<std::string> out;
  size_t a = 0;
  for (size_t i = 0; i <= n; ++i)
    if (i == n || t[i] == '\n') {
      out.emplace_back(t + a, i - a);
      a = i + 1;
    }
  return out;
}

std::string strip(const std::string& s) {
  size_t a = 0, b = s.size();
  while (a < b && is_space(s[a])) ++a;
  while (b > a && is_space(s[b - 1])) --b;
  return s.substr(a, b - a);
}

std::string no_space(const std::string& s) {
  std::string o;
  for (char c : s)
    if (!is_space(c)) o.push_back(c);
  return o;
}

bool parse_fasta(const std::vector<std::string>& lines, Parsed& P) {
  bool have = false;
  for (const std::string& l : lines) {
    if (!l.empty() && l[0] == '>') {
      P.seqs.emplace_back();
      have = true;
    } else if (!strip(l).empty()) {
      if (!have) {
        P.err = "sequence text before the first header";
        return false;
      }
      P.seqs.back() += no_space(l);
    }
  }
  return true;
}

bool parse_stockholm(const std::vector<std::string>& lines, Parsed& P) {
  std::unordered_map<std::string, size_t> index;
  for (const std::string& l : lines) {
    const std::string t = strip(l);
    if (t.empty() || t[0] == '#') continue;
    if (t == "//") break;
    size_t k = 0;
    while (k < t.size() && !is_space(t[k])) ++k;
    const std::string name = t.substr(0, k), rest = no_space(t.substr(k));
    auto it = index.find(name);
    if (it == index.end()) {
      index.emplace(name, P.seqs.size());
      P.seqs.push_back(rest);
    } else {
      P.seqs[it->second] += rest;
    }
  }
  return true;
}

void set_msg(char* err, size_t err_len, const std::string& m) {
  if (err && err_len) {
    strncpy(err, m.c_str(), err_len - 1);
    err[err_len - 1] = 0;
  }
}

}  // namespace

extern "C" int plm_parse_alignment(const char* text, size_t len, int32_t format, uint8_t* codes_out,
                                   size_t capacity, int32_t* B_out, int32_t* N_out, char* err,
                                   size_t err_len) {
  if (!text || !B_out || !N_out) {
    set_msg(err, err_len, "null pointer");
    return PLM_E_INVALID;
  }
  const std::vector<std::string> lines = split_lines(text, len);
  int32_t fmt = format;
  if (fmt == PLM_FORMAT_AUTO) {
    fmt = -1;
    for (const std::string& l : lines) {
      if (strip(l).empty()) continue;
      if (l.compare(0, 11, "# STOCKHOLM") == 0) fmt = PLM_FORMAT_STOCKHOLM;
      else if (strip(l)[0] == '>') fmt = PLM_FORMAT_FASTA;
      break;
    }
    if (fmt < 0) {
      set_msg(err, err_len, "unknown alignment format");
      return PLM_E_INVALID;
    }
  }
  Parsed P;
  bool ok = fmt == PLM_FORMAT_FASTA ? parse_fasta(lines, P)
            : fmt == PLM_FORMAT_STOCKHOLM ? parse_stockholm(lines, P)
                                          : (P.err = "unknown format code", false);
  if (!ok) {
    set_msg(err, err_len, P.err);
    return PLM_E_INVALID;
  }
  if (P.seqs.empty()) {
    set_msg(err, err_len, "no sequences");
    return PLM_E_INVALID;
  }
  std::vector<std::vector<uint8_t>> rows(P.seqs.size());
  for (size_t b = 0; b < P.seqs.size(); ++b) {
    for (char ch : P.seqs[b]) {
      const uint8_t c = code_of(ch);
      if (c == 255) {
        set_msg(err, err_len, std::string("unexpected character '") + ch + "' in sequence " + std::to_string(b));
        return PLM_E_INVALID;
      }
      if (c != 254) rows[b].push_back(c);
    }
  }
  const size_t N = rows[0].size();
  for (size_t b = 0; b < rows.size(); ++b)
    if (rows[b].size() != N || N == 0) {
      set_msg(err, err_len, "sequence " + std::to_string(b) + " has aligned length " +
                                std::to_string(rows[b].size()) + ", the first has " + std::to_string(N));
      return PLM_E_INVALID;
    }
  if (N > 0x7fffffff || rows.size() > 0x7fffffff) {
    set_msg(err, err_len, "alignment too large");
    return PLM_E_INVALID;
  }
  *B_out = (int32_t)rows.size();
  *N_out = (int32_t)N;
  if (!codes_out) return PLM_OK;  // size query
  if (capacity < rows.size() * N) {
    set_msg(err, err_len, "codes buffer too small");
    return PLM_E_WORKSPACE;
  }
  for (size_t b = 0; b < rows.size(); ++b) memcpy(codes_out + b * N, rows[b].data(), N);
  return PLM_OK;
}
