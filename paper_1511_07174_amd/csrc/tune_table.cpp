// Reader of the autotuner's JSON table (host code only, no device work).
//
// The table is the file the autotuner writes: an object whose "entries" array
// holds {"key": "getrf_nb" | "potrf_nb" | "vbatch_tile", "dtype": "f64" | "f32",
// "n_max": <int>, "value": <int>} records.  Other members (the device the table
// was measured on, the raw timings, notes) are skipped.  An optional "arch"
// string names the device; a table measured on another architecture is
// refused.  The parser accepts the JSON grammar (objects, arrays, strings with
// escapes, numbers, true / false / null) and nothing more.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <string>
#include <vector>
#include "tune_table.hpp"

namespace cds {

namespace {

struct Parser {
  const char* p;
  const char* end;
  std::string err;

  void ws() {
    while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
  }
  bool fail(const char* what) {
    if (err.empty()) err = what;
    return false;
  }
  bool lit(const char* s) {
    const size_t k = strlen(s);
    if ((size_t)(end - p) < k || strncmp(p, s, k) != 0) return fail("unexpected token");
    p += k;
    return true;
  }
  bool string(std::string& out) {
    ws();
    if (p >= end || *p != '"') return fail("string expected");
    ++p;
    out.clear();
    while (p < end && *p != '"') {
      if (*p == '\\') {
        ++p;
        if (p >= end) return fail("bad escape");
        const char c = *p++;
        switch (c) {
          case '"': case '\\': case '/': out.push_back(c); break;
          case 'b': out.push_back('\b'); break;
          case 'f': out.push_back('\f'); break;
          case 'n': out.push_back('\n'); break;
          case 'r': out.push_back('\r'); break;
          case 't': out.push_back('\t'); break;
          case 'u':
            if (end - p < 4) return fail("bad escape");
            p += 4;              // the keys and values read here are ASCII; the code point is dropped
            out.push_back('?');
            break;
          default: return fail("bad escape");
        }
      } else {
        out.push_back(*p++);
      }
    }
    if (p >= end) return fail("unterminated string");
    ++p;
    return true;
  }
  bool number(double& v, bool& integral) {
    ws();
    const char* s = p;
    if (p < end && (*p == '-' || *p == '+')) ++p;
    bool digits = false;
    integral = true;
    while (p < end && ((*p >= '0' && *p <= '9') || *p == '.' || *p == 'e' || *p == 'E' || *p == '-' || *p == '+')) {
      if (*p == '.' || *p == 'e' || *p == 'E') integral = false;
      if (*p >= '0' && *p <= '9') digits = true;
      ++p;
    }
    if (!digits) return fail("number expected");
    std::string t(s, p);
    char* q = nullptr;
    v = strtod(t.c_str(), &q);
    if (q == t.c_str() || *q != '\0') return fail("bad number");
    return true;
  }
  // Skip any value.
  bool skip(int depth = 0) {
    if (depth > 64) return fail("nesting too deep");
    ws();
    if (p >= end) return fail("value expected");
    if (*p == '"') { std::string s; return string(s); }
    if (*p == '{') {
      ++p;
      ws();
      if (p < end && *p == '}') { ++p; return true; }
      while (true) {
        std::string k;
        if (!string(k)) return false;
        ws();
        if (p >= end || *p != ':') return fail("':' expected");
        ++p;
        if (!skip(depth + 1)) return false;
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') { ++p; return true; }
        return fail("',' or '}' expected");
      }
    }
    if (*p == '[') {
      ++p;
      ws();
      if (p < end && *p == ']') { ++p; return true; }
      while (true) {
        if (!skip(depth + 1)) return false;
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') { ++p; return true; }
        return fail("',' or ']' expected");
      }
    }
    if (*p == 't') return lit("true");
    if (*p == 'f') return lit("false");
    if (*p == 'n') return lit("null");
    double v;
    bool in;
    return number(v, in);
  }
  // One record of "entries".
  bool entry(TuneRecord& r) {
    ws();
    if (p >= end || *p != '{') return fail("entry object expected");
    ++p;
    bool has_key = false, has_dt = false, has_n = false, has_v = false;
    ws();
    if (p < end && *p == '}') return fail("empty entry");
    while (true) {
      std::string k;
      if (!string(k)) return false;
      ws();
      if (p >= end || *p != ':') return fail("':' expected");
      ++p;
      if (k == "key") {
        std::string v;
        if (!string(v)) return false;
        if (v == "getrf_nb") r.key = 0;
        else if (v == "potrf_nb") r.key = 1;
        else if (v == "vbatch_tile") r.key = 2;
        else return fail("unknown key");
        has_key = true;
      } else if (k == "dtype") {
        std::string v;
        if (!string(v)) return false;
        if (v == "f64") r.dtype = 0;
        else if (v == "f32") r.dtype = 1;
        else return fail("unknown dtype");
        has_dt = true;
      } else if (k == "n_max" || k == "value") {
        double v;
        bool in;
        if (!number(v, in)) return false;
        if (!in || v < -9.2e18 || v > 9.2e18) return fail("integer expected");
        if (k == "n_max") { r.n_max = (int64_t)v; has_n = true; }
        else { r.value = (int64_t)v; has_v = true; }
      } else {
        if (!skip()) return false;
      }
      ws();
      if (p < end && *p == ',') { ++p; continue; }
      if (p < end && *p == '}') { ++p; break; }
      return fail("',' or '}' expected");
    }
    if (!(has_key && has_dt && has_n && has_v)) return fail("entry lacks key, dtype, n_max or value");
    return true;
  }
};

}  // namespace

int read_tune_table(const char* path, std::vector<TuneRecord>& out, std::string& arch, std::string& err) {
  out.clear();
  arch.clear();
  FILE* f = fopen(path, "rb");
  if (!f) {
    err = "cannot open the table";
    return 1;
  }
  std::string text;
  char buf[65536];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) {
    text.append(buf, got);
    if (text.size() > ((size_t)64 << 20)) {
      fclose(f);
      err = "table larger than 64 MiB";
      return 1;
    }
  }
  fclose(f);
  Parser ps{text.data(), text.data() + text.size(), std::string()};
  ps.ws();
  if (ps.p >= ps.end || *ps.p != '{') {
    err = "the table is not a JSON object";
    return 1;
  }
  ++ps.p;
  bool have_entries = false;
  ps.ws();
  if (ps.p < ps.end && *ps.p == '}') {
    ++ps.p;
  } else {
    while (true) {
      std::string k;
      if (!ps.string(k)) break;
      ps.ws();
      if (ps.p >= ps.end || *ps.p != ':') { ps.fail("':' expected"); break; }
      ++ps.p;
      if (k == "entries") {
        ps.ws();
        if (ps.p >= ps.end || *ps.p != '[') { ps.fail("entries must be an array"); break; }
        ++ps.p;
        have_entries = true;
        ps.ws();
        if (ps.p < ps.end && *ps.p == ']') {
          ++ps.p;
        } else {
          bool ok = true;
          while (true) {
            TuneRecord r{};
            if (!ps.entry(r)) { ok = false; break; }
            out.push_back(r);
            ps.ws();
            if (ps.p < ps.end && *ps.p == ',') { ++ps.p; continue; }
            if (ps.p < ps.end && *ps.p == ']') { ++ps.p; break; }
            ps.fail("',' or ']' expected");
            ok = false;
            break;
          }
          if (!ok) break;
        }
      } else if (k == "arch") {
        if (!ps.string(arch)) break;
      } else {
        if (!ps.skip()) break;
      }
      ps.ws();
      if (ps.p < ps.end && *ps.p == ',') { ++ps.p; continue; }
      if (ps.p < ps.end && *ps.p == '}') { ++ps.p; break; }
      ps.fail("',' or '}' expected");
      break;
    }
  }
  if (ps.err.empty()) {
    ps.ws();
    if (ps.p != ps.end) ps.fail("trailing characters after the table");
  }
  if (ps.err.empty() && !have_entries) ps.fail("no entries array");
  if (!ps.err.empty()) {
    err = ps.err;
    out.clear();
    return 1;
  }
  return 0;
}

}  // namespace cds
