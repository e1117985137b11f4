// Reader of the schedule autotuner's cache: a JSON object whose keys name a
// workload (architecture, Nf, Nd, band, delay law, dtypes, Nt rounded up to a
// power of two) and whose values hold the fastest schedule fields found for
// it under "options". Only the subset of JSON the cache uses is needed, but
// any well-formed document parses; entries other than the requested one are
// skipped.
#include "fdmt_tune.h"

#include <cctype>
#include <cerrno>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <sstream>

namespace fdmt {

namespace {

struct Reader {
  const std::string &s;
  size_t i = 0;
  std::string err;

  explicit Reader(const std::string &text) : s(text) {}

  void ws() {
    while (i < s.size() && std::isspace(static_cast<unsigned char>(s[i]))) ++i;
  }
  bool fail(const std::string &m) {
    if (err.empty()) err = m + " at byte " + std::to_string(i);
    return false;
  }
  bool expect(char c) {
    ws();
    if (i >= s.size() || s[i] != c) return fail(std::string("expected '") + c + "'");
    ++i;
    return true;
  }
  bool string(std::string &out) {
    ws();
    if (i >= s.size() || s[i] != '"') return fail("expected a string");
    ++i;
    out.clear();
    while (i < s.size() && s[i] != '"') {
      char c = s[i++];
      if (c == '\\') {
        if (i >= s.size()) return fail("unterminated escape");
        const char e = s[i++];
        switch (e) {
          case '"': case '\\': case '/': out += e; break;
          case 'b': out += '\b'; break;
          case 'f': out += '\f'; break;
          case 'n': out += '\n'; break;
          case 'r': out += '\r'; break;
          case 't': out += '\t'; break;
          case 'u':  // keys and option names are ASCII; keep the escape's code unit if it is
            if (i + 4 > s.size()) return fail("short \\u escape");
            out += static_cast<char>(std::strtol(s.substr(i, 4).c_str(), nullptr, 16) & 0x7f);
            i += 4;
            break;
          default: return fail("unknown escape");
        }
      } else {
        out += c;
      }
    }
    if (i >= s.size()) return fail("unterminated string");
    ++i;
    return true;
  }
  bool number(double &out) {
    ws();
    const char *b = s.c_str() + i;
    char *e = nullptr;
    errno = 0;
    out = std::strtod(b, &e);
    if (e == b || errno == ERANGE) return fail("expected a number");
    i += static_cast<size_t>(e - b);
    return true;
  }
  // Any value, discarded.
  bool skip() {
    ws();
    if (i >= s.size()) return fail("unexpected end");
    const char c = s[i];
    if (c == '{') {
      ++i;
      ws();
      if (i < s.size() && s[i] == '}') return ++i, true;
      for (;;) {
        std::string k;
        if (!string(k) || !expect(':') || !skip()) return false;
        ws();
        if (i < s.size() && s[i] == ',') { ++i; continue; }
        return expect('}');
      }
    }
    if (c == '[') {
      ++i;
      ws();
      if (i < s.size() && s[i] == ']') return ++i, true;
      for (;;) {
        if (!skip()) return false;
        ws();
        if (i < s.size() && s[i] == ',') { ++i; continue; }
        return expect(']');
      }
    }
    if (c == '"') {
      std::string t;
      return string(t);
    }
    for (const char *lit : {"true", "false", "null"}) {
      const size_t n = std::char_traits<char>::length(lit);
      if (s.compare(i, n, lit) == 0) return i += n, true;
    }
    double d;
    return number(d);
  }
  // An object of numbers: {"name": number, ...}.
  bool numbers(std::map<std::string, double> &out) {
    if (!expect('{')) return false;
    ws();
    if (i < s.size() && s[i] == '}') return ++i, true;
    for (;;) {
      std::string k;
      double v;
      if (!string(k) || !expect(':') || !number(v)) return false;
      out[k] = v;
      ws();
      if (i < s.size() && s[i] == ',') { ++i; continue; }
      return expect('}');
    }
  }
  // An entry: an object whose "options" member is read, everything else skipped.
  bool entry(std::map<std::string, double> &out, bool &has) {
    if (!expect('{')) return false;
    ws();
    if (i < s.size() && s[i] == '}') return ++i, true;
    for (;;) {
      std::string k;
      if (!string(k) || !expect(':')) return false;
      if (k == "options") {
        has = true;
        if (!numbers(out)) return false;
      } else if (!skip()) {
        return false;
      }
      ws();
      if (i < s.size() && s[i] == ',') { ++i; continue; }
      return expect('}');
    }
  }
};

std::string fmt_g6(double x) {
  char b[64];
  std::snprintf(b, sizeof b, "%.6g", x);
  return b;
}

const char *dtype_name(int d) {
  switch (d) {
    case 0: return "f32";
    case 1: return "f16";
    case 2: return "u8";
    case 3: return "i32";
    default: return "?";
  }
}

}  // namespace

std::string tune_key(const std::string &arch, int nf, int64_t nt, int nd, double f_min, double f_max,
                     int in_dtype, int acc_dtype, double gamma, int rule) {
  int64_t bucket = 1;
  while (bucket < nt) bucket *= 2;
  std::string k = arch + "/nf" + std::to_string(nf) + "/nd" + std::to_string(nd) + "/band" + fmt_g6(f_min) + "-" +
                  fmt_g6(f_max);
  if (gamma != -2.0) k += "/gamma" + fmt_g6(gamma);
  if (rule == 1) k += "/twoC";
  k += std::string("/") + dtype_name(in_dtype) + "->" + dtype_name(acc_dtype) + "/nt" + std::to_string(bucket);
  return k;
}

std::string tune_lookup(const std::string &path, const std::string &key, std::map<std::string, double> &options,
                        bool &found) {
  found = false;
  options.clear();
  std::ifstream f(path, std::ios::binary);
  if (!f) return "";  // no cache: nothing tuned
  std::ostringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  Reader r(text);
  if (!r.expect('{')) return path + ": " + r.err;
  r.ws();
  if (r.i < text.size() && text[r.i] == '}') return "";
  for (;;) {
    std::string k;
    if (!r.string(k) || !r.expect(':')) return path + ": " + r.err;
    if (k == key) {
      bool has = false;
      std::map<std::string, double> o;
      if (!r.entry(o, has)) return path + ": " + r.err;
      if (has) {
        options = o;
        found = true;
      }
    } else if (!r.skip()) {
      return path + ": " + r.err;
    }
    r.ws();
    if (r.i < text.size() && text[r.i] == ',') {
      ++r.i;
      continue;
    }
    if (!r.expect('}')) return path + ": " + r.err;
    r.ws();
    if (r.i != text.size()) return path + ": trailing characters after the cache object";
    return "";
  }
}

}  // namespace fdmt
