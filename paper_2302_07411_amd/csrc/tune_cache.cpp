// Autotuner cache: the launch shape each autotuner chose, per shape class,
// kept in a JSON file named by the environment variable CV_TUNE_CACHE (no
// variable: no caching).  The file is one object whose members map a shape
// class (a string the autotuner builds from the geometries it tuned for) to
// an object of integer fields, e.g.
//   {"batch|...": {"threads": 1024, "group_wgs": 8, "max_groups": 0}}
// It is read at each lookup and rewritten whole (through a temporary file
// and a rename) at each store, so several processes may share it; a file
// that does not parse is treated as empty and replaced by the next store.
#include <stdio.h>
#include <stdlib.h>

#include <cctype>
#include <map>
#include <mutex>
#include <string>

#include "runtime.h"

namespace cv {
namespace rt {
namespace {

using Entry = std::map<std::string, int64_t>;
using Table = std::map<std::string, Entry>;

std::mutex g_mu;

const char* cache_path() {
  const char* p = getenv("CV_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

// A small parser for the file's subset of JSON: an object of objects of
// integers; string members have no escapes.
struct Parser {
  const std::string& s;
  size_t i = 0;
  void ws() {
    while (i < s.size() && isspace((unsigned char)s[i])) i++;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      i++;
      return true;
    }
    return false;
  }
  bool str(std::string* out) {
    ws();
    if (i >= s.size() || s[i] != '"') return false;
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) return false;
    *out = s.substr(i + 1, j - i - 1);
    if (out->find('\\') != std::string::npos) return false;
    i = j + 1;
    return true;
  }
  bool num(int64_t* out) {
    ws();
    size_t j = i;
    if (j < s.size() && s[j] == '-') j++;
    const size_t d = j;
    while (j < s.size() && isdigit((unsigned char)s[j])) j++;
    if (j == d) return false;
    *out = strtoll(s.substr(i, j - i).c_str(), nullptr, 10);
    i = j;
    return true;
  }
  template <typename F>
  bool object(F member) {
    if (!eat('{')) return false;
    if (eat('}')) return true;
    do {
      std::string k;
      if (!str(&k) || !eat(':') || !member(k)) return false;
    } while (eat(','));
    return eat('}');
  }
};

Table read_table(const char* path) {
  Table t;
  FILE* f = fopen(path, "rb");
  if (!f) return t;
  std::string s;
  char buf[4096];
  size_t n;
  while ((n = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, n);
  fclose(f);
  Parser p{s};
  Table parsed;
  const bool ok = p.object([&](const std::string& key) {
    Entry e;
    const bool inner = p.object([&](const std::string& field) {
      int64_t v;
      if (!p.num(&v)) return false;
      e[field] = v;
      return true;
    });
    if (inner) parsed[key] = e;
    return inner;
  });
  p.ws();
  return ok && p.i == s.size() ? parsed : t;
}

bool write_table(const char* path, const Table& t) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "wb");
  if (!f) return false;
  fputs("{\n", f);
  size_t k = 0;
  for (const auto& kv : t) {
    fprintf(f, "  \"%s\": {", kv.first.c_str());
    size_t m = 0;
    for (const auto& fv : kv.second)
      fprintf(f, "%s\"%s\": %lld", m++ ? ", " : "", fv.first.c_str(), (long long)fv.second);
    fprintf(f, "}%s\n", ++k < t.size() ? "," : "");
  }
  fputs("}\n", f);
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

bool tune_lookup(const std::string& key, std::map<std::string, int64_t>* fields) {
  const char* path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lock(g_mu);
  const Table t = read_table(path);
  const auto it = t.find(key);
  if (it == t.end()) return false;
  *fields = it->second;
  return true;
}

bool tune_store(const std::string& key, const std::map<std::string, int64_t>& fields) {
  const char* path = cache_path();
  if (!path) return false;
  std::lock_guard<std::mutex> lock(g_mu);
  Table t = read_table(path);
  t[key] = fields;
  return write_table(path, t);
}

}  // namespace rt
}  // namespace cv
