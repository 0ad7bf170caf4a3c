// The process-wide table of tuned launch shapes (see tuning.hpp).
#include "tuning.hpp"

#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

#ifndef NDMG_SOURCE_KEY
#define NDMG_SOURCE_KEY "unkeyed"
#endif

namespace ndmg {

namespace {

using Key = std::tuple<int, int, int, int, int>;   // kind, n, elem, mode, pair class

std::mutex g_mu;
std::map<Key, std::pair<int, int>> g_table;
thread_local int g_force_variant = -1, g_force_kz = -1;

bool parse_entry(const std::string& line, Key* k, std::pair<int, int>* v, std::string* err) {
  std::istringstream is(line);
  std::string kind, prec;
  int n = 0, mode = 0, cls = 0, p0 = 0, p1 = 0;
  if (!(is >> kind >> n >> prec >> mode >> cls >> p0 >> p1)) {
    *err = "malformed tuning line: " + line;
    return false;
  }
  int kd = -1;
  if (kind == "stencil") kd = kTuneStencil;
  else if (kind == "patch") kd = kTunePatch;
  else if (kind == "patchaddr") kd = kTunePatchAddr;
  const int elem = prec == "fp64" ? 8 : (prec == "fp32" ? 4 : 0);
  if (kd < 0 || elem == 0 || n < 2 || cls < 0 || cls > 4 || p0 < 0 || p1 < 1 ||
      (kd == kTunePatchAddr && p0 != 32 && p0 != 64)) {
    *err = "bad tuning entry: " + line;
    return false;
  }
  *k = Key(kd, n, elem, mode, cls);
  *v = {p0, p1};
  return true;
}

}  // namespace

int tune_count_class(int count) {
  if (count <= 1) return 0;
  if (count <= 3) return 1;
  if (count <= 15) return 2;
  if (count <= 63) return 3;
  return 4;
}

bool tune_lookup(int kind, int n, int elem, int mode, int count, int* p0, int* p1) {
  std::lock_guard<std::mutex> lock(g_mu);
  const auto it = g_table.find(Key(kind, n, elem, mode, tune_count_class(count)));
  if (it == g_table.end()) return false;
  *p0 = it->second.first;
  *p1 = it->second.second;
  return true;
}

void tune_force_stencil(int variant, int kz) {
  g_force_variant = variant;
  g_force_kz = kz;
}

bool tune_forced_stencil(int* variant, int* kz) {
  if (g_force_variant < 0) return false;
  *variant = g_force_variant;
  *kz = g_force_kz;
  return true;
}

const char* source_key() { return NDMG_SOURCE_KEY; }

bool tune_set_line(const std::string& line, std::string* err) {
  Key k;
  std::pair<int, int> v;
  if (!parse_entry(line, &k, &v, err)) return false;
  std::lock_guard<std::mutex> lock(g_mu);
  g_table[k] = v;
  return true;
}

void tune_clear() {
  std::lock_guard<std::mutex> lock(g_mu);
  g_table.clear();
}

bool tune_load(const std::string& path, std::string* err) {
  std::ifstream f(path);
  if (!f) {
    *err = "cannot read " + path;
    return false;
  }
  std::map<Key, std::pair<int, int>> table;
  std::string line;
  bool keyed = false;
  while (std::getline(f, line)) {
    const size_t c = line.find('#');
    if (c != std::string::npos) line.resize(c);
    std::istringstream is(line);
    std::string first;
    if (!(is >> first)) continue;
    if (first == "key") {
      std::string key;
      is >> key;
      if (key != source_key()) {
        *err = "tuning table " + path + " was measured on other kernel sources (key " + key + ", library " +
               source_key() + ")";
        return false;
      }
      keyed = true;
      continue;
    }
    if (!keyed) {
      *err = "tuning table " + path + " has no key line before its entries";
      return false;
    }
    Key k;
    std::pair<int, int> v;
    if (!parse_entry(line, &k, &v, err)) return false;
    table[k] = v;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  g_table = std::move(table);
  return true;
}

}  // namespace ndmg
